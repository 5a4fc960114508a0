"""Full-size checks on the bench workload L4-2k/20k/150k/1M-d200-k8 (n = 1,172,000), in the
launch configuration the benchmark times (panel stream, automatic panel width).

* every row of the block product with H against the oracle's float64 product from the upper
  triangle (both precisions of X, full and partial blocks);
* the mixed solve's eigenpairs against properties that hold at any size: the true residual
  computed on the CPU by the oracle's product, orthonormality, and agreement with the float64
  solve's eigenvalues.
"""
import numpy as np
import pytest
import torch

import levelgen
import oracle

pytestmark = pytest.mark.gpu

P = None
W = levelgen.WORKLOADS[1]
_A = None


def setup_module(module):
    global P
    import paper_2407_08901_amd as _P
    _P.lib()
    P = _P


def _matrix():
    global _A
    if _A is None:
        _A = W.generate()
    return _A


def _ctx(A, **kw):
    rp, col, val = P.upload(A, dtype=torch.float64)
    return P.sppc_setup(rp, col, val, A.level_offsets, W.n_small_levels, W.k, P.sppc_default_opts(**kw))


@pytest.mark.parametrize("b", [8, 5])
def test_block_product_every_row(b):
    A = _matrix()
    print("case fullsize product n=%d b=%d" % (A.n, b), flush=True)
    rng = np.random.default_rng(100 + b)
    X = rng.standard_normal((A.n, b))
    ref = oracle.product_from_upper(A.row_ptr, A.col, A.val, A.n, X)
    scale = oracle.product_from_upper(A.row_ptr, A.col, np.abs(A.val), A.n, np.abs(X))
    ctx = _ctx(A, precision=P.SPPC_PREC_MIXED)
    Yd = torch.empty((A.n, b), dtype=torch.float64, device="cuda")
    P.sppc_spmm(ctx, torch.from_numpy(X).cuda(), Yd)
    torch.cuda.synchronize()
    err = np.abs(Yd.cpu().numpy() - ref) / scale
    assert np.max(err) < 1e-14
    # float32 X: each product rounded to float32 (relative 2^-24), sums in float64
    X32 = X.astype(np.float32)
    ref32 = oracle.product_from_upper(A.row_ptr, A.col, A.val, A.n, X32.astype(np.float64))
    P.sppc_spmm(ctx, torch.from_numpy(X32).cuda(), Yd)
    torch.cuda.synchronize()
    err32 = np.abs(Yd.cpu().numpy() - ref32) / scale
    assert np.max(err32) < 2.0 ** -24 * 1.01
    P.sppc_destroy(ctx)


def test_mixed_solve_true_residual_and_plain_agreement():
    A = _matrix()
    print("case fullsize solve n=%d" % A.n, flush=True)
    res = {}
    for name, prec in (("mixed", P.SPPC_PREC_MIXED), ("plain", P.SPPC_PREC_FP64)):
        ctx = _ctx(A, precision=prec)
        ev, Z, rrn, st, status = P.sppc_solve(ctx)
        P.sppc_destroy(ctx)
        assert status == P.SPPC_OK and st["converged"] == 1
        res[name] = (np.array(ev), Z.cpu().numpy(), np.array(rrn))
    for name, (ev, Z, rrn) in res.items():
        R = oracle.product_from_upper(A.row_ptr, A.col, A.val, A.n, Z) - Z * ev[None, :]
        true = np.linalg.norm(R, axis=0) / np.abs(ev)
        assert np.max(true) < 1e-6, (name, true)
        assert np.max(np.abs(true - rrn)) < 1e-9, (name, true, rrn)
        assert np.max(np.abs(Z.T @ Z - np.eye(W.k))) < 1e-12
        assert np.all(np.diff(ev) >= 0)
    assert np.max(np.abs(res["mixed"][0] - res["plain"][0]) / np.abs(res["plain"][0])) < 1e-10

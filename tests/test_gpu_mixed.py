"""Mixed precision (float32 products accumulated in float64, float64 basis and Rayleigh-Ritz,
float64 residual refinement) against the float64 oracle / dense eigensolver."""
import numpy as np
import pytest
import torch

import levelgen
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2407_08901_amd as P
    P.lib()
    return P


def _solve(P, A, ns, k, **kw):
    rp, col, val = P.upload(A, dtype=torch.float64)
    ctx = P.sppc_setup(rp, col, val, A.level_offsets, ns, k, P.sppc_default_opts(**kw))
    out = P.sppc_solve(ctx)
    P.sppc_destroy(ctx)
    return out


@pytest.mark.parametrize("case", ["cfg0", "mid"])
def test_mixed_solve_matches_float64(P, case):
    if case == "cfg0":
        w = levelgen.WORKLOADS[0]
        A, ns, k = w.generate(), w.n_small_levels, w.k
    else:
        A, ns, k = levelgen.generate((150, 1500, 12000), 60, 31), 1, 8
    print("case mixed %s n=%d k=%d" % (case, A.n, k), flush=True)
    ev, Z, rrn, st, status = _solve(P, A, ns, k, precision=P.SPPC_PREC_MIXED)
    assert status == P.SPPC_OK and st["converged"] == 1
    H = oracle.symmetric_from_upper(A.row_ptr, A.col, A.val, A.n)
    lam = np.linalg.eigvalsh(H.toarray())[:k] if A.n <= 6000 else \
        oracle.sppc(H, int(A.level_offsets[ns]), k, oracle.Options(tol=1e-9)).theta
    rel = np.max(np.abs(np.array(ev) - lam) / np.abs(lam))
    assert rel < 1e-8, rel
    Zh = Z.cpu().numpy()
    R = H @ Zh - Zh * np.array(ev)[None, :]
    assert np.max(np.linalg.norm(R, axis=0) / np.abs(ev)) < 1e-6   # true float64 residual
    assert np.max(np.abs(Zh.T @ Zh - np.eye(k))) < 1e-12


def test_mixed_refinement_reaches_a_tight_tolerance(P):
    """Below the float32 noise floor the float64 refinement has to do the work."""
    w = levelgen.WORKLOADS[0]
    A = w.generate()
    ev, Z, rrn, st, status = _solve(P, A, w.n_small_levels, w.k, precision=P.SPPC_PREC_MIXED, tol=1e-9)
    assert status == P.SPPC_OK and max(rrn) < 1e-9
    assert st["refine_steps"] >= 1
    H = oracle.symmetric_from_upper(A.row_ptr, A.col, A.val, A.n)
    lam = np.linalg.eigvalsh(H.toarray())[: w.k]
    assert np.max(np.abs(np.array(ev) - lam) / np.abs(lam)) < 1e-12

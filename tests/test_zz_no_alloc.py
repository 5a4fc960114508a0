"""The allocation-free block product (sppc_spmm_noalloc) through the C ABI against sppc_spmm.

Both calls run the same kernels; the allocation-free one stages the padded copy of X in the
library's static device scratch instead of the context's buffer.  Their outputs agree to the
floating-point bar of the block-product tests (float64 sums whose order depends on scheduling:
1e-14 relative to |H| |X|), on two calls in a row, the second with a smaller input, and a call
whose padded copy would not fit the scratch is refused.
"""
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


def _ctx(P, A, k, dtype):
    rp, col, val = P.upload(A, dtype=dtype)
    # panel_width forces the column-panel copy of H, whose kernels read X with row stride 4/8/16
    return P.sppc_setup(rp, col, val, A.level_offsets, 1, k, P.sppc_default_opts(panel_width=4096))


def _check_pair(P, A, ctx, b, xdtype, seed):
    rng = np.random.default_rng(seed)
    Xh = rng.standard_normal((A.n, b))
    if xdtype == torch.float32:
        Xh = Xh.astype(np.float32).astype(np.float64)
    X = torch.from_numpy(Xh).to("cuda", dtype=xdtype)
    Y0 = torch.full((A.n, b), np.nan, dtype=torch.float64, device="cuda")
    Y1 = torch.full((A.n, b), np.nan, dtype=torch.float64, device="cuda")
    P.sppc_spmm(ctx, X, Y0)
    P.sppc_spmm_noalloc(ctx, X, Y1)
    torch.cuda.synchronize()
    y0, y1 = Y0.cpu().numpy(), Y1.cpu().numpy()
    scale = oracle.product_from_upper(A.row_ptr, A.col, np.abs(A.val), A.n, np.abs(Xh))
    assert np.all(np.isfinite(y1))
    assert np.max(np.abs(y1 - y0) / np.maximum(scale, 1e-300)) < 1e-14
    # and both against the oracle's float64 product (float32 X: float32 products, error 2^-24)
    ref = oracle.product_from_upper(A.row_ptr, A.col, A.val, A.n, Xh)
    tol = 1e-14 if xdtype == torch.float64 else 2.0 ** -24
    assert np.max(np.abs(y1 - ref) / np.maximum(scale, 1e-300)) < tol


def test_noalloc_matches_spmm_two_calls_second_smaller(P):
    A = levelgen.generate((600, 6000, 54100), 40, 77)       # n = 60,700
    print("case noalloc n=%d b=7 float64 X" % A.n, flush=True)
    ctx = _ctx(P, A, 8, torch.float64)
    _check_pair(P, A, ctx, 7, torch.float64, 1)
    B = levelgen.generate((300, 3000, 20000), 30, 78)       # n = 23,300: a smaller input
    print("case noalloc n=%d b=3 float32 X" % B.n, flush=True)
    ctx2 = _ctx(P, B, 4, torch.float32)
    _check_pair(P, B, ctx2, 3, torch.float32, 2)
    # the first context again after the smaller call (the scratch keeps the last call's contents)
    print("case noalloc n=%d b=5 float64 X again" % A.n, flush=True)
    _check_pair(P, A, ctx, 5, torch.float64, 3)
    P.sppc_destroy(ctx2)
    P.sppc_destroy(ctx)


def test_noalloc_refuses_a_copy_beyond_the_scratch(P):
    A = levelgen.generate((300, 3000, 300000), 20, 79)      # n = 303,300: n x 16 x 8 B > 32 MiB
    print("case noalloc limit n=%d" % A.n, flush=True)
    ctx = _ctx(P, A, 4, torch.float64)
    X = torch.ones((A.n, 13), dtype=torch.float64, device="cuda")
    Y = torch.empty((A.n, 13), dtype=torch.float64, device="cuda")
    with pytest.raises(P.SPPCError) as e:
        P.sppc_spmm_noalloc(ctx, X, Y)
    assert e.value.status == P.SPPC_E_ARG and "scratch" in str(e.value)
    # 16 columns per row, aligned: no copy is needed, so the call runs
    _check_pair(P, A, ctx, 16, torch.float64, 4)
    P.sppc_destroy(ctx)

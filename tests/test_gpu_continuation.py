"""Continuation with the small-space preconditioner against the float64 CPU reference."""
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


def _H(A):
    return oracle.symmetric_from_upper(A.row_ptr, A.col, A.val, A.n)


@pytest.mark.parametrize("mixed,ptol", [(False, 1e-13), (True, 1e-13), (False, 1e-8)])
def test_small_space_correction_matches_reference(P, mixed, ptol):
    # ptol 1e-13: the classical single-reduction CG; 1e-8: its pipelined form (loose tolerances)
    A = levelgen.generate((37, 411, 2999), 44, 19)
    k, ns = 3, 1
    n0 = int(A.level_offsets[ns])
    print("case small correction mixed=%d ptol=%g n=%d" % (mixed, ptol, A.n), flush=True)
    H = _H(A)
    rp, col, val = P.upload(A)
    opts = P.sppc_default_opts(precond_tol=ptol,
                               precision=P.SPPC_PREC_MIXED if mixed else P.SPPC_PREC_FP64)
    ctx = P.sppc_setup(rp, col, val, A.level_offsets, ns, k, opts)
    for _ in range(3):
        P.sppc_correct(ctx, P.SPPC_CORR_PERTURBATIVE)
        theta, rrn, added = P.sppc_rayleigh_ritz(ctx)
    Z = P.sppc_get(ctx, 10, A.n * k, device=True).cpu().numpy().reshape(A.n, k)
    R = P.sppc_get(ctx, 11, A.n * k, device=True).cpu().numpy().reshape(A.n, k)
    act = [i for i in range(k) if not rrn[i] < 1e-6]
    assert act
    P.sppc_correct(ctx, P.SPPC_CORR_SMALL)
    T = P.sppc_get(ctx, 5, A.n * len(act), device=True).cpu().numpy().reshape(A.n, len(act))
    for a, i in enumerate(act):
        ref = oracle.small_space_correction(H, n0, theta[i], R[:, i], Z[:, i])
        err = np.max(np.abs(T[:, a] - ref)) / np.max(np.abs(ref))
        # the small solve to ptol with float64 products in both precisions; the error of the
        # solution is at most the condition of the deflated operator (~1e2 here) times ptol
        assert err < (1e-9 if ptol < 1e-12 else 1e-5), (i, err)
    P.sppc_destroy(ctx)


@pytest.mark.parametrize("case", ["cfg0", "mid"])
def test_small_space_continuation_converges_to_the_eigenpairs(P, case):
    if case == "cfg0":
        w = levelgen.WORKLOADS[0]
        A, ns, k = w.generate(), w.n_small_levels, w.k
    else:
        A, ns, k = levelgen.generate((150, 1500, 12000), 60, 33), 1, 8
    print("case small continuation %s n=%d" % (case, A.n), flush=True)
    lam = np.linalg.eigvalsh(_H(A).toarray())[:k]
    rp, col, val = P.upload(A)
    steps = {}
    for kind in (P.SPPC_CORR_JACOBI, P.SPPC_CORR_SMALL):
        ctx = P.sppc_setup(rp, col, val, A.level_offsets, ns, k, P.sppc_default_opts(precond=kind))
        ev, Z, rrn, st, status = P.sppc_solve(ctx)
        P.sppc_destroy(ctx)
        assert status == P.SPPC_OK
        assert np.max(np.abs(np.array(ev) - lam) / np.abs(lam)) < 1e-10
        assert max(rrn) < 1e-6
        steps[kind] = st["cont_steps"]
    print("continuation steps: diagonal %d, small-space %d" % (steps[P.SPPC_CORR_JACOBI], steps[P.SPPC_CORR_SMALL]))
    assert steps[P.SPPC_CORR_SMALL] <= steps[P.SPPC_CORR_JACOBI]

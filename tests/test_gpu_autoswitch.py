"""The automatic switch (opts.auto_switch) against the oracle's.

SPPC stops at the first step whose new correction vectors lie almost in the basis (sine of the
angle below 1e-4) or after which the largest residual has not halved over three steps; the
continuation takes over from there.  On a ragged three-level matrix the residual rule decides
(step 4); on a four-level matrix the angle rule does (step 8).  The GPU must stop at the
oracle's step and reach the oracle's eigenvalues; each case first checks that no quantity the
rule reads lies near its threshold in the oracle's run, so that rounding cannot move the
decision.
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


def _case(name):
    if name == "cfg0":
        w = levelgen.WORKLOADS[0]
        return w.generate(), w.n_small_levels, w.k
    if name == "ragged":
        return levelgen.generate((37, 411, 2999), 44, 9), 1, 3
    return levelgen.generate((40, 400, 3000, 8000), 60, 5), 2, 4


def _oracle_switch(H, n0, k):
    """The oracle's switch step, with the margins of the quantities that decided it."""
    full = oracle.sppc(H, n0, k, oracle.Options(continuation=False, maxiter=15, final_check=False))
    top = [float(np.max(h["rrn"])) for h in full.history]
    for p in range(1, 16):
        ang = float(np.min(full.history[p]["angles"]))
        assert not (1e-4 / 1.3 < ang < 1e-4 * 1.3), ("angle near the threshold", p, ang)
        if p >= 3:
            ratio = top[p] / top[p - 3]
            assert not (0.5 / 1.2 < ratio < 0.5 * 1.2), ("residual ratio near 1/2", p, ratio)
        if ang < 1e-4 or (p >= 3 and top[p] >= 0.5 * top[p - 3]):
            return p
    return None


@pytest.mark.parametrize("name,precond,precision", [
    ("ragged", "JACOBI", "FP64"),
    ("four_levels", "RMMDIIS", "FP64"),
    ("four_levels", "RMMDIIS", "MIXED"),
])
def test_automatic_switch_matches_the_oracle(P, name, precond, precision):
    A, ns, k = _case(name)
    n0 = int(A.level_offsets[ns])
    print("case auto switch %s %s %s n=%d" % (name, precond, precision, A.n), flush=True)
    H = oracle.symmetric_from_upper(A.row_ptr, A.col, A.val, A.n)
    first = _oracle_switch(H, n0, k)
    assert first is not None and first < 15
    ref = oracle.sppc(H, n0, k, oracle.Options(auto_switch=True, rmm_diis=precond == "RMMDIIS"))
    assert ref.converged and [h for h in ref.history if h["phase"] == "sppc"][-1]["p"] == first
    rp, col, val = P.upload(A, dtype=torch.float64)
    opts = P.sppc_default_opts(auto_switch=1, precond=getattr(P, "SPPC_CORR_" + precond),
                               precision=getattr(P, "SPPC_PREC_" + precision))
    ctx = P.sppc_setup(rp, col, val, A.level_offsets, ns, k, opts)
    ev, Z, rrn, st, status = P.sppc_solve(ctx)
    P.sppc_destroy(ctx)
    assert status == P.SPPC_OK and st["converged"] == 1 and max(rrn) < 1e-6
    assert st["iterations"] == first, (st["iterations"], first)
    tol = 1e-10 if precision == "FP64" else 1e-8
    assert np.max(np.abs(np.array(ev) - ref.theta) / np.abs(ref.theta)) < tol
    Zh = Z.cpu().numpy()
    R = oracle.product_from_upper(A.row_ptr, A.col, A.val, A.n, Zh) - Zh * np.array(ev)[None, :]
    assert np.max(np.linalg.norm(R, axis=0) / np.abs(ev)) < 1e-6


def test_automatic_switch_needs_a_switch_point(P):
    # with p_switch = 0 (pure SPPC up to maxiter) the automatic rule does not apply
    A, ns, k = _case("cfg0")
    print("case auto switch without p_switch", flush=True)
    rp, col, val = P.upload(A, dtype=torch.float64)
    opts = P.sppc_default_opts(auto_switch=1, p_switch=0, maxiter=12, final_check=0)
    ctx = P.sppc_setup(rp, col, val, A.level_offsets, ns, k, opts)
    ev, Z, rrn, st, status = P.sppc_solve(ctx)
    P.sppc_destroy(ctx)
    assert st["iterations"] == 12 and st["cont_steps"] == 0

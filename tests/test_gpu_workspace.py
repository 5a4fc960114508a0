"""The caller-owned workspace through the C ABI: sppc_workspace_size, then sppc_setup on a
PyTorch-allocated block from which every device array of the context is taken.

For several problem shapes and option sets the solve on the workspace equals the solve on
library-allocated memory, the peak the library reports lies within the size it asked for (and not
far below it), the device's free memory does not move while the context lives (all of its device
memory came from the workspace), and a workspace that is too small is refused with SPPC_E_NOMEM.
"""
import numpy as np
import pytest
import torch

import levelgen

pytestmark = pytest.mark.gpu

CASES = [
    ("cfg0 plain", levelgen.WORKLOADS[0], torch.float64, {}),
    ("cfg0 mixed rmmdiis+learned", levelgen.WORKLOADS[0], torch.float64,
     dict(precision=1, precond=4, rmm_precond=2)),
    ("cfg0 davidson learned", levelgen.WORKLOADS[0], torch.float64, dict(precond=2)),
    ("cfg0 pair 2", levelgen.small_workload((100, 800, 4000), 60, 20240712, 1, 1), torch.float64, dict(pair_index=2)),
    ("n117200 panel mixed rmmdiis", levelgen.train_workload(2000, "L4"), torch.float64, dict(precision=1, precond=4)),
    ("n117200 panel plain float32 values", levelgen.train_workload(2001, "L4"), torch.float32, {}),
]


@pytest.fixture(scope="module")
def P():
    import paper_2407_08901_amd as P
    P.lib()
    P.sppc_set_memory_cache(0)
    return P


def _solve(P, ctx, kw):
    if kw.get("precond") == P.SPPC_CORR_MPNN or kw.get("rmm_precond") == P.SPPC_CORR_MPNN:
        from paper_2407_08901_amd import mpnn_train
        P.sppc_mpnn_set_weights(ctx, mpnn_train.load_for("rmmdiis" if kw.get("precond") == 4 else "davidson"))
    return P.sppc_solve(ctx, want_vectors=False)


@pytest.mark.parametrize("name,w,dtype,kw", CASES, ids=[c[0] for c in CASES])
def test_solve_on_a_torch_workspace(P, name, w, dtype, kw):
    A = w.generate()
    print("case workspace %s n=%d" % (name, A.n), flush=True)
    rp, col, val = P.upload(A, dtype=dtype)
    opts = P.sppc_default_opts(**kw)
    need = P.sppc_workspace_size(rp, col, val, A.level_offsets, w.n_small_levels, w.k, opts)
    ref_ctx = P.sppc_setup(rp, col, val, A.level_offsets, w.n_small_levels, w.k, opts)
    ev0, _, rrn0, st0, s0 = _solve(P, ref_ctx, kw)
    P.sppc_destroy(ref_ctx)
    ws = P.workspace_tensor(need)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    ctx = P.sppc_setup(rp, col, val, A.level_offsets, w.n_small_levels, w.k, opts, workspace=ws)
    ev, _, rrn, st, status = _solve(P, ctx, kw)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    P.sppc_destroy(ctx)
    assert status == s0 == P.SPPC_OK
    # two solves that each stop at rrn < 1e-6 (the small-space CG polls its convergence
    # asynchronously, so iteration counts can differ): the bar of the other form comparisons
    assert np.max(np.abs(np.array(ev) - ev0) / np.abs(ev0)) < 1e-10
    peak = st["workspace_peak"]
    print("workspace %d bytes, peak %d (%.2f), free memory moved by %d bytes" % (need, peak, peak / need,
                                                                              free0 - free1), flush=True)
    assert 0 < peak <= need and peak >= 0.5 * need
    assert abs(free0 - free1) < 8 << 20


def test_too_small_a_workspace_is_refused(P):
    w = levelgen.train_workload(2000, "L4")
    A = w.generate()
    print("case workspace too small n=%d" % A.n, flush=True)
    rp, col, val = P.upload(A)
    opts = P.sppc_default_opts()
    need = P.sppc_workspace_size(rp, col, val, A.level_offsets, w.n_small_levels, w.k, opts)
    for frac in (0.5, 0.9):
        ws = P.workspace_tensor(int(need * frac))
        with pytest.raises(P.SPPCError) as e:
            P.sppc_setup(rp, col, val, A.level_offsets, w.n_small_levels, w.k, opts, workspace=ws)
        assert e.value.status == P.SPPC_E_NOMEM
    # and the full size still works afterwards
    ws = P.workspace_tensor(need)
    ctx = P.sppc_setup(rp, col, val, A.level_offsets, w.n_small_levels, w.k, opts, workspace=ws)
    ev, _, rrn, st, status = P.sppc_solve(ctx, want_vectors=False)
    assert status == P.SPPC_OK
    P.sppc_destroy(ctx)


@pytest.mark.parametrize("name,sizes,d,seed,ns,k,tol", [
    ("rmmdiis hand-over", (7, 61, 509, 3001, 7919), 30, 505, 2, 4, 1e-6),
    ("rmmdiis refined after its check", (54, 451, 3771), 46, 789128, 2, 16, 1e-9)])
def test_hybrid_continuations_on_a_torch_workspace(P, name, sizes, d, seed, ns, k, tol):
    # the Davidson steps after a stagnated RMM-DIIS and the float64 refinement after a failed
    # check run inside the workspace that sppc_workspace_size sized for the hybrid
    A = levelgen.generate(sizes, d, seed)
    print("case workspace %s n=%d" % (name, A.n), flush=True)
    rp, col, val = P.upload(A)
    opts = P.sppc_default_opts(precond=P.SPPC_CORR_RMMDIIS, tol=tol, max_cont=200)
    need = P.sppc_workspace_size(rp, col, val, A.level_offsets, ns, k, opts)
    ctx = P.sppc_setup(rp, col, val, A.level_offsets, ns, k, opts)
    ev0, _, _, st0, s0 = P.sppc_solve(ctx, want_vectors=False)
    P.sppc_destroy(ctx)
    ws = P.workspace_tensor(need)
    ctx = P.sppc_setup(rp, col, val, A.level_offsets, ns, k, opts, workspace=ws)
    ev, _, rrn, st, status = P.sppc_solve(ctx, want_vectors=False)
    P.sppc_destroy(ctx)
    assert status == s0 == P.SPPC_OK and max(rrn) < tol
    assert st["rmm_handover"] + st["refine_steps"] > 0
    assert 0 < st["workspace_peak"] <= need
    assert np.max(np.abs(np.array(ev) - np.array(ev0)) / np.abs(np.array(ev0))) < 1e-10

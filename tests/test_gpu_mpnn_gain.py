"""What the trained preconditioner gains over the diagonal step, on matrices it was not trained on.

The committed weights were trained on seeds 1000..1023 of the n = 4900 three-level shape; the
held-out matrices are seeds 3000..3007 of that shape and one four-level n = 234,400 matrix.
Both preconditioners must reach the same eigenpairs.  In the Davidson continuation the learned
step must need at least 15% fewer continuation steps in total (fewer basis vectors, so less
Gram-Schmidt and Rayleigh-Ritz work) without a longer solve (wall time at most 1.1x the diagonal
step's, best of two runs).  Products with H are reported, counting the network's own two per pair
and application: at these sizes the learned form uses more of them than it saves.  The table is
printed (pytest -s).  The RMM-DIIS step's weights for five-level matrices are checked on two
held-out matrices of their training shape (last test).
"""
import json
import time

import numpy as np
import pytest
import torch

import levelgen

pytestmark = pytest.mark.gpu

HELD_OUT = [("n4900 seed%d" % sd, (100, 800, 4000), 60, sd, 1, 4) for sd in range(3000, 3008)]
HELD_OUT.append(("n234400 seed77 k8", (400, 4000, 30000, 200000), 100, 77, 2, 8))


@pytest.fixture(scope="module")
def P():
    import paper_2407_08901_amd as P
    P.lib()
    return P


def _solve(P, A, ns, k, kind, w=None, reps=2):
    rp, col, val = P.upload(A)
    best = None
    for _ in range(reps):
        ctx = P.sppc_setup(rp, col, val, A.level_offsets, ns, k, P.sppc_default_opts(precond=kind))
        if w is not None:
            P.sppc_mpnn_set_weights(ctx, w)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev, Z, rrn, st, status = P.sppc_solve(ctx)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        P.sppc_destroy(ctx)
        best = ms if best is None else min(best, ms)
    return np.array(ev), np.array(rrn), st, status, best


def test_trained_network_on_held_out_matrices(P):
    from paper_2407_08901_amd import mpnn_train
    w = mpnn_train.load_for("davidson")
    rows = []
    tot = {"cont_j": 0, "cont_m": 0, "prod_j": 0, "prod_m": 0, "ms_j": 0.0, "ms_m": 0.0}
    for name, sizes, d, sd, ns, k in HELD_OUT:
        print("case gain %s" % name, flush=True)
        A = levelgen.generate(sizes, d, sd)
        ev_j, rrn_j, st_j, s_j, ms_j = _solve(P, A, ns, k, P.SPPC_CORR_JACOBI)
        ev_m, rrn_m, st_m, s_m, ms_m = _solve(P, A, ns, k, P.SPPC_CORR_MPNN, w)
        assert s_j == P.SPPC_OK and s_m == P.SPPC_OK
        assert np.max(rrn_m) < 1e-6
        assert np.max(np.abs(ev_m - ev_j) / np.abs(ev_j)) < 1e-10
        for key, a, b in (("cont", st_j["cont_steps"], st_m["cont_steps"]), ("prod", st_j["n_spmv"], st_m["n_spmv"]),
                          ("ms", ms_j, ms_m)):
            tot[key + "_j"] += a
            tot[key + "_m"] += b
        rows.append(dict(matrix=name, cont_jacobi=st_j["cont_steps"], cont_mpnn=st_m["cont_steps"],
                         learned_steps=st_m["mpnn_steps"], fallbacks=st_m["mpnn_fallbacks"],
                         products_jacobi=st_j["n_spmv"], products_mpnn=st_m["n_spmv"],
                         ms_jacobi=round(ms_j, 1), ms_mpnn=round(ms_m, 1)))
    for r in rows:
        print(json.dumps(r))
    print(json.dumps(tot))
    assert tot["cont_m"] <= 0.85 * tot["cont_j"]
    assert tot["ms_m"] <= 1.1 * tot["ms_j"]


def test_learned_rmm_diis_step_on_held_out_five_level_matrices(P):
    """The RMM-DIIS step's weights for five-level matrices (trained on seeds 3000..3011 of the
    n = 386,100 five-level shape) on two held-out matrices of that shape: on the samples the method
    produces there (pair target, see mpnn_train) the network's loss is at most 0.8x the diagonal
    step's; in the mixed-precision SPPC + RMM-DIIS solve the learned step needs at most one sweep
    (4 iterations) per matrix more than the diagonal one over the two matrices together, counting the
    Davidson steps after a hand-over (RMM-DIIS slows to well under a halving per three sweeps on these
    matrices, and the sweep at which it hands over follows the rounding of the products; measured
    71-72 against 71), and both reach the same eigenvalues.  Products with H, wall times and the pairs that the residual sent back
    to the diagonal step are printed: each learned application costs two products of its own, and
    where RMM-DIIS itself converges slowly many pairs miss the 0.9x reduction the residual check asks
    of a learned step."""
    from paper_2407_08901_amd import mpnn_train
    w5 = mpnn_train.load_for("rmmdiis", 5)
    it_d = it_n = 0
    for sd in (3100, 3101):
        wl = levelgen.train_workload(sd, "L5")
        print("case learned RMM-DIIS step %s seed %d" % (wl.name, sd), flush=True)
        data = mpnn_train.build_dataset([sd], "L5", "pair", log=lambda m: None)
        loss_d = mpnn_train.evaluate(data, np.zeros(P.SPPC_MPNN_NPARAM, np.float32))
        loss_n = mpnn_train.evaluate(data, w5)
        for d in data:
            P.sppc_destroy(d["ctx"])
        A = wl.generate()
        rp, col, val = P.upload(A)
        out = {}
        for name, kw in (("diagonal", dict(rmm_precond=P.SPPC_CORR_JACOBI)),
                         ("learned", dict(rmm_precond=P.SPPC_CORR_MPNN))):
            ctx = P.sppc_setup(rp, col, val, A.level_offsets, wl.n_small_levels, wl.k,
                               P.sppc_default_opts(precision=P.SPPC_PREC_MIXED, precond=P.SPPC_CORR_RMMDIIS, **kw))
            if name == "learned":
                P.sppc_mpnn_set_weights(ctx, w5)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ev, Z, rrn, st, status = P.sppc_solve(ctx, want_vectors=False)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3
            P.sppc_destroy(ctx)
            assert status == P.SPPC_OK and max(rrn) < 1e-6, name
            out[name] = (np.array(ev), st, ms)
        ev_d, st_d, ms_d = out["diagonal"]
        ev_n, st_n, ms_n = out["learned"]
        print(json.dumps(dict(seed=sd, loss_diagonal=round(loss_d, 4), loss_network=round(loss_n, 4),
                              iterations_diagonal=st_d["cont_steps"], iterations_learned=st_n["cont_steps"],
                              rmm_iterations_diagonal=st_d["rmm_iterations"], rmm_iterations_learned=st_n["rmm_iterations"],
                              handover_diagonal=st_d["rmm_handover"], handover_learned=st_n["rmm_handover"],
                              learned_steps=st_n["mpnn_steps"], fallbacks=st_n["mpnn_fallbacks"],
                              products_diagonal=st_d["n_spmv"], products_learned=st_n["n_spmv"],
                              ms_diagonal=round(ms_d, 1), ms_learned=round(ms_n, 1))), flush=True)
        assert loss_n <= 0.8 * loss_d
        assert np.max(np.abs(ev_n - ev_d) / np.abs(ev_d)) < 1e-8
        it_d += st_d["cont_steps"]
        it_n += st_n["cont_steps"]
    assert it_n <= it_d + 8

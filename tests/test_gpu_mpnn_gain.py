"""What the trained preconditioner gains over the diagonal step, on matrices it was not trained on.

The committed weights were trained on seeds 1000..1019 of the n = 4900 three-level shape; the
held-out matrices are seeds 3000..3007 of that shape and one four-level n = 234,400 matrix.
Both preconditioners must reach the same eigenpairs; the learned one must need at least 10%
fewer continuation steps in total.  The measured table is printed (pytest -s).
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


def _solve(P, A, ns, k, kind, w=None):
    rp, col, val = P.upload(A)
    ctx = P.sppc_setup(rp, col, val, A.level_offsets, ns, k, P.sppc_default_opts(precond=kind))
    if w is not None:
        P.sppc_mpnn_set_weights(ctx, w)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev, Z, rrn, st, status = P.sppc_solve(ctx)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    P.sppc_destroy(ctx)
    return np.array(ev), np.array(rrn), st, status, ms


def test_trained_network_needs_fewer_continuation_steps(P):
    from paper_2407_08901_amd import mpnn_train
    w = mpnn_train.load()
    rows = []
    tot_j = tot_m = 0
    for name, sizes, d, sd, ns, k in HELD_OUT:
        print("case gain %s" % name, flush=True)
        A = levelgen.generate(sizes, d, sd)
        ev_j, rrn_j, st_j, s_j, ms_j = _solve(P, A, ns, k, P.SPPC_CORR_JACOBI)
        ev_m, rrn_m, st_m, s_m, ms_m = _solve(P, A, ns, k, P.SPPC_CORR_MPNN, w)
        assert s_j == P.SPPC_OK and s_m == P.SPPC_OK
        assert np.max(rrn_m) < 1e-6
        assert np.max(np.abs(ev_m - ev_j) / np.abs(ev_j)) < 1e-10
        tot_j += st_j["cont_steps"]
        tot_m += st_m["cont_steps"]
        rows.append(dict(matrix=name, cont_jacobi=st_j["cont_steps"], cont_mpnn=st_m["cont_steps"],
                         learned_steps=st_m["mpnn_steps"], products_jacobi=st_j["n_spmv"],
                         products_mpnn=st_m["n_spmv"], ms_jacobi=round(ms_j, 1), ms_mpnn=round(ms_m, 1)))
    for r in rows:
        print(json.dumps(r))
    print("continuation steps: diagonal %d, learned %d" % (tot_j, tot_m))
    assert tot_m <= 0.9 * tot_j

"""Writes the float64 CPU oracle's solution of a benchmark workload, for the full-size checks of
the GPU path.  Calls only oracle/ (and levelgen/ for the input).

Stored per workload (tests/golden/oracle_eigs_<name>.json):
  * E0       the 28 lowest eigenvalues of H0hat (dense eigendecomposition, Alg. 2 step 1);
  * steps    the Ritz values, relative residuals and basis size after every SPPC step
             p = 0..p_switch (Alg. 2, eq. rrn), in the float64 form with exact small solves;
  * evals    the k lowest eigenvalues, solved to rrn <= tol by SPPC + the diagonal-step
             continuation, certified by an explicit product (the final check).

The dense eigendecomposition of H0hat (n0 = 22,000) and the continuation to rrn 1e-10 dominate:
about 50 minutes on 8 cores for a workload of n = 1.17M.

    python tests/golden/make_oracle_eigs.py --workload 1 [--tol 1e-10]
    python tests/golden/make_oracle_eigs.py --workload L5-tenth
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import levelgen  # noqa: E402
import oracle  # noqa: E402

N_E0 = 28  # the most H0hat eigenpairs the GPU path deflates


def out_path(name: str) -> str:
    return os.path.join(HERE, "oracle_eigs_%s.json" % name.replace("/", "-"))


def workload(key: str) -> levelgen.Workload:
    if key in levelgen.EXTRA_WORKLOADS:
        return levelgen.EXTRA_WORKLOADS[key]
    return levelgen.WORKLOADS[int(key)]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="1")
    ap.add_argument("--tol", type=float, default=1e-10)
    args = ap.parse_args()
    w = workload(args.workload)
    t0 = time.time()
    A = w.generate()
    H = oracle.symmetric_from_upper(A.row_ptr, A.col, A.val, A.n)
    print("matrix %s n=%d nnz(full)=%d  %.0f s" % (w.name, A.n, H.nnz, time.time() - t0), flush=True)
    z = oracle.zeroth_order(oracle.core.small_space_matrix(H, w.n0))
    print("zeroth order (dense eigh of H0hat, n0=%d)  %.0f s" % (w.n0, time.time() - t0), flush=True)

    def log(h):
        print("%-7s p=%-3d m=%-4d max rrn %.3e  %.0f s" % (h["phase"], h["p"], h["m"], max(h["rrn"]),
                                                          time.time() - t0), flush=True)

    res = oracle.sppc(H, w.n0, w.k, oracle.Options(tol=args.tol), z=z, callback=log)
    steps = [{"p": int(h["p"]), "m": int(h["m"]), "theta": [float(x) for x in h["theta"]],
              "rrn": [float(x) for x in h["rrn"]]}
             for h in res.history if h["phase"] == "sppc"]
    rec = {
        "workload": w.name, "n": A.n, "n0": w.n0, "k": w.k, "matrix_sha256": A.sha256(),
        "tol": args.tol, "converged": bool(res.converged), "evals": [float(x) for x in res.theta],
        "rrn": [float(x) for x in res.rrn], "steps": len(res.history) - 1,
        "E0": [float(x) for x in z.w[:N_E0]],
        "sppc_steps": steps,
        "command": "python tests/golden/make_oracle_eigs.py --workload %s --tol %g" % (args.workload, args.tol),
        "seconds": round(time.time() - t0, 1),
    }
    with open(out_path(w.name), "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps({k: v for k, v in rec.items() if k != "sppc_steps"}), flush=True)


if __name__ == "__main__":
    np.set_printoptions(precision=17)
    main()

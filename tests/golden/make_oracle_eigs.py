"""Writes the float64 CPU oracle's k lowest eigenpairs' eigenvalues of a benchmark workload,
solved to a tight relative residual, for the full-size eigenvalue checks of the GPU path.
Calls only oracle/ (and levelgen/ for the input); takes about half an hour on 8 cores for
L4-2k/20k/150k/1M-d200-k8 (the dense eigendecomposition of H0hat, n0 = 22,000, dominates).

    python tests/golden/make_oracle_eigs.py [--workload 1] [--tol 1e-10]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import levelgen  # noqa: E402
import oracle  # noqa: E402


def out_path(name: str) -> str:
    return os.path.join(HERE, "oracle_eigs_%s.json" % name.replace("/", "-"))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", type=int, default=1)
    ap.add_argument("--tol", type=float, default=1e-10)
    args = ap.parse_args()
    w = levelgen.WORKLOADS[args.workload]
    t0 = time.time()
    A = w.generate()
    H = oracle.symmetric_from_upper(A.row_ptr, A.col, A.val, A.n)
    print("matrix n=%d nnz(full)=%d  %.0f s" % (A.n, H.nnz, time.time() - t0), flush=True)

    def log(h):
        print("%-5s p=%-3d m=%-4d max rrn %.3e  %.0f s" % (h["phase"], h["p"], h["m"], max(h["rrn"]),
                                                          time.time() - t0), flush=True)

    res = oracle.sppc(H, w.n0, w.k, oracle.Options(tol=args.tol), callback=log)
    rec = {
        "workload": w.name, "n": A.n, "n0": w.n0, "k": w.k, "matrix_sha256": A.sha256(),
        "tol": args.tol, "converged": bool(res.converged), "evals": [float(x) for x in res.theta],
        "rrn": [float(x) for x in res.rrn], "steps": len(res.history) - 1,
        "command": "python tests/golden/make_oracle_eigs.py --workload %d --tol %g" % (args.workload, args.tol),
        "seconds": round(time.time() - t0, 1),
    }
    with open(out_path(w.name), "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()

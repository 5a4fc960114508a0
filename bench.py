#!/usr/bin/env python3
"""Benchmark: time to the k lowest eigenpairs at relative residual 1e-6 on one MI355X, against
plain float64 SPPC on the same GPU.

One step = sppc_setup (device format, H0hat eigenpairs, p = 0) + sppc_solve (SPPC steps,
continuation, final float64 check) with H already resident in HBM as an upper-triangular CSR.
Default workload: L5-2k/20k/200k/1.5M/6M-d300-k16 (n = 7,722,000, 1.17e9 stored upper entries,
float32 values), k = 16.  The timed form (--mode, default mixed+rmmdiis+mpnn) is the mixed
precision + learned preconditioner form: float32 products with float64 accumulation, small-space
solves to 1e-6, the paper's SPPC + RMM-DIIS hybrid after the perturbative steps with the learned
correction of the diagonal step (per-pair fallback to the diagonal step, judged by the true
residual), and the float64 check.  The same number of steps of plain float64 SPPC (small solves
to 1e-12, Davidson continuation) and of the hybrid with the diagonal step follow (--no-compare
skips them; --full-compare adds more forms).  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload 4]
                  [--mode plain|mixed|plain+mpnn|mixed+mpnn|plain+small|mixed+small|plain+rmmdiis|
                          mixed+rmmdiis|plain+rmmdiis+mpnn|mixed+rmmdiis+mpnn|plain-inexact]
                  [--no-compare] [--full-compare] [--auto-switch]
                  [--no-cpu-baseline] [--calibrate-copy] [--spmm-only R [--spmm-f32] [--spmm-upper]]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published

# HBM traffic per product with H from FETCH_SIZE / WRITE_SIZE counter runs of this same command,
# scaled by a plain-copy calibration (profiles/k_spmm_panel_*_hbm_counters.md).
# Keyed by (workload, mode); valid only while the kernel source has the recorded sha256.
MEASURED_TRAFFIC = {
    # profiles/k_spmm_panel_L5-7.72M-k16_hbm_counters.md: per product the bench times (the library's own products of
    # one solve: 13 with float32 X, 9 with float64 X)
    ("L5-2k/20k/200k/1.5M/6M-d300-k16", "mixed+rmmdiis+mpnn"): (180413000000,
        "b24d19b347654d9e61af5f3cfd9da85c403873d830212cc4f350ede1e3cee8e0"),
}


def measured_traffic(workload, mode):
    import hashlib
    rec = MEASURED_TRAFFIC.get((workload, mode))
    if rec is None:
        return None
    src = os.path.join(ROOT, "paper_2407_08901_amd", "csrc", "kernels_sparse.hip")
    try:
        with open(src, "rb") as f:
            ok = hashlib.sha256(f.read()).hexdigest() == rec[1]
    except OSError:
        ok = False
    return rec[0] if ok else None
MODES = ("plain", "mixed", "plain+mpnn", "mixed+mpnn", "plain+small", "mixed+small", "plain+rmmdiis", "mixed+rmmdiis",
         "plain+rmmdiis+mpnn", "mixed+rmmdiis+mpnn", "plain-inexact")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", type=int, default=4)
    ap.add_argument("--mode", default="mixed+rmmdiis+mpnn", choices=MODES)
    ap.add_argument("--no-compare", action="store_true",
                    help="do not time plain float64 SPPC and the hybrid with the diagonal step as well")
    ap.add_argument("--full-compare", action="store_true",
                    help="also time the Davidson continuations, float64 with inexact small solves and the "
                         "automatic switch")
    ap.add_argument("--compare-steps", type=int, default=5,
                    help="timed steps of each comparison form (at most --steps)")
    ap.add_argument("--auto-switch", action="store_true",
                    help="switch to the continuation once SPPC stagnates instead of after step 15")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device copy of known size (HBM counter calibration)")
    ap.add_argument("--spmm-only", type=int, default=0,
                    help="only time this many block products with H (profiling runs)")
    ap.add_argument("--spmm-f32", action="store_true", help="with --spmm-only: float32 X (mixed form)")
    ap.add_argument("--n-deflate", type=int, default=0,
                    help="eigenpairs of H0hat deflated in the small-space solves (0: the library's default)")
    ap.add_argument("--rmm-weights", default=None,
                    help="weights file of the learned RMM-DIIS step (default: the package's)")
    ap.add_argument("--spmm-width", type=int, default=0, help="with --spmm-only: block width (default k)")
    ap.add_argument("--spmm-upper", action="store_true",
                    help="with --spmm-only: also time the product from the upper triangle alone")
    ap.add_argument("--panel-width", type=int, default=-1,
                    help="columns per panel of the block product (-1 automatic, 0 plain CSR)")
    ap.add_argument("--verbose", action="store_true")
    return ap.parse_args()


def calibrate_copy():
    import torch
    nbytes = 1 << 30
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_each_way": nbytes, "launches": 5}))


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: the solver runs on one GPU (it has no multi-GPU path); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy()
        return
    import torch
    import levelgen
    import paper_2407_08901_amd as P

    P.lib()
    w = levelgen.WORKLOADS[args.workload]
    t0 = time.time()
    A = w.generate()
    t_gen = time.time() - t0
    # the n = 7.7M workload is stored with float32 values (14 GB upper triangle); the others are
    # handed over in float64 (every value is float32-exact either way)
    rp, col, val = P.upload(A, dtype=torch.float32 if args.workload == 4 else torch.float64)
    torch.cuda.synchronize()

    if args.spmm_only:
        opts = P.sppc_default_opts(precision=P.SPPC_PREC_MIXED if args.spmm_f32 else P.SPPC_PREC_FP64,
                                   panel_width=args.panel_width)
        ctx = P.sppc_setup(rp, col, val, A.level_offsets, w.n_small_levels, w.k, opts)
        X = torch.randn(A.n, args.spmm_width or w.k, dtype=torch.float64, device="cuda")
        if args.spmm_f32:
            X = X.float()
        Y = torch.empty(A.n, X.shape[1], dtype=torch.float64, device="cuda")
        P.sppc_spmm(ctx, X, Y)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.spmm_only):
            P.sppc_spmm(ctx, X, Y)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.spmm_only
        rec = {"spmm_launches": args.spmm_only, "n": A.n, "b": X.shape[1], "panel_width": args.panel_width,
               "x": "f32" if args.spmm_f32 else "f64", "ms_per_launch_wall": round(dt * 1e3, 4)}
        if args.spmm_upper:
            # the same product from the upper triangle alone (float64 atomic adds for the lower half)
            Y2 = torch.empty_like(Y)
            P.sppc_spmm_upper(rp, col, val, X, Y2)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.spmm_only):
                P.sppc_spmm_upper(rp, col, val, X, Y2)
            torch.cuda.synchronize()
            dt2 = (time.perf_counter() - t0) / args.spmm_only
            rel = float(((Y2 - Y).abs().max() / Y.abs().max()).item())
            mat_full = (2 * int(A.row_ptr[-1]) - A.n) * (4 + val.element_size()) + (A.n + 1) * 8
            mat_up = int(A.row_ptr[-1]) * (4 + val.element_size()) + (A.n + 1) * 8
            rec.update({"upper_ms_per_launch_wall": round(dt2 * 1e3, 4), "upper_vs_full_max_rel_diff": rel,
                        "matrix_bytes_full": mat_full, "matrix_bytes_upper": mat_up})
        print(json.dumps(rec))
        return

    from paper_2407_08901_amd import mpnn_train
    weights = {"davidson": mpnn_train.load_for("davidson"),
               "rmmdiis": mpnn_train.load(args.rmm_weights) if args.rmm_weights
               else mpnn_train.load_for("rmmdiis", len(w.level_sizes))}

    def mode_opts(mode, auto_switch=None):
        auto_switch = args.auto_switch if auto_switch is None else auto_switch
        mixed = mode.startswith("mixed")
        rmm = "+rmmdiis" in mode
        mpnn = mode.endswith("mpnn")
        precond = (P.SPPC_CORR_RMMDIIS if rmm else P.SPPC_CORR_MPNN if mpnn else
                   P.SPPC_CORR_SMALL if mode.endswith("small") else P.SPPC_CORR_JACOBI)
        # plain-inexact: float64 with the small-space solves to the mixed form's inner tolerance
        extra = {"inner_tol": 1e-6} if mode == "plain-inexact" else {}
        if rmm and mpnn:
            extra["rmm_precond"] = P.SPPC_CORR_MPNN
        return P.sppc_default_opts(precision=P.SPPC_PREC_MIXED if mixed else P.SPPC_PREC_FP64, precond=precond,
                                   verbose=1 if args.verbose else 0, panel_width=args.panel_width,
                                   auto_switch=1 if auto_switch else 0, n_deflate=args.n_deflate, **extra)

    # one device workspace from PyTorch for every context of the run (the largest any timed form
    # needs), allocated before the timing: no allocation or release inside the timed steps
    forms = [(args.mode, None)]
    if not args.no_compare:
        forms += [("plain", False), ("mixed+rmmdiis", False)]
        if args.full_compare:
            forms += [("mixed+mpnn", False), ("plain-inexact", False), ("mixed", False), ("mixed+rmmdiis", True)]
    ws_bytes = max(P.sppc_workspace_size(rp, col, val, A.level_offsets, w.n_small_levels, w.k, mode_opts(m, a))
                   for m, a in forms)
    workspace = P.workspace_tensor(ws_bytes)

    def make_step(mode, auto_switch=None):
        mpnn = mode.endswith("mpnn")
        rmm = "+rmmdiis" in mode
        opts = mode_opts(mode, auto_switch)

        def one_step():
            ctx = P.sppc_setup(rp, col, val, A.level_offsets, w.n_small_levels, w.k, opts, workspace=workspace)
            if mpnn:
                P.sppc_mpnn_set_weights(ctx, weights["rmmdiis" if rmm else "davidson"])
            ev, Z, rrn, st, status = P.sppc_solve(ctx, want_vectors=True)
            P.sppc_destroy(ctx)
            return ev, rrn, st, status
        return one_step

    def timed(mode, auto_switch=None, steps=None, warmup=None):
        steps = args.steps if steps is None else steps
        warmup = args.warmup if warmup is None else warmup
        one_step = make_step(mode, auto_switch)
        for _ in range(warmup):
            one_step()
        torch.cuda.synchronize()
        results = []
        t_start = time.perf_counter()
        for _ in range(steps):
            results.append(one_step())
        torch.cuda.synchronize()
        return (time.perf_counter() - t_start) / steps, results

    per, results = timed(args.mode)
    ev, rrn, st, status = results[-1]

    # roofline of the dominant kernel: the block product with H, from the library's own HIP
    # events on its stream (kernel launches only) and its algorithmic byte count
    spmm_ms = sum(r[2]["t_spmm_ms"] for r in results)
    spmm_calls = sum(r[2]["spmm_calls"] for r in results)
    alg_bytes = sum(r[2]["spmm_alg_bytes"] for r in results)
    achieved = alg_bytes / (spmm_ms * 1e-3) / 1e9 if spmm_ms > 0 else 0.0
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None if args.auto_switch else measured_traffic(w.name, args.mode),
            "kernel": "k_spmm_panel (block product with H; one product is a sequence of round launches)",
            "launches": spmm_calls,
            "avg_launch_ms": round(spmm_ms / max(spmm_calls, 1), 4),
            "alg_bytes_per_launch_avg": int(alg_bytes / max(spmm_calls, 1))}

    mixed = args.mode.startswith("mixed")
    fallbacks = sum(r[2]["mpnn_fallbacks"] for r in results)
    learned_its = sum(r[2]["mpnn_steps"] for r in results)
    line = {
        "metric": "time to k eigenpairs at resid 1e-6 vs plain FP64 SPPC; SpMM HBM GB/s",
        "value": round(per, 4), "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(per * 1e3, 2), "higher_is_better": False, "scaling": "strong",
        "vs_baseline": None, "dtype": "f32+f64" if mixed else "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "n": A.n, "n0": w.n0, "k": w.k, "nnz_upper": A.nnz,
                   "tol": 1e-6, "mode": args.mode, "auto_switch": bool(args.auto_switch)},
        "converged": bool(st["converged"]), "max_rrn": max(rrn), "evals": ev,
        "iterations": st["iterations"], "cont_steps": st["cont_steps"], "refine_steps": st["refine_steps"],
        "mpnn_steps": st["mpnn_steps"], "n_spmv": st["n_spmv"],
        "rmm_iterations": st["rmm_iterations"], "rmm_handover": bool(st["rmm_handover"]),
        "learned": {"iterations_per_solve": round(learned_its / len(results), 2),
                    "fallback_pairs_per_solve": round(fallbacks / len(results), 2),
                    "fallback_rate": round(fallbacks / (len(results) * w.k), 4)},
        "breakdown_ms": {k: round(st[k], 2) for k in ("t_setup_ms", "t_solve_ms", "t_spmm_ms", "t_small_ms",
                                                      "t_ortho_ms", "t_rr_ms", "t_h0_ms")},
        "cg_iterations": st["cg_iterations"], "h0_iterations": st["h0_iterations"],
        "workspace": {"bytes": ws_bytes, "peak": st["workspace_peak"], "source": "torch.empty (caller-owned)"},
        "roofline": roof,
        "generate_s": round(t_gen, 2),
    }
    ev_p = None
    if not args.no_compare:
        csteps = max(1, min(args.steps, args.compare_steps))
        cwarm = min(args.warmup, 1)

        def summary(mode, auto_switch=False):
            same = mode == args.mode and auto_switch == args.auto_switch
            per_m, res_m = (per, results) if same else timed(mode, auto_switch, csteps, cwarm)
            ev_m, rrn_m, st_m, _ = res_m[-1]
            return per_m, ev_m, {"s": round(per_m, 4), "steps": len(res_m), "iterations": st_m["iterations"],
                                 "cont_steps": st_m["cont_steps"], "refine_steps": st_m["refine_steps"],
                                 "mpnn_steps": st_m["mpnn_steps"], "n_spmv": st_m["n_spmv"],
                                 "rmm_iterations": st_m["rmm_iterations"], "rmm_handover": bool(st_m["rmm_handover"]),
                                 "max_rrn": max(rrn_m), "converged": bool(st_m["converged"])}
        per_p, ev_p, d = summary("plain")
        line["plain_fp64"] = dict(d, max_rel_eval_diff=float(np.max(np.abs(np.array(ev) - np.array(ev_p)) /
                                                                      np.abs(np.array(ev_p)))))
        line["speedup_vs_plain_fp64"] = round(per_p / per, 3)
        # the same hybrid with the diagonal step: what the network gains or costs
        base = args.mode.replace("+mpnn", "") if args.mode.endswith("rmmdiis+mpnn") else "mixed+rmmdiis"
        per_r, ev_r, d = summary(base)
        line["without_network" if base != args.mode else "mixed_rmmdiis"] = dict(
            d, mode=base, speedup_vs_plain=round(per_p / per_r, 3), value_over_this=round(per / per_r, 3))
        if args.full_compare:
            per_l, ev_l, d = summary("mixed+mpnn")
            line["mixed_learned_davidson"] = dict(d, speedup_vs_plain=round(per_p / per_l, 3))
            per_i, ev_i, d = summary("plain-inexact")
            line["plain_fp64_inner_1e-6"] = dict(d, speedup_vs_plain=round(per_p / per_i, 3))
            per_d, ev_d, d = summary("mixed")
            line["mixed_davidson"] = dict(d, speedup_vs_plain=round(per_p / per_d, 3))
            per_a, ev_a, d = summary("mixed+rmmdiis", auto_switch=True)
            line["mixed_rmmdiis_auto_switch"] = dict(d, speedup_vs_plain=round(per_p / per_a, 3))
    # each eigenvalue's error against the float64 oracle's solution of this matrix, stored by
    # tests/golden/make_oracle_eigs.py (solved there to rrn 1e-10), when it is present
    ref = oracle_eigs(w, A)
    if ref is not None:
        line["eval_rel_err_vs_oracle"] = [float(abs(a - b) / abs(b)) for a, b in zip(ev, ref)]
        if ev_p is not None:
            line["plain_fp64"]["max_eval_rel_err_vs_oracle"] = float(
                np.max(np.abs(np.array(ev_p) - ref) / np.abs(ref)))
    else:
        line["eval_rel_err_vs_oracle"] = None  # no stored oracle solution of this matrix
    if not args.no_cpu_baseline:
        steps_ref = line.get("plain_fp64", {"iterations": st["iterations"], "cont_steps": st["cont_steps"]})
        line["cpu_baseline"] = cpu_baseline(A, w, steps_ref["iterations"] + steps_ref["cont_steps"] + 1)
    print(json.dumps(line))


def oracle_eigs(w, A):
    path = os.path.join(ROOT, "tests", "golden", "oracle_eigs_%s.json" % w.name.replace("/", "-"))
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("workload") != w.name or rec.get("matrix_sha256") != A.sha256() or not rec.get("converged"):
        return None
    return np.array(rec["evals"])


def cpu_baseline(A, w, steps):
    """The CPU oracle timed on bounded samples of the same workload, extrapolated to one solve of
    `steps` SPPC + continuation steps (the plain float64 run's count: the oracle follows that form).

    One oracle step = one direct block product with H for H Psi^(p-1), the k exact spectral
    small-space solves, block Gram-Schmidt + QR, one block product with H for the new block and
    Rayleigh-Ritz.  Pieces: the block product from the upper triangle (oracle.product_from_upper)
    timed on the leading rows that hold ~2% of the stored entries and scaled by the entry count;
    one exact small solve on a 2000-row leading block of H0hat scaled by (n0/2000)^2 per column;
    Gram-Schmidt + QR + Rayleigh-Ritz on a 200,000-row sample scaled by n / 200,000; the dense
    eigendecomposition of H0hat timed on its leading 2000 x 2000 block and scaled by (n0/2000)^3.
    """
    import platform
    import subprocess

    import scipy.sparse as sp
    import threadpoolctl

    from oracle import core as oc
    info = threadpoolctl.threadpool_info()
    threads = max([i.get("num_threads", 1) for i in info] + [1])
    try:
        model = [l.split(":", 1)[1].strip() for l in subprocess.run(["lscpu"], capture_output=True, text=True).stdout.splitlines()
                 if l.startswith("Model name")][0]
    except Exception:
        model = platform.processor() or "unknown"
    n, n0, k = A.n, w.n0, w.k
    rng = np.random.default_rng(0)
    # (1) block product with H from the upper triangle, on the leading rows (~2% of the entries)
    r1 = int(np.searchsorted(A.row_ptr, 0.02 * A.nnz))
    r1 = max(1, min(n, r1))
    e1 = int(A.row_ptr[r1])
    X = rng.standard_normal((n, k))
    t0 = time.perf_counter()
    oc.product_from_upper(np.concatenate([A.row_ptr[:r1 + 1], np.full(n - r1, e1, dtype=np.int64)]),
                          A.col[:e1], A.val[:e1], n, X)
    t_spmm = (time.perf_counter() - t0) * A.nnz / max(e1, 1)
    # (2) zeroth order: dense eigh of the leading ns x ns block of H0hat, scaled by (n0/ns)^3
    ns = min(n0, 2000)
    U = sp.csr_matrix((A.val[:int(A.row_ptr[ns])].astype(np.float64), A.col[:int(A.row_ptr[ns])],
                       A.row_ptr[:ns + 1]), shape=(ns, n)).tocsc()[:, :ns].toarray()
    H0s = U + U.T - np.diag(np.diag(U))
    t0 = time.perf_counter()
    z_s = oc.zeroth_order(H0s)
    t_eig = (time.perf_counter() - t0) * (n0 / ns) ** 3
    # (3) one exact small-space solve on the leading ns block, scaled by (n0/ns)^2 per column
    t0 = time.perf_counter()
    oc.small_solve(z_s, 0, rng.standard_normal(ns))
    t_small = (time.perf_counter() - t0) * (n0 / ns) ** 2 * k
    # (4) block Gram-Schmidt + QR and Rayleigh-Ritz at the mean basis size, on a row sample
    m = max(k, steps * k // 2)
    nr = min(n, 200000)
    Q = np.linalg.qr(rng.standard_normal((nr, m)))[0]
    HQ = rng.standard_normal((nr, m))
    Psi = rng.standard_normal((nr, k))
    t0 = time.perf_counter()
    oc.orthonormalize_block(Q, Psi, 1e-10)
    oc.rayleigh_ritz(Q, HQ, k)
    t_dense = (time.perf_counter() - t0) * n / nr
    per_step = 2 * t_spmm + t_small + t_dense
    est = t_eig + steps * per_step
    return {"value": round(est, 1), "unit": "s", "cores": threads, "kind": "oracle", "extrapolated": True,
            "cpu": model, "threads_env": {v: os.environ.get(v) for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS")},
            "sample": ("extrapolation from bounded samples of the oracle on this workload (%s, %d BLAS threads): "
                       "block product from the upper triangle on the leading %d rows (%.1f%% of the entries), "
                       "scaled: %.2f s per product; dense eigh of the leading %dx%d block of H0hat scaled by "
                       "(n0/%d)^3: %.1f s; %d exact small solves (one timed at n0=%d, scaled by (n0/%d)^2): %.2f s; "
                       "Gram-Schmidt+QR and Rayleigh-Ritz at m=%d on %d rows, scaled to n: %.2f s; per step 2 "
                       "products + small solves + dense; x %d steps (the plain float64 run's SPPC + "
                       "continuation steps)") % (model, threads, r1, 100.0 * e1 / A.nnz, t_spmm, ns, ns, ns, t_eig,
                                                 k, ns, ns, t_small, m, nr, t_dense, steps)}


if __name__ == "__main__":
    main()

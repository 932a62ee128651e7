"""Benchmark: d = 3, n = 512 triangular Kronecker solve on one MI355X.

Workload: sum_mu X x_mu T_mu = B with T_mu upper quasi-triangular (real Schur
form: diagonal U[1,2], strict upper N(0,1)/sqrt(n), a 2x2 bump at every 8th
position), B ~ N(0,1), seeded synthetic inputs resident in HBM.  One step is
one complete triangular solve (copy of B into X, every leaf wave and every
update).  Metric: TFLOP/s = F_tri / t_step with
F_tri = 2 sum_mu (n_mu (n_mu - 1)/2 + bumps_mu) N / n_mu (one FMA = 2 flops).

Prints one JSON line (rank 0, N = 1).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64 = 78.6  # TFLOP/s, MI355X dense FP64 (matrix = vector)
PEAK_HBM = 8000.0  # GB/s


def cpu_baseline(n, seed, cores):
    """The oracle (plain C, OpenMP) on a bounded sample of the same workload:
    the far-corner sub-problem [n-s, n)^3, which is itself a triangular
    Laplace-like equation with the trailing diagonal blocks of T."""
    import numpy as np

    import oracle
    import tt_inputs as ti
    s = min(n, 400)
    lo = n - s
    p = ti.laplace_tri((n, n, n), seed=seed, bumps="every8")
    while p["T"][0][lo, lo - 1] != 0.0:  # do not cut a 2x2 block
        lo -= 1
    T = [np.ascontiguousarray(t[lo:, lo:]) for t in p["T"]]
    B = np.ascontiguousarray(p["B"][lo:, lo:, lo:])
    if cores:
        oracle.set_threads(cores)
    F = oracle.flops_tri(T, B.shape)
    t0 = time.perf_counter()
    oracle.lap_solve(T, B)
    dt = time.perf_counter() - t0
    return {"value": F / dt / 1e12, "unit": "TFLOP/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"far-corner sub-problem {B.shape[0]}^3 of the same d=3 n={n} workload "
                      f"({F:.3e} flops in {dt:.2f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--nmin", type=int, default=0)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-cores", type=int, default=0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the triangular solve of one equation runs on one device).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1905_09539_amd as tt
    import tt_inputs as ti

    n = args.n
    p = ti.laplace_tri((n, n, n), seed=args.seed, bumps="every8")
    T = [torch.from_numpy(t).cuda() for t in p["T"]]
    B = torch.from_numpy(p["B"]).cuda()
    X = torch.empty_like(B)
    t0 = time.perf_counter()
    plan = tt.Plan(T, B.shape, nmin=args.nmin)
    plan_s = time.perf_counter() - t0
    flops = plan.flops
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        plan.solve(B, X)
    plan.status()
    torch.cuda.synchronize()

    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        plan.solve(B, X)
    e1.record(stream)
    torch.cuda.synchronize()
    plan.status()
    ms = e0.elapsed_time(e1) / args.steps
    tflops = flops / (ms * 1e-3) / 1e12

    # per-kernel-class timing: HIP events around every launch, each on the
    # stream the launch is on (leaves: the caller's stream; updates: the
    # plan's side stream)
    prof = plan.profile(B, X)
    upd, leaf = prof["update"], prof["leaf"]
    ach = upd["flops"] / (upd["ms"] * 1e-3) / 1e12
    roof = {"bound": "mfma", "achieved": ach, "peak": PEAK_FP64, "unit": "TFLOP/s", "frac": ach / PEAK_FP64,
            "kernel": "upd_kernel", "traffic": None}
    kernels = {
        "upd_kernel": {"ms": upd["ms"], "launches": upd["launches"], "tflops": ach,
                       "gbs": upd["bytes"] / (upd["ms"] * 1e-3) / 1e9},
        "leaf_kernel": {"ms": leaf["ms"], "launches": leaf["launches"],
                        "tflops": leaf["flops"] / (leaf["ms"] * 1e-3) / 1e12,
                        "gbs": leaf["bytes"] / (leaf["ms"] * 1e-3) / 1e9},
        "leaf_span_ms": prof["leaf_span_ms"],
    }

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(n, args.seed, args.cpu_cores)

    out = {
        "metric": "TFLOP/s of d=3 n=512 triangular solve",
        "value": tflops,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"d=3 triangular Laplace-like solve, n1=n2=n3={n}, T_mu real Schur form "
                               "(diag U[1,2], N(0,1)/sqrt(n) upper, 2x2 bump every 8th row), B~N(0,1)",
                   "n": n, "flops": flops, "leaf_nmin": args.nmin or 16},
        "frac_of_fp64_peak": tflops / PEAK_FP64,
        "roofline": roof,
        "kernels": kernels,
        "plan_build_s": plan_s,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()

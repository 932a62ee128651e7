"""Benchmark: d = 3, n = 512 triangular Kronecker solve on one MI355X.

Workload: sum_mu X x_mu T_mu = B with T_mu upper quasi-triangular (real Schur
form: diagonal U[1,2], strict upper N(0,1)/sqrt(n), a 2x2 bump at every 8th
position), B ~ N(0,1), seeded synthetic inputs resident in HBM.  One step is
one complete triangular solve (every leaf wave and every update; the
right-hand side is read from B and the solution written to X).  Metric: TFLOP/s = F_tri / t_step with
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
    """The oracle (plain C, OpenMP) on the same workload: one run of the whole
    n^3 solve on all host cores, and a single-thread run on the far-corner
    sub-problem [n-s, n)^3 (itself a triangular Laplace-like equation with
    the trailing diagonal blocks of T)."""
    import numpy as np

    import oracle
    import tt_inputs as ti
    p = ti.laplace_tri((n, n, n), seed=seed, bumps="every8")
    if cores:
        oracle.set_threads(cores)
    F = oracle.flops_tri(p["T"], p["B"].shape)
    t0 = time.perf_counter()
    oracle.lap_solve(p["T"], p["B"])
    dt = time.perf_counter() - t0
    all_cores = oracle.num_threads()
    s = min(n, 256)
    lo = n - s
    while lo > 0 and p["T"][0][lo, lo - 1] != 0.0:  # do not cut a 2x2 block
        lo -= 1
    T = [np.ascontiguousarray(t[lo:, lo:]) for t in p["T"]]
    B = np.ascontiguousarray(p["B"][lo:, lo:, lo:])
    F1 = oracle.flops_tri(T, B.shape)
    oracle.set_threads(1)
    t1 = time.perf_counter()
    oracle.lap_solve(T, B)
    dt1 = time.perf_counter() - t1
    oracle.set_threads(all_cores)
    return {"value": F / dt / 1e12, "unit": "TFLOP/s", "cores": all_cores, "kind": "oracle",
            "sample": f"the whole d=3 n={n} solve of the same workload, one run ({F:.4e} flops in {dt:.2f} s)",
            "single_thread": {"value": F1 / dt1 / 1e12, "unit": "TFLOP/s", "cores": 1,
                              "sample": f"far-corner sub-problem {B.shape[0]}^3 of the same workload "
                                        f"({F1:.4e} flops in {dt1:.2f} s)"}}


def measured_traffic():
    """HBM bytes per launch of the leaf and update kernels from the committed
    rocprofv3 counter summary (FETCH_SIZE and WRITE_SIZE, scaled by the same
    counters for a plain copy of known size), or None for a kernel whose
    sources changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "tri512_pmc_traffic.md")
    out = {}
    if not os.path.exists(path):
        return out
    h = hashlib.sha256()
    for f in ["tt_leaf.hip", "tt_kernels.hip", "tt_plan.cpp"]:
        with open(os.path.join(ROOT, "paper_1905_09539_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    digest, vals = None, {}
    with open(path) as fh:
        for line in fh:
            parts = line.strip().strip("`").split()
            if len(parts) == 2 and parts[0] == "sources_sha256:":
                digest = parts[1]
            if len(parts) == 3 and parts[0] == "bytes_per_launch:":
                vals[parts[1]] = float(parts[2])
    if digest != h.hexdigest():
        return out
    return vals


def _timed(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def _residual(A, X, B):
    """||B - sum_mu X x_mu A_mu||_F / ||B||_F with torch matmul (d = 3)."""
    import torch
    n0, n1, n2 = X.shape
    R = B.clone()
    R -= torch.matmul(A[0], X.reshape(n0, n1 * n2)).reshape(n0, n1, n2)
    R -= torch.matmul(A[1], X)
    R -= torch.matmul(X, A[2].t().contiguous())
    return float(torch.linalg.vector_norm(R) / torch.linalg.vector_norm(B))


def _pair_residual(A, C, X, B):
    """||B - sum_mu X x_1 C_1 .. x_mu A_mu .. x_d C_d||_F / ||B||_F (torch)."""
    import torch
    R = B.clone()
    d = X.dim()
    for mu in range(d):
        Y = X
        for nu in range(d):
            M = A[nu] if nu == mu else C[nu]
            Y = torch.movedim(torch.tensordot(M, Y, dims=([1], [nu])), 0, nu)
        R -= Y
    return float(torch.linalg.vector_norm(R) / torch.linalg.vector_norm(B))


class _Progress(dict):
    """Result dict that reports each finished workload on stderr."""

    def __setitem__(self, key, value):
        super().__setitem__(key, value)
        print(f"bench: {key} {json.dumps(value)}", file=sys.stderr, flush=True)


def extras(args):
    """The other workloads of the method, timed the same way (inputs resident
    in HBM, HIP events on the caller's stream).  args.only: None (all) or a
    list of name prefixes."""
    import torch

    import paper_1905_09539_amd as tt
    import tt_inputs as ti
    out = _Progress()
    steps = max(2, args.steps // 4)

    def want(name):
        return args.only is None or any(name.startswith(w) for w in args.only)

    def flush():
        torch.cuda.synchronize()
        torch.cuda.empty_cache()

    if want("dense_512"):
        # dense coefficients, d = 3, n = 512 (Algorithm 1: transforms + solve)
        n = 512
        p = ti.laplace_dense((n, n, n), seed=args.seed)
        B = torch.from_numpy(p["B"]).cuda()
        X = torch.empty_like(B)
        plan = tt.Plan(p["A"], B.shape, general=True)
        ms = _timed(lambda: plan.solve(B, X), steps, 1)
        plan.status()
        Ad = [torch.from_numpy(a).cuda() for a in p["A"]]
        out["dense_512"] = {"ms": ms, "tflops": plan.flops / (ms * 1e-3) / 1e12, "flops": plan.flops,
                            "host_schur_s": plan.info()["schur_seconds"], "residual": _residual(Ad, X, B)}
        del plan, B, X, Ad, p
        flush()

    if want("mixed_768"):
        # mixed precision vs FP64, d = 3, n = 768, eigenvalue sums in [3, 6]
        n = 768
        p = ti.laplace_dense((n, n, n), seed=args.seed)
        B = torch.from_numpy(p["B"]).cuda()
        Ad = [torch.from_numpy(a).cuda() for a in p["A"]]
        X64 = torch.empty_like(B)
        Xmp = torch.empty_like(B)
        plan64 = tt.Plan(p["A"], B.shape, general=True)
        ms64 = _timed(lambda: plan64.solve(B, X64), 2, 1)
        plan64.status()
        r64 = _residual(Ad, X64, B)
        del plan64
        flush()
        res = {"ms_fp64": ms64, "residual_fp64": r64}
        for name, prec in (("fp32", tt.TT_MP_FP32), ("bf16", tt.TT_MP_BF16)):
            planmp = tt.Plan(p["A"], B.shape, general=True, prec=prec, tol=1e-13)
            msmp = _timed(lambda: planmp.solve(B, Xmp), 2, 1)
            planmp.status()
            info = planmp.info()
            rmp = _residual(Ad, Xmp, B)
            diff = float(torch.linalg.vector_norm(Xmp - X64) / torch.linalg.vector_norm(X64))
            res.update({f"ms_mp_{name}": msmp, f"speedup_{name}": ms64 / msmp,
                        f"iterations_{name}": info["iterations"], f"last_ratio_{name}": info["ratio"],
                        f"residual_mp_{name}": rmp, f"rel_diff_{name}_vs_fp64": diff})
            del planmp
            flush()
        out["mixed_768"] = res
        del B, Ad, X64, Xmp, p
        flush()

    # pair form, d = 4: (96, 96, 96, 96) and the merge case (1024, 1024, 8, 8)
    for shp in [(96, 96, 96, 96), (1024, 1024, 8, 8)]:
        key = "pair_" + "x".join(str(x) for x in shp)
        if not want(key):
            continue
        p = ti.pair_tri(shp, seed=args.seed)
        A = [torch.from_numpy(a).cuda() for a in p["A"]]
        C = [torch.from_numpy(c).cuda() for c in p["C"]]
        B = torch.from_numpy(p["B"]).cuda()
        X = torch.empty_like(B)
        plan = tt.Plan(A, B.shape, C=C)
        ms = _timed(lambda: plan.solve(B, X), steps, 1)
        plan.status()
        out[key] = {"ms": ms, "flops": plan.flops, "tflops": plan.flops / (ms * 1e-3) / 1e12}
        del plan, A, C, B, X, p
        flush()

    if want("general_pair"):
        # dense pairs, d = 4 (96, 96, 96, 96): host QZ per mode, then
        # transforms and the triangular solve on the GPU
        p = ti.pair_dense((96, 96, 96, 96), seed=args.seed)
        B = torch.from_numpy(p["B"]).cuda()
        X = torch.empty_like(B)
        plan = tt.Plan(p["A"], B.shape, C=p["C"], general=True)
        ms = _timed(lambda: plan.solve(B, X), steps, 1)
        plan.status()
        Ad = [torch.from_numpy(a).cuda() for a in p["A"]]
        Cd = [torch.from_numpy(c).cuda() for c in p["C"]]
        out["general_pair_96x96x96x96"] = {"ms": ms, "flops": plan.flops,
                                           "tflops": plan.flops / (ms * 1e-3) / 1e12,
                                           "host_qz_s": plan.info()["schur_seconds"],
                                           "residual": _pair_residual(Ad, Cd, X, B)}
        del plan, Ad, Cd, B, X, p
        flush()

    # second operator class (eq. (3.1)), triangular, d = 3 and d = 4
    for shp in [(384, 384, 384), (96, 96, 96, 96)]:
        key = "gsylv_" + "x".join(str(x) for x in shp)
        if not want(key):
            continue
        p = ti.gsylv_tri(shp, seed=args.seed)
        A = [torch.from_numpy(a).cuda() for a in p["A"]]
        C = torch.from_numpy(p["C"]).cuda()
        B = torch.from_numpy(p["B"]).cuda()
        X = torch.empty_like(B)
        plan = tt.Plan(A, B.shape, C=C, gsylv=True)
        ms = _timed(lambda: plan.solve(B, X), steps, 1)
        plan.status()
        # ||B - X x_1 A_1 - X x_1 C x_2 A_2 .. x_d A_d||_F / ||B||_F
        R = B - torch.tensordot(A[0], X, dims=([1], [0]))
        Y = X
        for nu in range(len(shp)):
            Y = torch.movedim(torch.tensordot(C if nu == 0 else A[nu], Y, dims=([1], [nu])), 0, nu)
        R -= Y
        out[key] = {"ms": ms, "flops": plan.flops, "tflops": plan.flops / (ms * 1e-3) / 1e12,
                    "residual": float(torch.linalg.vector_norm(R) / torch.linalg.vector_norm(B))}
        del plan, A, C, B, X, p, R, Y
        flush()

    if want("order5"):
        # order 5 (Laplace-like, merged pair of modes), (40, 40, 40, 40, 40)
        shp = (40, 40, 40, 40, 40)
        p = ti.laplace_tri(shp, seed=args.seed)
        T = [torch.from_numpy(t).cuda() for t in p["T"]]
        B = torch.from_numpy(p["B"]).cuda()
        X = torch.empty_like(B)
        plan = tt.Plan(T, B.shape)
        ms = _timed(lambda: plan.solve(B, X), steps, 1)
        plan.status()
        R = B.clone()
        for mu in range(5):
            R -= torch.movedim(torch.tensordot(T[mu], X, dims=([1], [mu])), 0, mu)
        out["order5_40"] = {"ms": ms, "flops": plan.flops, "tflops": plan.flops / (ms * 1e-3) / 1e12,
                            "residual": float(torch.linalg.vector_norm(R) / torch.linalg.vector_norm(B))}
        del plan, T, B, X, p, R
        flush()

    if want("adjoint"):
        # adjoint: 64 uneven d = 3 problems, forward + backward (dB and dT)
        probs = ti.uneven_batch(64, 32, 192, seed=args.seed)
        T = [[torch.from_numpy(t).cuda() for t in q["T"]] for q in probs]
        Bs = [torch.from_numpy(q["B"]).cuda() for q in probs]
        Gs = [torch.from_numpy(q["G"]).cuda() for q in probs]
        plan = tt.Plan(None, batch_T=T, batch_shapes=[q["B"].shape for q in probs])
        Xs = [torch.empty_like(b) for b in Bs]
        msf = _timed(lambda: plan.solve(Bs, Xs), steps, 1)
        plan.status()
        msb = _timed(lambda: tt.solve_backward_batched(T, Xs, Gs), steps, 1)
        # the same backward with a reusable adjoint plan (planning and
        # workspace allocation outside the timed region, as in a training loop)
        planb = tt.Plan(None, batch_T=T, batch_shapes=[q["B"].shape for q in probs], trans=True)
        dBs = [torch.empty_like(g) for g in Gs]
        dTs = [[torch.empty_like(t) for t in Tb] for Tb in T]

        def backward():
            planb.solve(Gs, dBs)
            planb.coefficient_grads(T, Xs, dBs, dTs)

        msbp = _timed(backward, steps, 1)
        planb.status()
        out["adjoint_batch64"] = {"ms_forward": msf, "ms_backward": msb, "ms_backward_plan": msbp,
                                  "forward_flops": plan.flops}
    return dict(out)


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
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--only", type=lambda v: v.split(","), default=None,
                    help="run only the other workloads whose names start with these comma-separated prefixes "
                         "(no headline solve; prints one JSON object of their results)")
    ap.add_argument("--no-graph", action="store_true",
                    help="launch every step's kernels directly instead of replaying a recorded HIP graph")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the triangular solve of one equation runs on one device).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1905_09539_amd as tt
    import tt_inputs as ti

    if args.only is not None:
        print(json.dumps({"workloads": extras(args)}), flush=True)
        return

    n = args.n
    p = ti.laplace_tri((n, n, n), seed=args.seed, bumps="every8")
    T = [torch.from_numpy(t).cuda() for t in p["T"]]
    B = torch.from_numpy(p["B"]).cuda()
    X = torch.empty_like(B)
    t0 = time.perf_counter()
    plan = tt.Plan(T, B.shape, nmin=args.nmin)
    plan_s = time.perf_counter() - t0
    flops = plan.flops
    # reference for the hardware byte counters of a profiled run: one plain
    # copy with the library's copy kernel, 8 n^3 bytes read and written
    tt.copy_device(B, X)
    torch.cuda.synchronize()

    def timed(graph):
        # a step: the whole solve (every leaf wave and every update; the
        # right-hand side is read from B, X is written); with graph, replayed
        # from the HIP graph recorded by the first warmup step on a created
        # stream
        stream = torch.cuda.Stream() if graph else torch.cuda.current_stream()
        for _ in range(args.warmup):
            plan.solve(B, X, stream=stream, graph=graph)
        plan.status()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(args.steps):
            plan.solve(B, X, stream=stream, graph=graph)
        e1.record(stream)
        torch.cuda.synchronize()
        plan.status()
        return e0.elapsed_time(e1) / args.steps

    ms_eager = timed(False)
    ms = ms_eager if args.no_graph else timed(True)
    tflops = flops / (ms * 1e-3) / 1e12
    N = n ** 3
    # accuracy of the X the timed steps wrote: ||B - sum_mu X x_mu T_mu|| / ||B||
    residual = _residual(T, X, B)

    # Per-kernel timing: the same steps again with HIP events around every
    # launch, each on the stream it runs on (leaves on the caller's stream,
    # updates on the plan's side stream), averaged over the launches.
    tot = {"leaf": [0.0, 0.0, 0.0, 0], "update": [0.0, 0.0, 0.0, 0]}
    for _ in range(args.steps):
        prof = plan.profile(B, X)
        for k in tot:
            for i, f in enumerate(["ms", "flops", "bytes", "launches"]):
                tot[k][i] += prof[k][f]
    alone = plan.profile(B, X, serial=True)  # each kernel alone, for reference
    traffic = measured_traffic()

    def roof(kind):
        # algorithmic work per launch: the update kernel's flops (2 M K P per
        # tile set); the leaf kernel's minimum bytes, 16 B per element (read
        # its right-hand side, write its solution), i.e. 16 N / launches
        t_ms, fl, by, n_l = tot[kind]
        avg_s = t_ms / n_l * 1e-3
        if kind == "update":
            ach = (fl / n_l) / avg_s / 1e12
            r = {"bound": "mfma", "achieved": ach, "peak": PEAK_FP64, "unit": "TFLOP/s", "frac": ach / PEAK_FP64,
                 "kernel": "upd_kernel", "algorithmic_per_launch": fl / n_l}
        else:
            per_launch = 16.0 * float(N) / (n_l / args.steps)
            ach = per_launch / avg_s / 1e9
            r = {"bound": "hbm", "achieved": ach, "peak": PEAK_HBM, "unit": "GB/s", "frac": ach / PEAK_HBM,
                 "kernel": "leaf_kernel", "algorithmic_per_launch": per_launch,
                 "planner_bytes_per_launch": by / n_l}
        r["traffic"] = traffic.get(r["kernel"])
        r["avg_launch_us"] = avg_s * 1e6
        r["launches"] = n_l
        return r

    dom = "leaf" if tot["leaf"][0] >= tot["update"][0] else "update"
    other = "update" if dom == "leaf" else "leaf"
    kernels = {
        "upd_kernel": {"ms_per_solve": tot["update"][0] / args.steps, "alone_ms_per_solve": alone["update"]["ms"],
                       "tflops": tot["update"][1] / (tot["update"][0] * 1e-3) / 1e12,
                       "gbs": tot["update"][2] / (tot["update"][0] * 1e-3) / 1e9},
        "leaf_kernel": {"ms_per_solve": tot["leaf"][0] / args.steps, "alone_ms_per_solve": alone["leaf"]["ms"],
                        "tflops": tot["leaf"][1] / (tot["leaf"][0] * 1e-3) / 1e12,
                        "gbs": tot["leaf"][2] / (tot["leaf"][0] * 1e-3) / 1e9},
        "serial_solve_ms": alone["solve_ms"],
    }

    del plan, X
    torch.cuda.empty_cache()
    ext = None if args.no_extras else extras(args)

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
                   "n": n, "flops": flops, "leaf_nmin": args.nmin or 16,
                   "launch": "direct" if args.no_graph else "hip_graph_replay"},
        "ms_per_step_direct_launch": ms_eager,
        "frac_of_fp64_peak": tflops / PEAK_FP64,
        "residual": residual,
        "roofline": roof(dom),
        "roofline_other": roof(other),
        "kernels": kernels,
        "plan_build_s": plan_s,
        "cpu_baseline": cpu,
        "workloads": ext,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()

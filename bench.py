#!/usr/bin/env python3
"""Throughput benchmark of the matrix-free Stokes operator on one MI355X.

Workload (default): 3D stationary Stokes, Taylor-Hood Q2/Q1 on 64^3 hex cells
of the unit cube, interior vertices perturbed by seeded uniform noise of up to
0.2h (trilinear geometry), nu = 1; FP64 operator application y = K x with x ~
U[-1, 1].  One timed step is one application of the full Stokes operator (A u
+ B p; B^T u) to a fresh vector: the step rotates over enough src/dst pairs
(> 512 MB in total) that the 256 MB Infinity Cache cannot hold them, so the
vectors come from HBM.

Prints one JSON line: value = DoFs/s of the FP64 Stokes vmult, the roofline
of the operator launch (algorithmic bytes / average launch time from HIP
events, against the 8 TB/s HBM peak), the same for k = 3, 4 and FP32, a
mixed-precision solve, and the CPU oracle timed on a bounded sample.
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

HBM_PEAK = 8.0e12  # B/s, MI355X


def algorithmic_bytes(dim, n, k, word):
    nv = (k * n + 1) ** dim
    np_ = ((k - 1) * n + 1) ** dim
    N = dim * nv + np_
    verts = (n + 1) ** dim * dim * word
    return N, 2 * N * word + verts


def time_vmult(mfs, torch, h, N, prec, steps, warmup, rotate_bytes=600e6):
    dt = torch.float64 if prec == mfs.MFS_FP64 else torch.float32
    word = 8 if prec == mfs.MFS_FP64 else 4
    pairs = max(2, int(np.ceil(rotate_bytes / (2 * N * word))))
    g = torch.Generator(device="cuda")
    g.manual_seed(1)
    srcs = [torch.rand(N, dtype=dt, device="cuda", generator=g) * 2 - 1 for _ in range(pairs)]
    dsts = [torch.empty(N, dtype=dt, device="cuda") for _ in range(pairs)]
    stream = torch.cuda.current_stream()
    for i in range(warmup):
        mfs.mfs_vmult(h, mfs.MFS_OP_STOKES, prec, 0, dsts[i % pairs], srcs[i % pairs])
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for i in range(steps):
        ev[i][0].record(stream)
        mfs.mfs_vmult(h, mfs.MFS_OP_STOKES, prec, 0, dsts[i % pairs], srcs[i % pairs])
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = np.array([a.elapsed_time(b) * 1e-3 for a, b in ev])
    del srcs, dsts
    return wall, per


def cpu_baseline_oracle(n=12, k=2):
    """The oracle's element-loop Stokes vmult (element matrices by full
    quadrature, no sum factorisation) on a bounded sample mesh, 1 thread."""
    try:
        from threadpoolctl import threadpool_limits
    except Exception:  # pragma: no cover
        threadpool_limits = None
    import inputs
    from oracle import fem

    X = inputs.structured_vertices(3, [n] * 3, noise=0.2, seed=0)
    S = fem.Space(3, [n] * 3, X, k)
    x = inputs.uniform_vector(S.n_dofs, 1)
    ctx = threadpool_limits(1) if threadpool_limits else None
    try:
        t0 = time.perf_counter()
        reps = 0
        while True:
            fem.element_loop_stokes_vmult(S, 1.0, x)
            reps += 1
            if time.perf_counter() - t0 > 10.0:
                break
        t = (time.perf_counter() - t0) / reps
    finally:
        if ctx is not None:
            ctx.__exit__(None, None, None)
    return {"value": S.n_dofs / t, "unit": "DoF/s", "cores": 1, "kind": "oracle",
            "sample": f"3D Q{k}/Q{k-1} Stokes vmult on {n}^3 cells (vertex noise 0.2h), {S.n_dofs} DoFs, "
                      f"{reps} repetitions, element loop with element matrices by full quadrature, 1 thread"}


def solve_section(mfs, torch, inputs, args):
    """3D Q2/Q1 solve on the same perturbed mesh to a 1e-8 relative residual:
    FP32 multigrid preconditioner inside FP64 FGMRES vs the plain FP64 method."""
    from paper_2603_29621_amd import serving

    n, k = args.solve_n, 2
    req = inputs.Request(0, 0.0, n, k, 1.0, 0.2, 0)
    out = {"workload": f"3D Stokes Q2/Q1 {n}^3 cells, vertex noise 0.2h, nu=1, manufactured solution, rtol 1e-8"}
    for name, prec in (("fp32_mg_fp64_fgmres", mfs.MFS_FP32), ("fp64", mfs.MFS_FP64)):
        opts = mfs.mfs_default_options(precond_precision=prec, rtol=1e-8, maxit=300)
        s = torch.cuda.Stream()
        t0 = time.perf_counter()
        h, b, x = serving._setup_request(req, opts, s)
        t1 = time.perf_counter()
        times, its, res = [], 0, 0.0
        for rep in range(2):
            x.zero_()
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            info = mfs.mfs_solve(h, b, x, opts, stream=s.cuda_stream)
            times.append(time.perf_counter() - t2)
            its, res = info.iterations, info.rel_residual
        mfs.mfs_destroy(h)
        out[name] = {"setup_s": t1 - t0, "solve_s": min(times), "solves_per_s": 1.0 / min(times),
                     "iterations": its, "rel_residual": res}
    out["speedup_mixed_vs_fp64"] = out["fp64"]["solve_s"] / out["fp32_mg_fp64_fgmres"]["solve_s"]
    return out


def serving_section(args):
    """Bounded sample of the served stream: Poisson arrivals, n in {8, 16, 32},
    k in {2, 3}; continuous batching with FP32 multigrid vs sequential FP64."""
    import inputs
    from paper_2603_29621_amd import serving

    reqs = inputs.request_stream(args.serve_requests, args.serve_rate, seed=0, sizes=(8, 16, 32), degrees=(2, 3))
    served = serving.Server(200e9).run(reqs)
    seq = serving.run_sequential(reqs)
    return {"sample": f"{args.serve_requests} requests, Poisson rate {args.serve_rate}/s, n in {{8,16,32}}, "
                      f"k in {{2,3}}, nu log-uniform [1e-2, 1], noise 0.1h, rtol 1e-8",
            "served_fp32_mg": serving.summarize(served), "sequential_fp64": serving.summarize(seq)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--k", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--prec", choices=["f64", "f32"], default="f64", help="precision of the headline run")
    ap.add_argument("--no-solve", action="store_true", help="skip the solve and served-stream measurements")
    ap.add_argument("--solve-n", type=int, default=64)
    ap.add_argument("--serve-requests", type=int, default=24)
    ap.add_argument("--serve-rate", type=float, default=8.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (single-GPU build).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import inputs
    import paper_2603_29621_amd as mfs

    mfs.lib()
    dim, n, k = 3, args.n, args.k
    X = inputs.structured_vertices(dim, [n] * dim, noise=0.2, seed=0)
    opts = mfs.mfs_default_options(mg_levels=0)

    def run(kk, prec, steps, warmup):
        h = mfs.mfs_setup(dim, [n] * dim, X, kk, 1.0, opts)
        try:
            N, bytes64 = algorithmic_bytes(dim, n, kk, 8)
            word = 8 if prec == mfs.MFS_FP64 else 4
            _, B = algorithmic_bytes(dim, n, kk, word)
            wall, per = time_vmult(mfs, torch, h, N, prec, steps, warmup)
        finally:
            mfs.mfs_destroy(h)
        avg = float(per.mean())
        return {"N": N, "wall": wall, "avg_launch_s": avg, "bytes": B, "dofs_per_s": N * steps / wall,
                "achieved_GBs": B / avg / 1e9, "frac": B / avg / HBM_PEAK}

    main_prec = mfs.MFS_FP64 if args.prec == "f64" else mfs.MFS_FP32
    main_run = run(k, main_prec, args.steps, args.warmup)
    sweep = {}
    if not args.no_sweep:
        for kk in (2, 3, 4):
            for prec, name in ((mfs.MFS_FP64, "f64"), (mfs.MFS_FP32, "f32")):
                if kk == k and prec == main_prec:
                    r = main_run
                else:
                    r = run(kk, prec, max(10, args.steps // 2), 3)
                sweep[f"Q{kk}Q{kk-1}_{name}"] = {"dofs_per_s": r["dofs_per_s"], "frac_hbm": r["frac"],
                                                  "avg_launch_us": r["avg_launch_s"] * 1e6, "N": r["N"]}
    line = {
        "metric": "Stokes vmult DoFs/s (% HBM roofline)",
        "value": main_run["dofs_per_s"],
        "unit": "DoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_run["wall"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.prec,
        "data": "synthetic",
        "config": {"workload": f"3D Stokes Taylor-Hood Q{k}/Q{k-1} vmult, {n}^3 hex cells of the unit cube, "
                               f"trilinear geometry (vertex noise 0.2h, seed 0), nu=1",
                   "n_dofs": main_run["N"], "rotating_buffers_bytes": 600e6},
        "roofline": {"bound": "hbm", "achieved": main_run["achieved_GBs"], "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                     "frac": main_run["frac"], "traffic": None,
                     "bytes_per_launch": main_run["bytes"], "avg_launch_us": main_run["avg_launch_s"] * 1e6},
        "sweep": sweep,
    }
    if not args.no_solve:
        line["solve"] = solve_section(mfs, torch, inputs, args)
        line["serving"] = serving_section(args)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_oracle()
    print(json.dumps(line))


if __name__ == "__main__":
    main()

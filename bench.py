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
FP64_PEAK = 78.6e12  # flop/s, MI355X vector
# Estimated algorithmic FP64 flops per DoF of the Q_k/Q_{k-1} vmult on trilinear
# cells with even-odd sum factorisation (k = 2, 3, 4).
FLOP_PER_DOF = {2: 318.0, 3: 243.0, 4: 217.0}
# HBM bytes per FP64 Q2/Q1 vmult on 64^3 cells measured with rocprofv3 FETCH_SIZE and
# WRITE_SIZE (scaled by 2.00 and 1.00, the factors a 256 MiB device copy gives) for the
# current cell + combine kernels; to be re-measured whenever those kernels change.
MEASURED_TRAFFIC = {(2, 64, "f64"): 308.8e6}
# Executed FP64 flops per vmult, counted with rocprofv3 (SQ_INSTS_VALU_{FMA,MUL,ADD,TRANS}_F64,
# 64 lanes per wave instruction, an FMA as 2 flops) over the same kernels: Q2/Q1 cell kernel
# 4.326 GFLOP + combine 0.019 GFLOP on 64^3 cells; Q3/Q2 cell kernel 11.996 + gather 0.091.
COUNTED_FP64_FLOP = {(2, 64): 4.345e9, (3, 64): 12.087e9}


def algorithmic_bytes(dim, n, k, word):
    nv = (k * n + 1) ** dim
    np_ = ((k - 1) * n + 1) ** dim
    N = dim * nv + np_
    verts = (n + 1) ** dim * dim * word
    return N, 2 * N * word + verts


def stream_copy_bandwidth(torch, nbytes=1 << 30, reps=10):
    """Achievable HBM bandwidth: a device-to-device copy of 1 GiB (read + write
    bytes over the event time, best of the repetitions)."""
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) * 1e-3)
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / best


def progress(msg):
    """One line per finished step on stderr (stdout carries only the JSON line)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def time_vmult(mfs, torch, h, N, prec, steps, warmup, rotate_bytes=600e6, op=None):
    op = mfs.MFS_OP_STOKES if op is None else op
    dt = torch.float64 if prec == mfs.MFS_FP64 else torch.float32
    word = 8 if prec == mfs.MFS_FP64 else 4
    pairs = max(2, int(np.ceil(rotate_bytes / (2 * N * word))))
    g = torch.Generator(device="cuda")
    g.manual_seed(1)
    srcs = [torch.rand(N, dtype=dt, device="cuda", generator=g) * 2 - 1 for _ in range(pairs)]
    dsts = [torch.empty(N, dtype=dt, device="cuda") for _ in range(pairs)]
    stream = torch.cuda.current_stream()
    for i in range(warmup):
        mfs.mfs_vmult(h, op, prec, 0, dsts[i % pairs], srcs[i % pairs])
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for i in range(steps):
        ev[i][0].record(stream)
        mfs.mfs_vmult(h, op, prec, 0, dsts[i % pairs], srcs[i % pairs])
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = np.array([a.elapsed_time(b) * 1e-3 for a, b in ev])
    del srcs, dsts
    return wall, per


def cpu_baseline_oracle(n=12, k=2, seconds=10.0):
    """The oracle's element-loop Stokes vmult (element matrices by full
    quadrature, no sum factorisation) on a bounded sample mesh, 1 thread,
    repeated for about ``seconds``."""
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
            if time.perf_counter() - t0 > seconds:
                break
        t = (time.perf_counter() - t0) / reps
    finally:
        if ctx is not None:
            ctx.__exit__(None, None, None)
    return {"value": S.n_dofs / t, "unit": "DoF/s", "cores": 1, "kind": "oracle",
            "sample": f"3D Q{k}/Q{k-1} Stokes vmult on {n}^3 cells (vertex noise 0.2h), {S.n_dofs} DoFs, "
                      f"{reps} repetitions, element loop with element matrices by full quadrature, 1 thread"}


def spacetime_section(mfs, torch, X, args):
    """Space-time Kronecker operator (G_Q (x) M + tau I_Q (x) A) of Sec. 4 on
    the headline mesh (Q2/Q1, 64^3 trilinear cells), DG(1) and DG(2) in time
    (Q = 2, 3 stages), against Q separate Stokes vmults: DoFs/s counts the Q
    stage vectors."""
    from paper_2603_29621_amd import spacetime as pst

    n, k = args.n, 2
    h = mfs.mfs_setup(3, [n] * 3, X, k, 1.0, mfs.mfs_default_options(mg_levels=0))
    out = {"workload": f"Q2/Q1 {n}^3 trilinear cells, tau = 1e-2, DG(Q-1) in time"}
    try:
        nv, np_ = mfs.mfs_n_dofs(h, 0)
        N = 3 * nv + np_
        for Q in (2, 3):
            G = pst.dg_stage_matrices(Q - 1)[0]
            for prec, name in ((mfs.MFS_FP64, "f64"), (mfs.MFS_FP32, "f32")):
                dt = torch.float64 if prec == mfs.MFS_FP64 else torch.float32
                x = torch.rand(Q * N, dtype=dt, device="cuda") * 2 - 1
                y = torch.empty_like(x)
                w = torch.empty(Q * 3 * nv, dtype=dt, device="cuda")
                stream = torch.cuda.current_stream()
                for _ in range(3):
                    mfs.mfs_st_vmult(h, G, 1e-2, prec, y, x, w)
                torch.cuda.synchronize()
                reps = max(5, args.steps // 2)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                for _ in range(reps):
                    mfs.mfs_st_vmult(h, G, 1e-2, prec, y, x, w)
                e1.record(stream)
                torch.cuda.synchronize()
                t = e0.elapsed_time(e1) * 1e-3 / reps
                out[f"Q{Q}_{name}"] = {"us": t * 1e6, "stage_dofs_per_s": Q * N / t}
                del x, y, w
        progress("space-time operator done")
    finally:
        mfs.mfs_destroy(h)
    return out


def stmg_section(mfs, torch, inputs, args):
    """hp space-time multigrid of Sec. 4 (FGMRES + one V-cycle) on the stage
    system of one slab: 2D unit square, 64^2 cells (between the 1,600 and
    6,400 cells of the paper's first two refinements of Exp. 2, which is 2D),
    vertex noise 0.1h, nu = 1e-3, tau = 1e-2, Q_k/Q_{k-1} with DG(k-1) in
    time (the pairing of Exp. 2), k = 2, 3; and 3D on 16^3 cells at k = 2; a
    consistent right-hand side b = K x_t from a seeded random x_t."""
    out = {"workload": "Taylor-Hood Q_k/Q_k-1 with DG(k-1) in time, 2D 64^2 cells (k = 2, 3) and 3D 16^3 cells "
                       "(k = 2), vertex noise 0.1h (seed 0), nu = 1e-3, tau = 1e-2, b = K x_t, FGMRES(30) to rtol "
                       "1e-8, one V-cycle per iteration"}
    cases = [(2, [64, 64], 2), (2, [64, 64], 3), (3, [16, 16, 16], 2)]
    for dim, n, k in cases:
        X = inputs.structured_vertices(dim, n, noise=0.1, seed=0)
        t0 = time.perf_counter()
        h = mfs.mfs_stmg_setup(dim, n, X, k, k - 1, 1e-3, 1e-2)
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t0
        try:
            lev = mfs.mfs_stmg_levels(h)
            N = lev[0]["length"]
            gen = torch.Generator(device="cuda").manual_seed(7)
            xt = torch.rand(N, dtype=torch.float64, device="cuda", generator=gen) * 2 - 1
            b = torch.empty_like(xt)
            mfs.mfs_stmg_vmult(h, 0, b, xt)  # Dirichlet rows of b = those of x_t
            xt_h = xt.cpu()
            y = torch.empty_like(xt)
            for _ in range(2):
                mfs.mfs_stmg_vcycle(h, y, b)
            stream = torch.cuda.current_stream()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            reps = 10
            e0.record(stream)
            for _ in range(reps):
                mfs.mfs_stmg_vcycle(h, y, b)
            e1.record(stream)
            torch.cuda.synchronize()
            vc = e0.elapsed_time(e1) * 1e-3 / reps
            b32, y32 = b.float(), torch.empty(N, dtype=torch.float32, device="cuda")
            for _ in range(2):
                mfs.mfs_stmg_vcycle(h, y32, b32, prec=mfs.MFS_FP32)
            e0.record(stream)
            for _ in range(reps):
                mfs.mfs_stmg_vcycle(h, y32, b32, prec=mfs.MFS_FP32)
            e1.record(stream)
            torch.cuda.synchronize()
            vc32 = e0.elapsed_time(e1) * 1e-3 / reps
            x32 = torch.zeros_like(xt)
            info32 = mfs.mfs_stmg_solve(h, b, x32, rtol=1e-8, maxit=400, prec=mfs.MFS_FP32)
            x = torch.zeros_like(xt)
            info = mfs.mfs_stmg_solve(h, b, x, rtol=1e-8, maxit=400)
            torch.cuda.synchronize()
            S = lev[0]
            nvel = N // S["Q"]
            # velocity error against x_t (the pressure is fixed up to a constant per stage)
            xs = x.cpu()
            nu_ = dim * int(np.prod([k * a + 1 for a in n]))
            vel = torch.cat([torch.arange(q * nvel, q * nvel + nu_) for q in range(S["Q"])])
            err = float((xs[vel] - xt_h[vel]).norm() / xt_h[vel].norm())
            err32 = float((x32.cpu()[vel] - xt_h[vel]).norm() / xt_h[vel].norm())
            out[f"{'3d_' if dim == 3 else ''}Q{k}Q{k-1}_dg{k-1}"] = {
                "n_dofs": N, "levels": [[L["n"][0], L["k"], L["Q"]] for L in lev], "setup_s": setup_s,
                "vcycle_ms": vc * 1e3, "solve_s": info.seconds, "iterations": info.iterations,
                "rel_residual": info.rel_residual, "status": info.status,
                "ms_per_iteration": info.seconds / max(1, info.iterations) * 1e3, "velocity_rel_error": err,
                "fp32_vcycle": {"vcycle_ms": vc32 * 1e3, "solve_s": info32.seconds, "iterations": info32.iterations,
                                "rel_residual": info32.rel_residual, "status": info32.status,
                                "velocity_rel_error": err32}}
        finally:
            mfs.mfs_stmg_destroy(h)
    progress("space-time multigrid done")
    return out


def oracle_checks(mfs, torch, inputs):
    """Mixed-precision solves (FP32 multigrid inside FP64 FGMRES to 1e-8, as
    served) on small meshes, each compared with the oracle's sparse direct
    solve of the same system: relative error and the oracle's FP64 residual
    of the GPU solution.  Part of the CPU-baseline leg (the only leg that runs
    the oracle)."""
    from oracle import fem, solve
    from paper_2603_29621_amd import serving

    out = []
    for i, (n, k, nu) in enumerate(((8, 2, 0.05), (4, 3, 0.4), (4, 4, 0.013), (6, 3, 1.0))):
        req = inputs.Request(i, 0.0, n, k, nu, 0.1, 7 + i)
        opts = mfs.mfs_default_options(precond_precision=mfs.MFS_FP32, rtol=1e-8, maxit=300)
        s = torch.cuda.Stream()
        h, b, x, arena = serving._setup_request(req, opts, s)
        info = mfs.mfs_solve(h, b, x, opts, stream=s.cuda_stream)
        mfs.mfs_destroy(h)
        xg = x.cpu().numpy()
        X = inputs.structured_vertices(3, [n] * 3, noise=0.1, seed=7 + i)
        S = fem.Space(3, [n] * 3, X, k)
        mats = fem.assemble_stokes(S, nu)
        f = inputs.manufactured_3d(S.geometry()[0], nu)[2]
        bo = solve.stokes_rhs(S, nu, f, np.zeros((S.Nv, 3)), mats)
        xd = solve.pressure_mean_free(S, solve.direct_solve(S, nu, bo, mats), mats["M"])
        K = fem.constrain(mats["K"], S.velocity_dirichlet_mask())
        out.append({"n": n, "k": k, "nu": nu, "n_dofs": S.n_dofs, "iterations": info.iterations,
                    "rel_error_vs_oracle": float(np.linalg.norm(xg - xd) / np.linalg.norm(xd)),
                    "oracle_rel_residual": float(np.linalg.norm(bo - K @ xg) / np.linalg.norm(bo))})
        progress(f"oracle check n={n} k={k}: error {out[-1]['rel_error_vs_oracle']:.2e}")
    return out


def solve_2d_section(mfs, torch, inputs, reps=5):
    """The small 2D case: Q2/Q1 on 16 x 16 Cartesian cells of the unit square,
    nu = 1, the manufactured solution u = curl(sin^2(pi x) sin^2(pi y)),
    p = cos(pi x) cos(pi y); FP64 block preconditioner with Chebyshev degree 3,
    FGMRES to 1e-10.  Launch-latency bound: wall time and iterations."""
    n, k, nu = [16, 16], 2, 1.0
    X = inputs.structured_vertices(2, n)
    opts = mfs.mfs_default_options(rtol=1e-10, precond_precision=mfs.MFS_FP64, cheb_degree=3)
    t0 = time.perf_counter()
    h = mfs.mfs_setup(2, n, X, k, nu, opts)
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    try:
        Nv, Np = mfs.mfs_n_dofs(h, 0)
        q = mfs.mfs_quadrature_points(h, n[0] * n[1], (k + 1) ** 2, 2)
        f = inputs.manufactured_2d(q, nu)[2]
        sp = mfs.mfs_support_points(h, k, Nv, 2)
        uex = inputs.manufactured_2d(sp, nu)[0]
        b = torch.empty(2 * Nv + Np, dtype=torch.float64, device="cuda")
        mfs.mfs_rhs(h, torch.from_numpy(np.ascontiguousarray(f)).cuda(),
                    torch.from_numpy(np.ascontiguousarray(uex.T.ravel())).cuda(), b)
        times, info = [], None
        for _ in range(reps):
            x = torch.zeros_like(b)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = mfs.mfs_solve(h, b, x, opts)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        u = x[:2 * Nv].cpu().numpy().reshape(2, Nv).T
        err = float(np.abs(u - uex).max())
    finally:
        mfs.mfs_destroy(h)
    return {"workload": "2D Stokes Q2/Q1, 16x16 Cartesian cells, nu=1, manufactured solution, FP64, Chebyshev 3, "
                        "rtol 1e-10", "n_dofs": 2 * Nv + Np, "setup_s": setup, "solve_s_median": float(np.median(times)),
            "iterations": info.iterations, "rel_residual": info.rel_residual, "u_max_error_vs_exact": err}


def solve_section(mfs, torch, inputs, args):
    """3D Q_k/Q_{k-1} solves (k = 2, 3, 4) on the perturbed mesh to a 1e-8
    relative residual: FP32 multigrid preconditioner inside FP64 FGMRES vs the
    plain FP64 method.  Each result's error is reported against a reference
    solve of the same system on the same GPU (FP64 preconditioner, FGMRES to
    1e-12)."""
    from paper_2603_29621_amd import serving

    n = args.solve_n
    out = {"workload": f"3D Stokes Q_k/Q_k-1 {n}^3 cells, vertex noise 0.2h, nu=1, manufactured solution, rtol 1e-8",
           "error_reference": "FP64-preconditioned FGMRES to rtol 1e-12 on the same GPU"}
    for k in args.solve_k:
        req = inputs.Request(0, 0.0, n, k, 1.0, 0.2, 0)
        res = {}
        ref = None
        for name, prec, rtol in (("reference", mfs.MFS_FP64, 1e-12), ("fp32_mg_fp64_fgmres", mfs.MFS_FP32, 1e-8),
                                 ("fp64", mfs.MFS_FP64, 1e-8)):
            opts = mfs.mfs_default_options(precond_precision=prec, rtol=rtol, maxit=300, graphs=args.graphs)
            s = torch.cuda.Stream()
            t0 = time.perf_counter()
            h, b, x, arena = serving._setup_request(req, opts, s)
            t1 = time.perf_counter()
            times, its, rr = [], 0, 0.0
            for rep in range(1 if name == "reference" else 2):
                x.zero_()
                torch.cuda.synchronize()
                t2 = time.perf_counter()
                info = mfs.mfs_solve(h, b, x, opts, stream=s.cuda_stream)
                times.append(time.perf_counter() - t2)
                its, rr = info.iterations, info.rel_residual
            mfs.mfs_destroy(h)
            torch.cuda.synchronize()
            if name == "reference":
                ref = x
                res["reference"] = {"iterations": its, "rel_residual": rr}
                continue
            err = float(torch.linalg.norm(x - ref) / torch.linalg.norm(ref))
            res[name] = {"setup_s": t1 - t0, "solve_s": min(times), "solves_per_s": 1.0 / min(times),
                         "iterations": its, "rel_residual": rr, "rel_error_vs_reference": err}
            del x, b
        del ref
        res["n_dofs"] = algorithmic_bytes(3, n, k, 8)[0]
        res["speedup_mixed_vs_fp64"] = res["fp64"]["solve_s"] / res["fp32_mg_fp64_fgmres"]["solve_s"]
        out[f"Q{k}Q{k - 1}"] = res
        progress(f"solve Q{k}Q{k - 1} {n}^3: {res['fp32_mg_fp64_fgmres']['solve_s']:.3f} s mixed, "
                 f"{res['fp64']['solve_s']:.3f} s FP64")
    return out


def ns_section(mfs, torch, inputs, args):
    """Stabilised Navier-Stokes (SUPG/PSPG, equal order): Jacobian vmult
    throughput on n^3 Cartesian cells for Q1Q1 and Q2Q2 (BDF2 dt = 1e-2,
    nu = 0.01, Newton linearisation about the 8-mode unit-RMS Fourier field),
    and one Newton-step linear solve J x = b (b = J y, y ~ U[-1, 1] with zero
    Dirichlet rows) with the monolithic FP32 multigrid inside FP64 FGMRES to
    1e-8, against the all-FP64 method."""
    out = {}
    dt, nu = 1e-2, 0.01
    for k in (1, 2):
        n = args.ns_n
        X = inputs.structured_vertices(3, [n] * 3)
        h = mfs.mfs_setup(3, [n] * 3, X, k, nu, mfs.mfs_default_options(pressure_offset=0, mg_levels=0))
        try:
            nv = (k * n + 1) ** 3
            N = 4 * nv
            u0 = torch.from_numpy(inputs.ns_velocity(3, [k * n + 1] * 3, seed=0)).cuda()
            mfs.mfs_set_linearization(h, u0, dt, 1)
            del u0
            for prec, name in ((mfs.MFS_FP64, "f64"), (mfs.MFS_FP32, "f32")):
                word = 8 if prec == mfs.MFS_FP64 else 4
                wall, per = time_vmult(mfs, torch, h, N, prec, max(10, args.steps // 2), 3,
                                       op=mfs.MFS_OP_NS_JACOBIAN)
                avg = float(per.mean())
                # algorithmic: src + dst + nodal u0 (FP64) + vertices; the stored
                # per-point linearisation data (16 words per Gauss point) on top
                alg = 2 * N * word + 3 * nv * 8 + (n + 1) ** 3 * 3 * word
                stored = n ** 3 * (k + 1) ** 3 * 16 * word
                out[f"Q{k}Q{k}_{name}"] = {"N": N, "dofs_per_s": N / avg, "avg_launch_us": avg * 1e6,
                                            "algorithmic_bytes": alg, "stored_qp_bytes": stored,
                                            "frac_hbm_algorithmic": alg / avg / HBM_PEAK,
                                            "frac_hbm_with_stored": (alg + stored) / avg / HBM_PEAK}
        finally:
            mfs.mfs_destroy(h)
    out["workload"] = (f"3D SUPG/PSPG Navier-Stokes Jacobian, {args.ns_n}^3 Cartesian cells, BDF2 dt={dt}, "
                       f"nu={nu}, Newton about the 8-mode Fourier field")
    # the same Jacobian on the locally refined mesh (hanging nodes)
    if args.ns_refined:
        out["refined"] = refined_ns_section(mfs, torch, inputs, args, dt, nu)
    if args.ns_jacobian_only:
        return out
    # Newton-step solve
    n, k = args.ns_solve_n, 2
    X = inputs.structured_vertices(3, [n] * 3)
    solve = {"workload": f"Q2Q2 {n}^3, J x = J y, rtol 1e-8, monolithic MG (h then p, 5 Jacobi sweeps, omega 0.5)"}
    for name, prec in (("fp32_mg_fp64_fgmres", mfs.MFS_FP32), ("fp64", mfs.MFS_FP64)):
        opts = mfs.mfs_default_options(pressure_offset=0, precond_precision=prec, rtol=1e-8, maxit=200,
                                       graphs=args.graphs)
        t0 = time.perf_counter()
        h = mfs.mfs_setup(3, [n] * 3, X, k, nu, opts)
        try:
            nv = (k * n + 1) ** 3
            N = 4 * nv
            mfs.mfs_set_linearization(h, torch.from_numpy(inputs.ns_velocity(3, [k * n + 1] * 3, seed=0)).cuda(),
                                      dt, 1)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            y = torch.from_numpy(inputs.uniform_vector(N, 3)).cuda()
            b = torch.empty_like(y)
            mfs.mfs_vmult(h, mfs.MFS_OP_NS_JACOBIAN, mfs.MFS_FP64, 0, b, y)  # Dirichlet rows of b = y
            times, info = [], None
            for rep in range(2):
                x = torch.zeros(N, dtype=torch.float64, device="cuda")
                torch.cuda.synchronize()
                t2 = time.perf_counter()
                info = mfs.mfs_solve(h, b, x, opts)
                times.append(time.perf_counter() - t2)
            solve[name] = {"setup_s": t1 - t0, "solve_s": min(times), "iterations": info.iterations,
                           "rel_residual": info.rel_residual, "status": info.status}
        finally:
            mfs.mfs_destroy(h)
    solve["speedup_mixed_vs_fp64"] = solve["fp64"]["solve_s"] / solve["fp32_mg_fp64_fgmres"]["solve_s"]
    solve["relaxation"] = relaxation_compare(mfs, torch, inputs, n, k, nu, X, args)
    out["solve"] = solve
    return out


def relaxation_compare(mfs, torch, inputs, n, k, nu, X, args):
    """The same Newton-step solve with the two relaxations of the monolithic
    multigrid: 5 damped point-Jacobi sweeps (omega 0.5) against 2 additive
    Schwarz sweeps on vertex patches (omega 1; Sec. 5, Exp. 4), FP32 multigrid
    in FP64 FGMRES, at the transient step and at dt = 1 (nearly stationary)."""
    out = {"workload": f"Q2Q2 {n}^3, J x = J y, rtol 1e-8, FP32 MG in FP64 FGMRES, set-up includes the "
                       "linearisation (and the patch inverses)"}
    N = 4 * (k * n + 1) ** 3
    u0 = torch.from_numpy(inputs.ns_velocity(3, [k * n + 1] * 3, seed=0)).cuda()
    y = torch.from_numpy(inputs.uniform_vector(N, 3)).cuda()
    for dt in (0.01, 1.0):
        row = {}
        for name, kw in (("jacobi_5", dict(relax_steps=5, relax_omega=0.5)),
                         ("asm_2", dict(relax_type=mfs.MFS_RELAX_ASM, relax_steps=2, relax_omega=1.0))):
            opts = mfs.mfs_default_options(pressure_offset=0, precond_precision=mfs.MFS_FP32, rtol=1e-8, maxit=200,
                                           graphs=args.graphs, **kw)
            h = mfs.mfs_setup(3, [n] * 3, X, k, nu, opts)
            try:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                mfs.mfs_set_linearization(h, u0, dt, 1)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                b = torch.empty_like(y)
                mfs.mfs_vmult(h, mfs.MFS_OP_NS_JACOBIAN, mfs.MFS_FP64, 0, b, y)
                times = []
                for rep in range(2):
                    x = torch.zeros(N, dtype=torch.float64, device="cuda")
                    torch.cuda.synchronize()
                    t2 = time.perf_counter()
                    info = mfs.mfs_solve(h, b, x, opts)
                    times.append(time.perf_counter() - t2)
                row[name] = {"linearization_s": t1 - t0, "solve_s": min(times), "iterations": info.iterations,
                             "rel_residual": info.rel_residual, "status": info.status}
            finally:
                mfs.mfs_destroy(h)
        out[f"dt={dt:g}"] = row
        progress(f"relaxation dt={dt:g}: Jacobi {row['jacobi_5']['iterations']} its {row['jacobi_5']['solve_s']:.3f} s, "
                 f"ASM {row['asm_2']['iterations']} its {row['asm_2']['solve_s']:.3f} s")
    return out


def refined_full_solve(mfs, torch, inputs, args, dt, nu, F):
    """The Newton-step solve J x = J y (y ~ U[-1, 1], Dirichlet rows of b = y)
    at the full refined size: n^3 base cells + 2 levels in the seeded sphere,
    Q2Q2, Newton linearisation about the Fourier field; one set-up, then FGMRES
    to 1e-8 with the FP32 monolithic multigrid and with the FP64 one."""
    n, k = args.ns_n, 2
    mesh = inputs.refined_mesh(n, seed=0, levels=2, radius=0.15)
    opts = mfs.mfs_default_options(pressure_offset=0, mg_levels=1, rtol=1e-8, maxit=200, graphs=args.graphs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = mfs.mfs_setup_refined(mesh, k, nu, opts)
    out = {"workload": f"Q2Q2 on {n}^3 base cells + 2 levels (radius 0.15, seed 0, {len(mesh['level'])} cells), "
                       "J x = J y, rtol 1e-8, GC levels then the structured h and p levels"}
    try:
        nu_, _ = mfs.mfs_n_dofs(h, 0)
        N = 4 * nu_
        pts = mfs.mfs_support_points(h, k, nu_, 3)
        u0 = np.empty((3, nu_))
        for a in range(0, nu_, 1 << 22):
            u0[:, a:a + (1 << 22)] = F(pts[a:a + (1 << 22)]).T
        del pts
        mfs.mfs_set_linearization(h, torch.from_numpy(u0.ravel()).cuda(), dt, 1)
        del u0
        torch.cuda.synchronize()
        out.update({"N": N, "levels": mfs.mfs_n_levels(h), "setup_s": time.perf_counter() - t0})
        progress(f"full refined set-up: {out['setup_s']:.1f} s, {N} DoFs")
        y = torch.from_numpy(inputs.uniform_vector(N, 3)).cuda()
        b = torch.empty_like(y)
        mfs.mfs_vmult(h, mfs.MFS_OP_NS_JACOBIAN, mfs.MFS_FP64, 0, b, y)
        del y
        for name, prec in (("fp32_mg_fp64_fgmres", mfs.MFS_FP32), ("fp64", mfs.MFS_FP64)):
            o = mfs.mfs_default_options(pressure_offset=0, mg_levels=1, precond_precision=prec, rtol=1e-8,
                                        maxit=200, graphs=args.graphs)
            x = torch.zeros(N, dtype=torch.float64, device="cuda")
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            info = mfs.mfs_solve(h, b, x, o)
            out[name] = {"solve_s": time.perf_counter() - t2, "iterations": info.iterations,
                         "rel_residual": info.rel_residual, "status": info.status}
            progress(f"full refined solve {name}: {out[name]['solve_s']:.2f} s, {info.iterations} iterations")
            del x
    finally:
        mfs.mfs_destroy(h)
    out["speedup_mixed_vs_fp64"] = out["fp64"]["solve_s"] / out["fp32_mg_fp64_fgmres"]["solve_s"]
    return out


def refined_ns_section(mfs, torch, inputs, args, dt, nu):
    """Jacobian throughput on n^3 Cartesian cells with 2 levels of local
    refinement in a seeded sphere (radius 0.15, 2:1 closure over faces and
    edges): gather through the hanging-node maps, cell kernel, transposed
    scatter."""
    n = args.ns_n
    mesh = inputs.refined_mesh(n, seed=0, levels=2, radius=0.15)
    F = inputs.fourier_field(0)
    out = {"workload": f"{n}^3 base cells + 2 levels in a sphere (centre {np.round(mesh['centre'], 3).tolist()}, "
                       f"radius 0.15, seed 0), {len(mesh['level'])} cells "
                       f"({np.bincount(mesh['level']).tolist()} per level), Newton, dt={dt}, nu={nu}"}
    for k in (1, 2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = mfs.mfs_setup_refined(mesh, k, nu)
        setup = time.perf_counter() - t0
        try:
            nu_, _ = mfs.mfs_n_dofs(h, 0)
            N = 4 * nu_
            pts = mfs.mfs_support_points(h, k, nu_, 3)
            u0 = np.empty((3, nu_))
            for a in range(0, nu_, 1 << 22):
                u0[:, a:a + (1 << 22)] = F(pts[a:a + (1 << 22)]).T
            del pts
            mfs.mfs_set_linearization(h, torch.from_numpy(u0.ravel()).cuda(), dt, 1)
            del u0
            res = {"N": N, "setup_s": setup}
            for prec, name in ((mfs.MFS_FP64, "f64"), (mfs.MFS_FP32, "f32")):
                _, per = time_vmult(mfs, torch, h, N, prec, max(10, args.steps // 2), 3, op=mfs.MFS_OP_NS_JACOBIAN)
                avg = float(per.mean())
                res[name] = {"dofs_per_s": N / avg, "avg_launch_us": avg * 1e6}
            out[f"Q{k}Q{k}"] = res
            progress(f"refined Q{k}Q{k} Jacobian: set-up {setup:.1f} s, {res['f64']['avg_launch_us']:.0f} us FP64")
        finally:
            mfs.mfs_destroy(h)
    if args.ns_jacobian_only:
        return out
    # load balance of the two multigrid hierarchies of this mesh for a Morton
    # partition over 12 processes (the paper's 12 cores), host-side
    t0 = time.perf_counter()
    out["partition_metrics_p12"] = mfs.mfs_refined_mg_metrics(mesh, 12)
    progress(f"partition metrics: {time.perf_counter() - t0:.1f} s, {out['partition_metrics_p12']}")
    if args.ns_full_solve:
        out["solve_full"] = refined_full_solve(mfs, torch, inputs, args, dt, nu, F)
    # Newton-step solve on the refined mesh of the solve size: monolithic
    # multigrid (global coarsening to the base mesh, then h and p)
    n, k = args.ns_solve_n, 2
    mesh = inputs.refined_mesh(n, seed=0, levels=2, radius=0.15)
    solve = {"workload": f"Q2Q2 on {n}^3 base cells + 2 levels (radius 0.15, seed 0, {len(mesh['level'])} cells), "
                         "J x = J y, rtol 1e-8, GC levels then the structured h and p levels, 5 Jacobi sweeps, "
                         "omega 0.5"}
    for name, prec in (("fp32_mg_fp64_fgmres", mfs.MFS_FP32), ("fp64", mfs.MFS_FP64)):
        opts = mfs.mfs_default_options(pressure_offset=0, mg_levels=1, precond_precision=prec, rtol=1e-8,
                                       maxit=200, graphs=args.graphs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = mfs.mfs_setup_refined(mesh, k, nu, opts)
        try:
            nu_, _ = mfs.mfs_n_dofs(h, 0)
            N = 4 * nu_
            u0 = F(mfs.mfs_support_points(h, k, nu_, 3)).T.ravel()
            mfs.mfs_set_linearization(h, torch.from_numpy(u0).cuda(), dt, 1)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            y = torch.from_numpy(inputs.uniform_vector(N, 3)).cuda()
            b = torch.empty_like(y)
            mfs.mfs_vmult(h, mfs.MFS_OP_NS_JACOBIAN, mfs.MFS_FP64, 0, b, y)  # Dirichlet rows of b = y
            times, info = [], None
            for rep in range(2):
                x = torch.zeros(N, dtype=torch.float64, device="cuda")
                torch.cuda.synchronize()
                t2 = time.perf_counter()
                info = mfs.mfs_solve(h, b, x, opts)
                times.append(time.perf_counter() - t2)
            solve[name] = {"N": N, "levels": mfs.mfs_n_levels(h), "setup_s": t1 - t0, "solve_s": min(times),
                           "iterations": info.iterations, "rel_residual": info.rel_residual, "status": info.status}
            progress(f"refined solve {name}: set-up {t1 - t0:.1f} s, solve {min(times):.3f} s")
        finally:
            mfs.mfs_destroy(h)
    solve["speedup_mixed_vs_fp64"] = solve["fp64"]["solve_s"] / solve["fp32_mg_fp64_fgmres"]["solve_s"]
    out["solve"] = solve
    return out


def bdf2_section(mfs, torch, inputs, args):
    """Three BDF2 steps of the stabilised Navier-Stokes equations (SUPG/PSPG,
    Q1Q1 and Q2Q2, Re = 100: nu = 0.01 with the unit-RMS 8-mode Fourier field
    as initial velocity, dt = 1e-2, zero velocity on the boundary) on n^3
    base cells with 2 levels of local refinement in a sphere, by Newton's
    method with FGMRES and one monolithic V-cycle (global coarsening, then h
    and p) per iteration: FP32 multigrid against FP64 multigrid, Newton to
    1e-8, corrections to 1e-6."""
    n, dt, nu = args.ns_solve_n, 1e-2, 0.01
    mesh = inputs.refined_mesh(n, seed=0, levels=2, radius=0.15)
    F = inputs.fourier_field(0)
    out = {"workload": f"{n}^3 base cells + 2 levels (radius 0.15, seed 0, {len(mesh['level'])} cells), BDF2 "
                       f"dt={dt}, nu={nu}, 3 steps from the Fourier field, no-slip walls, Newton rtol 1e-8, "
                       "FGMRES rtol 1e-6 per correction"}
    for k in (1, 2):
        states = {}
        for name, prec in (("fp32_mg", mfs.MFS_FP32), ("fp64_mg", mfs.MFS_FP64)):
            opts = mfs.mfs_default_options(pressure_offset=0, mg_levels=1, precond_precision=prec,
                                           graphs=args.graphs)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            h = mfs.mfs_setup_refined(mesh, k, nu, opts)
            setup = time.perf_counter() - t0
            try:
                nu_, _ = mfs.mfs_n_dofs(h, 0)
                pts = mfs.mfs_support_points(h, k, nu_, 3)
                wall = torch.from_numpy(np.any((pts == 0.0) | (pts == 1.0), axis=1)).cuda()
                un = torch.from_numpy(F(pts).T.ravel().copy()).cuda()
                unm1 = un.clone()
                p = torch.zeros(nu_, dtype=torch.float64, device="cuda")
                nopt = mfs.mfs_default_newton_options(precond_precision=prec)
                steps = []
                for step in range(3):
                    x = torch.cat([un, p])
                    for c in range(3):
                        x[c * nu_:(c + 1) * nu_][wall] = 0.0
                    info = mfs.mfs_ns_bdf2_step(h, un, unm1, x, dt, nopt)
                    steps.append({"newton_iterations": info.newton_iterations,
                                  "fgmres_iterations": info.linear_iterations, "res0": info.res0, "res": info.res,
                                  "status": info.status, "seconds": info.seconds})
                    unm1, un, p = un, x[:3 * nu_].clone(), x[3 * nu_:].clone()
                states[name] = x
                out[f"Q{k}Q{k}_{name}"] = {"N": 4 * nu_, "setup_s": setup, "steps": steps,
                                           "seconds_per_step": float(np.mean([v["seconds"] for v in steps]))}
                progress(f"BDF2 Q{k}Q{k} {name}: {[v['newton_iterations'] for v in steps]} Newton, "
                         f"{[v['fgmres_iterations'] for v in steps]} FGMRES, "
                         f"{out[f'Q{k}Q{k}_{name}']['seconds_per_step']:.2f} s per step")
            finally:
                mfs.mfs_destroy(h)
        a, b = states["fp32_mg"], states["fp64_mg"]
        out[f"Q{k}Q{k}_rel_diff_fp32_vs_fp64_mg"] = float(torch.linalg.norm(a - b) / torch.linalg.norm(b))
        out[f"Q{k}Q{k}_speedup_fp32_mg"] = (out[f"Q{k}Q{k}_fp64_mg"]["seconds_per_step"]
                                           / out[f"Q{k}Q{k}_fp32_mg"]["seconds_per_step"])
        del states, a, b
    return out


def hp_section(mfs, torch, inputs, args):
    """hp-adaptive Stokes (Sec. 3, minimum rule): velocity degree drawn per
    4^3-cell block from {2..6} (seed 0), pressure k-1, n^3 cells, vertex noise
    0.1h, nu = 1.  Stokes vmult throughput in FP64/FP32, and a solve
    K x = K y (y ~ U[-1, 1], zero Dirichlet rows) to 1e-8 with the FP32
    multigrid (hp p-levels to k = 2, then the structured h-levels) inside FP64
    FGMRES, against the all-FP64 method."""
    n = args.hp_n
    deg = inputs.block_degrees([n] * 3, seed=0, block=4, lo=2, hi=6)
    X = inputs.structured_vertices(3, [n] * 3, noise=0.1, seed=0)
    out = {"workload": f"hp Stokes {n}^3 cells, k per 4^3 block uniform in 2..6 (seed 0), pressure k-1, "
                       f"vertex noise 0.1h, nu=1",
           "degree_histogram": {int(k): int((deg == k).sum()) for k in range(2, 7)}}
    runs = (("fp32_mg_fp64_fgmres", mfs.MFS_FP32), ("fp64", mfs.MFS_FP64))
    for name, prec in (runs[1:] if args.hp_vmult_only else runs):
        opts = mfs.mfs_default_options(precond_precision=prec, rtol=1e-8, maxit=300, graphs=args.graphs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = mfs.mfs_setup_hp([n] * 3, X, deg, 1.0, opts)
        torch.cuda.synchronize()
        setup = time.perf_counter() - t0
        try:
            nu_, np_ = mfs.mfs_n_dofs(h, 0)
            N = 3 * nu_ + np_
            out["n_dofs"] = N
            if name == "fp64":
                for p, pname in ((mfs.MFS_FP64, "f64"), (mfs.MFS_FP32, "f32")):
                    _, per = time_vmult(mfs, torch, h, N, p, max(10, args.steps // 2), 3)
                    out[f"vmult_{pname}"] = {"dofs_per_s": N / float(per.mean()),
                                             "avg_launch_us": float(per.mean()) * 1e6}
                if args.hp_vmult_only:
                    return out
            y = torch.from_numpy(inputs.uniform_vector(N, 3)).cuda()
            b = torch.empty_like(y)
            mfs.mfs_vmult(h, mfs.MFS_OP_STOKES, mfs.MFS_FP64, 0, b, y)  # Dirichlet rows of b carry y
            times, info = [], None
            for rep in range(2):
                x = torch.zeros(N, dtype=torch.float64, device="cuda")
                torch.cuda.synchronize()
                t2 = time.perf_counter()
                info = mfs.mfs_solve(h, b, x, opts)
                times.append(time.perf_counter() - t2)
            out[name] = {"setup_s": setup, "solve_s": min(times), "iterations": info.iterations,
                         "rel_residual": info.rel_residual, "status": info.status}
        finally:
            mfs.mfs_destroy(h)
    out["speedup_mixed_vs_fp64"] = out["fp64"]["solve_s"] / out["fp32_mg_fp64_fgmres"]["solve_s"]
    return out


def serving_section(args):
    """The served stream: requests with n in {8, 16, 32, 64}, k in {2, 3, 4},
    nu log-uniform in [1e-2, 1], vertex noise 0.1h, rtol 1e-8.

    1. The plain method, sequential FP64 (FP64 preconditioner), runs the
       requests back to back: its per-request service time (set-up, solve,
       release) and its capacity (solves/s).
    2. Arrivals: Poisson at rate lambda = that capacity (offered load 1.0).
       The served loop (continuous batching, FP32 multigrid inside FP64
       FGMRES) replays the stream in real time.
    3. The sequential method's latencies under the same arrivals follow from
       its measured service times (one request at a time, in arrival order:
       completion_i = max(arrival_i, completion_i-1) + service_i).
    Every served solution is compared with the sequential FP64 solution of the
    same request (both kept on the device)."""
    import dataclasses

    import torch

    import inputs
    from paper_2603_29621_amd import serving

    nreq = args.serve_requests
    sizes, degrees = (8, 16, 32, 64), (2, 3, 4)
    unit = inputs.request_stream(nreq, 1.0, seed=0, sizes=sizes, degrees=degrees)
    seq_sol = {}

    def keep_seq(r):
        seq_sol[r.rid] = r.x
        if len(seq_sol) % 64 == 0:
            progress(f"sequential FP64: {len(seq_sol)}/{nreq}")

    back = [dataclasses.replace(r, arrival=0.0) for r in unit]
    seq = serving.run_sequential(back, realtime=False, keep_solutions=True, on_result=keep_seq)
    seq_span = max(r.completed for r in seq)
    rate = nreq / seq_span
    torch.cuda.empty_cache()
    reqs = inputs.request_stream(nreq, rate, seed=0, sizes=sizes, degrees=degrees)
    service = {r.rid: r.completed - r.admitted for r in seq}
    # FIFO replay of the sequential service times against the arrivals
    t = 0.0
    seq_rt = []
    for q in sorted(reqs, key=lambda q: q.arrival):
        start = max(q.arrival, t)
        t = start + service[q.rid]
        r = next(x for x in seq if x.rid == q.rid)
        seq_rt.append(dataclasses.replace(r, arrival=q.arrival, admitted=start, completed=t, x=None))
    diffs = []

    def compare(r):
        ref = seq_sol.pop(r.rid)
        diffs.append(float(torch.linalg.norm(r.x - ref) / torch.linalg.norm(ref)))
        r.x = None
        if len(diffs) % 64 == 0:
            progress(f"served: {len(diffs)}/{nreq}")

    served = serving.Server(args.serve_budget_gb * 1e9, graphs=args.graphs, keep_solutions=True).run(
        reqs, on_result=compare)
    seq_sol.clear()
    torch.cuda.empty_cache()
    d = np.array(diffs)
    # time with at least one request in service (union of admitted..completed):
    # solves per busy second bound the served loop's capacity from below
    iv = sorted((r.admitted, r.completed) for r in served)
    busy, cs, ce = 0.0, iv[0][0], iv[0][1]
    for a, b in iv[1:]:
        if a > ce:
            busy += ce - cs
            cs, ce = a, b
        else:
            ce = max(ce, b)
    busy += ce - cs
    return {"sample": f"{nreq} requests, Poisson arrivals at the sequential FP64 capacity ({rate:.3f}/s, offered "
                      f"load 1.0), n in {{8,16,32,64}}, k in {{2,3,4}}, nu log-uniform [1e-2, 1], noise 0.1h, "
                      f"rtol 1e-8",
            "served_fp32_mg": serving.summarize(served),
            "sequential_fp64": serving.summarize(seq_rt),
            "sequential_fp64_capacity_solves_per_s": rate,
            "served_fp32_mg_busy_s": busy,
            "served_fp32_mg_solves_per_busy_s": nreq / busy,
            "served_vs_sequential_fp64_rel_diff": {"max": float(d.max()), "p50": float(np.median(d))},
            "sequential_latency_note": "sequential latencies: measured back-to-back service times replayed "
                                       "against the same arrival times (FIFO, one request at a time)"}


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
    ap.add_argument("--solve-k", type=lambda v: [int(a) for a in v.split(",")], default=[2, 3, 4])
    ap.add_argument("--serve-requests", type=int, default=512)
    ap.add_argument("--serve-budget-gb", type=float, default=150.0)
    ap.add_argument("--no-graphs", dest="graphs", action="store_const", const=0, default=1,
                    help="launch the FP32 preconditioner kernel by kernel instead of replaying its recorded graph")
    ap.add_argument("--no-ns", action="store_true", help="skip the Navier-Stokes measurements")
    ap.add_argument("--no-hp", action="store_true", help="skip the hp measurements")
    ap.add_argument("--no-stmg", action="store_true", help="skip the space-time multigrid measurements")
    ap.add_argument("--hp-n", type=int, default=32)
    ap.add_argument("--ns-n", type=int, default=128)
    ap.add_argument("--no-ns-refined", dest="ns_refined", action="store_false",
                    help="skip the Jacobian on the locally refined mesh")
    ap.add_argument("--ns-solve-n", type=int, default=32)
    ap.add_argument("--no-ns-full-solve", dest="ns_full_solve", action="store_false",
                    help="skip the Newton-step solve at the full refined size")
    ap.add_argument("--ns-jacobian-only", action="store_true",
                    help="Navier-Stokes: Jacobian throughput only (no Newton-step solves, no BDF2 steps)")
    ap.add_argument("--hp-vmult-only", action="store_true", help="hp: vmult throughput only (no solves)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one 256 MiB device copy first (reference kernel for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (single-GPU build).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import inputs
    import paper_2603_29621_amd as mfs

    mfs.lib()
    if args.copy_calibration:
        a = torch.ones(2 ** 25, dtype=torch.float64, device="cuda")
        torch.empty_like(a).copy_(a)
        torch.cuda.synchronize()
        del a
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
    copy_bw = stream_copy_bandwidth(torch)
    progress(f"headline vmult: {main_run['avg_launch_s'] * 1e6:.1f} us")
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
        progress("sweep done")
        line_spacetime = spacetime_section(mfs, torch, X, args)
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
                     "frac": main_run["frac"], "traffic": MEASURED_TRAFFIC.get((k, n, args.prec)),
                     "bytes_per_launch": main_run["bytes"], "avg_launch_us": main_run["avg_launch_s"] * 1e6,
                     "stream_copy_GBs": copy_bw / 1e9, "frac_of_stream_copy": main_run["bytes"] /
                     main_run["avg_launch_s"] / copy_bw},
        "sweep": sweep,
    }
    if not args.no_sweep:
        line["spacetime"] = line_spacetime
    if not args.no_stmg:
        line["stmg"] = stmg_section(mfs, torch, inputs, args)
    if args.prec == "f64" and k in FLOP_PER_DOF:
        # executed flops (counter-derived) where counted for this size, beside the model
        model = FLOP_PER_DOF[k] * main_run["N"]
        counted = COUNTED_FP64_FLOP.get((k, n))
        fl = (counted if counted else model) / main_run["avg_launch_s"]
        line["roofline_alu"] = {"bound": "alu", "achieved": fl / 1e12, "peak": FP64_PEAK / 1e12, "unit": "TFLOP/s",
                                "frac": fl / FP64_PEAK, "flops": "counted" if counted else "model",
                                "counted_flop_per_dof": counted / main_run["N"] if counted else None,
                                "model_flop_per_dof": FLOP_PER_DOF[k],
                                "model_frac": model / main_run["avg_launch_s"] / FP64_PEAK}
    if not args.no_ns:
        line["navier_stokes"] = ns_section(mfs, torch, inputs, args)
        progress("navier_stokes done")
        if not args.ns_jacobian_only:
            line["navier_stokes"]["bdf2"] = bdf2_section(mfs, torch, inputs, args)
            progress("BDF2 done")
    if not args.no_hp:
        line["hp"] = hp_section(mfs, torch, inputs, args)
        progress("hp done")
    if not args.no_solve:
        line["solve"] = solve_section(mfs, torch, inputs, args)
        line["solve_2d"] = solve_2d_section(mfs, torch, inputs)
        progress("solve done")
        line["serving"] = serving_section(args)
        progress("serving done")
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_oracle()
        # the higher degrees of the sweep, on smaller sample meshes
        line["cpu_baseline"]["by_degree"] = {f"Q{k}Q{k - 1}": cpu_baseline_oracle(n, k, seconds=5.0)
                                             for n, k in ((8, 3), (6, 4))}
        progress("oracle vmult timed")
        line["cpu_baseline"]["mixed_precision_vs_oracle"] = oracle_checks(mfs, torch, inputs)
        progress("cpu baseline done")
    print(json.dumps(line))


if __name__ == "__main__":
    main()

"""Continuous-batching request loop for stationary Stokes solves.

Requests (mesh size, degree, viscosity, mesh seed) arrive over time.  The
loop admits a request when its planned device footprint fits the memory
budget (no head-of-line blocking: a request that does not fit yet is passed
over for younger ones that do, until it has waited ``max_bypass_s``; then
admission stops until it fits).  Each admitted request gets its own HIP
stream and problem handle, whose device memory is one arena from torch's
allocator (``mfs_setup_arena``; releasing it does not wait for the device);
setup (mesh upload, multigrid hierarchy, right-hand side) runs on worker
threads, and the main thread calls ``mfs_batch_step`` over all active
solves: every solve whose previous iteration has finished gets its next
FGMRES iteration, and the system operator applications of the Q2/Q1 solves
that step together share one grouped launch (the call never blocks).
Kernels of different requests
therefore overlap on the device, and a request's Krylov state, mesh and
hierarchy stay resident in HBM until it completes.

Latency = completion time - arrival time on the host clock.  The baseline
runs the same requests one after another in arrival order with the plain
FP64 method (FP64 preconditioner).
"""
from __future__ import annotations

import sys
import threading
import time
from collections import deque
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass

import numpy as np

import paper_2603_29621_amd as mfs


@dataclass
class Result:
    rid: int
    n: int
    k: int
    nu: float
    arrival: float
    admitted: float
    completed: float
    iterations: int
    rel_residual: float
    status: int
    x: object = None  # device solution (kept only when requested)

    @property
    def latency(self):
        return self.completed - self.arrival


def _options(precond, rtol, maxit, graphs=1):
    return mfs.mfs_default_options(precond_precision=precond, rtol=rtol, maxit=maxit, graphs=graphs)


def request_footprint(req, opts) -> int:
    """Device bytes of one request: library arena + b, x and the transient
    quadrature-point / forcing arrays of its right-hand side."""
    n = [req.n] * 3
    arena = mfs.mfs_footprint(3, n, _dummy_vertices(req.n), req.k, opts)  # depends on sizes only
    nv = (req.k * req.n + 1) ** 3
    np_ = ((req.k - 1) * req.n + 1) ** 3
    N = 3 * nv + np_
    nq = req.n ** 3 * (req.k + 1) ** 3
    return arena + 2 * N * 8 + 2 * nq * 3 * 8 + 3 * nv * 8


_dummy_cache = {}


def _dummy_vertices(n):
    if n not in _dummy_cache:
        import inputs

        _dummy_cache[n] = inputs.structured_vertices(3, [n] * 3)
    return _dummy_cache[n]


class _Active:
    __slots__ = ("req", "h", "stream", "b", "x", "fp", "admitted", "arena")


def _setup_request(req, opts, stream):
    """Build the problem in an arena from torch's allocator and its right-hand
    side on `stream` (worker thread).  Returns (handle, b, x, arena); the arena
    must stay alive until the handle is destroyed.  Releasing it returns the
    block to torch's cache, which does not wait for the device."""
    import torch

    import inputs

    X = inputs.structured_vertices(3, [req.n] * 3, noise=req.noise, seed=req.mesh_seed)
    fp = mfs.mfs_footprint(3, [req.n] * 3, X, req.k, opts)
    with torch.cuda.stream(stream):
        arena = torch.empty(fp, dtype=torch.uint8, device="cuda")
    h = mfs.mfs_setup_arena(3, [req.n] * 3, X, req.k, req.nu, arena, opts, stream=stream.cuda_stream)
    nv, np_ = mfs.mfs_n_dofs(h, 0)
    N = 3 * nv + np_
    nq = req.n ** 3 * (req.k + 1) ** 3
    with torch.cuda.stream(stream):
        q = torch.empty((nq, 3), dtype=torch.float64, device="cuda")
        mfs.mfs_quadrature_points_device(h, q, stream=stream.cuda_stream)
        f = inputs.manufactured_forcing_3d_torch(q, req.nu).contiguous()
        del q
        uD = torch.zeros(3 * nv, dtype=torch.float64, device="cuda")  # u = 0 on the boundary
        b = torch.empty(N, dtype=torch.float64, device="cuda")
        mfs.mfs_rhs(h, f, uD, b, stream=stream.cuda_stream)
        x = torch.zeros(N, dtype=torch.float64, device="cuda")
        stream.synchronize()
        del f, uD
    return h, b, x, arena


class Server:
    def __init__(self, budget_bytes: float, max_active: int = 32, precond=mfs.MFS_FP32, rtol: float = 1e-8,
                 maxit: int = 300, setup_workers: int = 2, max_bypass_s: float = 2.0, keep_solutions=False,
                 graphs: int = 1, batch: bool = True):
        self.budget = float(budget_bytes)
        self.max_active = max_active
        self.opts = _options(precond, rtol, maxit, graphs)
        self.setup_workers = setup_workers
        self.max_bypass_s = max_bypass_s
        self.keep = keep_solutions
        self.batch = batch  # advance the active solves with mfs_batch_step (grouped operator launches)

    def run(self, requests, realtime: bool = True, on_result=None):
        """Serve the requests; on_result(result), if given, is called as each one
        completes."""
        import torch

        pending = deque(sorted(requests, key=lambda r: r.arrival))
        waiting: list = []
        active: dict = {}
        setups: dict = {}
        results = []
        used = 0.0
        self.peak_used = 0.0
        fps = {}
        streams = []
        lock = threading.Lock()
        pool = ThreadPoolExecutor(self.setup_workers)
        group_stream = torch.cuda.Stream()
        t0 = time.perf_counter()
        try:
            while pending or waiting or active or setups:
                now = time.perf_counter() - t0
                while pending and (not realtime or pending[0].arrival <= now):
                    waiting.append(pending.popleft())
                # admission by footprint, FIFO with bounded bypass
                i = 0
                while i < len(waiting) and len(active) + len(setups) < self.max_active:
                    r = waiting[i]
                    fp = fps.get(r.rid) or request_footprint(r, self.opts)
                    fps[r.rid] = fp
                    if fp > self.budget:
                        raise ValueError(f"request {r.rid} needs {fp / 1e9:.1f} GB > budget")
                    if used + fp <= self.budget:
                        used += fp
                        self.peak_used = max(self.peak_used, used)
                        waiting.pop(i)
                        s = streams.pop() if streams else torch.cuda.Stream()
                        setups[r.rid] = (r, s, now, pool.submit(_setup_request, r, self.opts, s))
                        continue
                    if i == 0 and now - r.arrival > self.max_bypass_s:
                        break  # the oldest has waited long enough: stop bypassing it
                    i += 1
                progressed = False
                for rid in list(setups):
                    r, s, adm, fut = setups[rid]
                    if fut.done():
                        h, b, x, arena = fut.result()
                        mfs.mfs_solve_begin(h, b, x, self.opts, stream=s.cuda_stream)
                        a = _Active()
                        a.req, a.h, a.stream, a.b, a.x, a.fp, a.admitted = r, h, s, b, x, fps[rid], adm
                        a.arena = arena
                        active[rid] = a
                        del setups[rid]
                        progressed = True
                rids = list(active)
                if self.batch:
                    steps = mfs.mfs_batch_step([active[rid].h for rid in rids], stream=group_stream.cuda_stream)
                else:
                    steps = [mfs.mfs_solve_advance(active[rid].h) for rid in rids]
                for rid, (done, info) in zip(rids, steps):
                    a = active[rid]
                    if done:
                        t = time.perf_counter() - t0
                        res = Result(rid, a.req.n, a.req.k, a.req.nu, a.req.arrival if realtime else 0.0, a.admitted,
                                     t, info.iterations, info.rel_residual, info.status,
                                     a.x if self.keep else None)
                        results.append(res)
                        if on_result is not None:
                            on_result(res)
                        mfs.mfs_destroy(a.h)
                        a.arena = None
                        with lock:
                            used -= a.fp
                        streams.append(a.stream)
                        del active[rid]
                        progressed = True
                if not progressed:
                    time.sleep(20e-6)
        finally:
            pool.shutdown(wait=True)
        return sorted(results, key=lambda r: r.rid)


def run_sequential(requests, precond=mfs.MFS_FP64, rtol=1e-8, maxit=300, realtime=True, keep_solutions=False,
                   on_result=None):
    """Plain baseline: one solve at a time in arrival order."""
    import torch

    opts = _options(precond, rtol, maxit)
    out = []
    s = torch.cuda.Stream()
    t0 = time.perf_counter()
    for r in sorted(requests, key=lambda r: r.arrival):
        if realtime:
            wait = r.arrival - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
        adm = time.perf_counter() - t0
        h, b, x, arena = _setup_request(r, opts, s)
        info = mfs.mfs_solve(h, b, x, opts, stream=s.cuda_stream)
        t = time.perf_counter() - t0
        out.append(Result(r.rid, r.n, r.k, r.nu, r.arrival if realtime else 0.0, adm, t, info.iterations,
                          info.rel_residual, info.status, x if keep_solutions else None))
        if on_result is not None:
            on_result(out[-1])
        mfs.mfs_destroy(h)
        del arena
    return out


def summarize(results, makespan=None):
    lat = np.array([r.latency for r in results])
    span = makespan if makespan is not None else max(r.completed for r in results)
    return {"solves": len(results), "solves_per_s": len(results) / span, "makespan_s": span,
            "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
            "max_rel_residual": float(max(r.rel_residual for r in results)),
            "all_converged": bool(all(r.status == 0 for r in results)),
            "mean_iterations": float(np.mean([r.iterations for r in results]))}


if __name__ == "__main__":
    import argparse
    import json

    import torch

    import inputs

    ap = argparse.ArgumentParser(description="served stream of stationary Stokes solves")
    ap.add_argument("--requests", type=int, default=512)
    ap.add_argument("--rate", type=float, default=4.0, help="Poisson arrival rate [1/s]")
    ap.add_argument("--sizes", default="8,16,32,64")
    ap.add_argument("--degrees", default="2,3,4")
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--baseline", action="store_true", help="also run the sequential FP64 baseline")
    args = ap.parse_args()
    reqs = inputs.request_stream(args.requests, args.rate, seed=0,
                                 sizes=tuple(int(v) for v in args.sizes.split(",")),
                                 degrees=tuple(int(v) for v in args.degrees.split(",")))
    mfs.lib()
    torch.cuda.init()

    def reporter(name):
        done = []

        def report(res):
            done.append(res)
            if len(done) % 32 == 0 or len(done) == len(reqs):
                print(f"[{name}] {len(done)}/{len(reqs)} solved, t = {res.completed:.1f} s", file=sys.stderr,
                      flush=True)
        return report

    served = Server(args.budget_gb * 1e9).run(reqs, on_result=reporter("served"))
    out = {"sample": f"{args.requests} requests, Poisson rate {args.rate}/s, n in {{{args.sizes}}}, "
                     f"k in {{{args.degrees}}}, nu log-uniform [1e-2, 1], noise 0.1h, rtol 1e-8",
           "served_fp32_mg": summarize(served)}
    if args.baseline:
        out["sequential_fp64"] = summarize(run_sequential(reqs, on_result=reporter("sequential")))
    print(json.dumps(out))

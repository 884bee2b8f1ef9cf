"""Serving loop: each result is bit for bit the same alone and in the mix
(every 3D Stokes kernel accumulates in a fixed order: brick kernels with a
fixed-order face combine, node gathers, or atomics launched one cell colour
at a time), admission never exceeds the memory budget, every request
converges, and every served result agrees with the oracle's direct solve of
the same system within the bound its residual and the system's smallest
eigenvalue give."""
import numpy as np
import pytest
import torch

import inputs
import paper_2603_29621_amd as mfs
from oracle import fem, solve
from bounds import bordered_error_bound
from paper_2603_29621_amd import serving

pytestmark = pytest.mark.gpu


def _requests():
    reqs = inputs.request_stream(6, rate=1000.0, seed=3, sizes=(4, 8), degrees=(2, 3), noise=0.1)
    for r in reqs:
        r.arrival = 0.0
    return reqs


def test_alone_equals_mix_and_admission():
    reqs = _requests()
    opts = mfs.mfs_default_options()
    fps = [serving.request_footprint(r, opts) for r in reqs]
    budget = sum(sorted(fps)[-3:]) * 1.01  # at most about three requests at a time
    srv = serving.Server(budget, max_active=6, keep_solutions=True)
    mix = srv.run(reqs, realtime=False)
    assert srv.peak_used <= budget
    assert all(r.status == 0 and r.rel_residual <= 1e-8 for r in mix)
    for r in reqs:
        alone = serving.Server(budget, max_active=1, keep_solutions=True).run([r], realtime=False)[0]
        m = next(x for x in mix if x.rid == r.rid)
        assert alone.iterations == m.iterations
        assert torch.equal(alone.x, m.x), (r.rid, r.n, r.k)


@pytest.mark.parametrize("cases", [[(8, 2, 0.05), (4, 3, 0.4), (4, 4, 0.013)]])
def test_served_results_match_oracle(cases):
    """Requests of degrees 2, 3, 4 served together (FP32 multigrid inside
    FP64 FGMRES to 1e-8): each solution is compared with the oracle's sparse
    direct solve of the same system."""
    reqs = [inputs.Request(i, 0.0, n, k, nu, 0.1, 7 + i) for i, (n, k, nu) in enumerate(cases)]
    srv = serving.Server(64e9, max_active=4, keep_solutions=True)
    res = srv.run(reqs, realtime=False)
    for r, q in zip(res, reqs):
        assert r.status == 0 and r.rel_residual <= 1e-8
        X = inputs.structured_vertices(3, [q.n] * 3, noise=q.noise, seed=q.mesh_seed)
        S = fem.Space(3, [q.n] * 3, X, q.k)
        mats = fem.assemble_stokes(S, q.nu)
        f = inputs.manufactured_3d(S.geometry()[0], q.nu)[2]
        b = solve.stokes_rhs(S, q.nu, f, np.zeros((S.Nv, 3)), mats)
        xd = solve.pressure_mean_free(S, solve.direct_solve(S, q.nu, b, mats), mats["M"])
        x = r.x.cpu().numpy()
        K = fem.constrain(mats["K"], S.velocity_dirichlet_mask())
        # the oracle's FP64 residual of the served solution
        assert np.linalg.norm(b - K @ x) <= 1.05e-8 * np.linalg.norm(b)
        bound, lam = bordered_error_bound(S, q.nu, b, x, mats)
        err = np.linalg.norm(x - xd)
        print(f"served n={q.n} k={q.k} nu={q.nu}: ||x - x_oracle|| / ||x_oracle|| = "
              f"{err / np.linalg.norm(xd):.2e}, bound {bound / np.linalg.norm(xd):.2e} (|lambda|_min {lam:.2e})")
        assert err <= 1.5 * bound + 1e-12 * np.linalg.norm(xd)


def test_sequential_fp64_baseline_converges():
    reqs = _requests()[:3]
    res = serving.run_sequential(reqs, realtime=False)
    assert all(r.status == 0 and r.rel_residual <= 1e-8 for r in res)
    s = serving.summarize(res)
    assert s["solves"] == 3 and s["p99_latency_s"] >= s["p50_latency_s"]


def test_batch_step_equals_separate_solves():
    """Three Q2/Q1 solves begun together and advanced by mfs_batch_step (their
    system operators in one grouped launch per step) give the same solutions
    and iteration counts, bit for bit, as three separate mfs_solve calls; a
    Q3/Q2 solve in the same batch steps on its own."""
    from paper_2603_29621_amd.serving import _setup_request

    opts = mfs.mfs_default_options()
    reqs = [inputs.Request(i, 0.0, n, k, nu, 0.1, 20 + i)
            for i, (n, k, nu) in enumerate(((8, 2, 0.3), (6, 2, 0.05), (8, 2, 1.0), (4, 3, 0.2)))]
    ref = []
    for r in reqs:
        s = torch.cuda.Stream()
        h, b, x, arena = _setup_request(r, opts, s)
        info = mfs.mfs_solve(h, b, x, opts, stream=s.cuda_stream)
        ref.append((info.iterations, x.clone()))
        mfs.mfs_destroy(h)
        del arena
    live = []
    for r in reqs:
        s = torch.cuda.Stream()
        h, b, x, arena = _setup_request(r, opts, s)
        live.append((h, b, x, arena, s))
    for h, b, x, _, s in live:
        mfs.mfs_solve_begin(h, b, x, opts, stream=s.cuda_stream)
    gs = torch.cuda.Stream()
    done = [False] * len(live)
    infos = [None] * len(live)
    for _ in range(100000):
        idx = [i for i in range(len(live)) if not done[i]]
        if not idx:
            break
        out = mfs.mfs_batch_step([live[i][0] for i in idx], stream=gs.cuda_stream)
        for i, (d, info) in zip(idx, out):
            if d:
                done[i], infos[i] = True, info
    assert all(done)
    torch.cuda.synchronize()
    for (h, b, x, arena, s), info, (its, xr) in zip(live, infos, ref):
        assert info.status == 0 and info.iterations == its
        assert torch.equal(x, xr)
        mfs.mfs_destroy(h)

"""GPU parity of the BDF2 / Newton path of the stabilised Navier-Stokes
equations (Sec. 5) against the CPU oracle, through the C ABI: the
linearisation at a general state (nonzero pressure, BDF2 history u~ != u0,
delta_1 frozen at another velocity), the nonlinear residual there and the
Jacobian there, on structured and on locally refined meshes; and whole BDF2
steps by Newton-Krylov against the oracle's Newton iteration with direct
solves.

Tolerances: residual and Jacobian within 1e-12 relative (FP64), FP32
Jacobian within 2e-5, as for the Jacobian at a plain linearisation point.
Steps: with FP64 multigrid and tight tolerances (Newton 1e-10, FGMRES 1e-10)
the state after three steps within 1e-8 of the oracle's and the same number
of Newton corrections; with the FP32 multigrid and the default tolerances
(Newton 1e-8, FGMRES 1e-6) within 1e-6.
"""
import numpy as np
import pytest
import torch

import inputs
import paper_2603_29621_amd as mfs
from oracle import amr, bdf2, fem, ns

pytestmark = pytest.mark.gpu


def cuda(x, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda", dtype)


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def relerr(y, ref):
    d = y - ref
    return max(np.linalg.norm(d) / np.linalg.norm(ref), np.abs(d).max() / np.abs(ref).max())


def _state(n_nodes, dim, seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1, 1, (dim + 1) * n_nodes)
    uh = rng.uniform(-1, 1, dim * n_nodes)
    un = rng.uniform(-1, 1, dim * n_nodes)
    return x, uh, un


def _set_state(h, x, uh, un, nu, dt, dim, n_nodes):
    """delta_1 from u^n (state [u^n; 0]), then the state x with history uh."""
    xs = np.concatenate([un, np.zeros(n_nodes)])
    mfs.mfs_set_linearization_point(h, cuda(xs), cuda(un), dt, 1, 0)
    mfs.mfs_set_linearization_point(h, cuda(x), cuda(uh), dt, 1, 1)


@pytest.mark.parametrize("dim,n,k,noise", [(2, [6, 5], 2, 0.2), (3, [3, 2, 4], 1, 0.2), (3, [3, 4, 3], 2, 0.2),
                                           (3, [2, 3, 2], 3, 0.1), (3, [4, 4, 4], 2, 0.0)])
def test_residual_and_jacobian_at_a_general_state(dim, n, k, noise):
    nu, dt = 0.02, 0.05
    X = inputs.structured_vertices(dim, n, noise=noise, seed=4)
    h = mfs.mfs_setup(dim, n, X, k, nu, mfs.mfs_default_options(pressure_offset=0, mg_levels=0))
    try:
        S = fem.Space(dim, n, X, k, k)
        x, uh, un = _state(S.Nv, dim, 8)
        _set_state(h, x, uh, un, nu, dt, dim, S.Nv)
        delta = bdf2.frozen_delta(S, un, nu, dt)
        F = torch.empty((dim + 1) * S.Nv, dtype=torch.float64, device="cuda")
        mfs.mfs_ns_residual(h, F)
        ref = bdf2.residual(S, x, uh, delta, nu, dt)
        assert relerr(host(F), ref) <= 1e-12
        data = bdf2.point_data(S, x, uh, delta, nu, dt)
        d = inputs.uniform_vector((dim + 1) * S.Nv, 13)
        for newton in (1, 0):
            if newton == 0:
                mfs.mfs_set_linearization_point(h, cuda(x), cuda(uh), dt, 0, 1)
            refJ = ns.constrained_jacobian_apply(S, d, data, nu, dt, bool(newton))
            y = torch.empty((dim + 1) * S.Nv, dtype=torch.float64, device="cuda")
            mfs.mfs_vmult(h, mfs.MFS_OP_NS_JACOBIAN, mfs.MFS_FP64, 0, y, cuda(d))
            assert relerr(host(y), refJ) <= 1e-12
            y32 = torch.empty((dim + 1) * S.Nv, dtype=torch.float32, device="cuda")
            mfs.mfs_vmult(h, mfs.MFS_OP_NS_JACOBIAN, mfs.MFS_FP32, 0, y32, cuda(d, torch.float32))
            assert relerr(host(y32), refJ) <= 2e-5
    finally:
        mfs.mfs_destroy(h)


REFINED = {"n3L2": dict(n=3, seed=0, levels=2, centre=[0.4, 0.5, 0.55], radius=0.3),
           "n4L1": dict(n=4, seed=1, levels=1, radius=0.3)}


@pytest.mark.parametrize("name", list(REFINED))
@pytest.mark.parametrize("k", [1, 2])
def test_refined_residual_and_jacobian_at_a_general_state(name, k):
    nu, dt = 0.02, 0.05
    mesh = inputs.refined_mesh(**REFINED[name])
    h = mfs.mfs_setup_refined(mesh, k, nu)
    try:
        S = amr.AmrSpace(mesh, k)
        x, uh, un = _state(S.N, 3, 9)
        _set_state(h, x, uh, un, nu, dt, 3, S.N)
        delta = bdf2.frozen_delta(S, S.expand(un, 3), nu, dt)
        mask = S.ns_dirichlet_true()
        F = torch.empty(4 * S.N, dtype=torch.float64, device="cuda")
        mfs.mfs_ns_residual(h, F)
        raw = ns.residual(S, S.expand(x, 4), None, nu, dt, bdf2.residual_data(S, S.expand(uh, 3), delta, nu, dt))
        ref = S.restrict(raw, 4)
        ref[mask] = 0.0
        assert relerr(host(F), ref) <= 1e-12
        data = bdf2.point_data(S, S.expand(x, 4), S.expand(uh, 3), delta, nu, dt)
        d = inputs.uniform_vector(4 * S.N, 14)
        refJ = amr.jacobian_apply(S, d, None, nu, dt, True, data=data)
        y = torch.empty(4 * S.N, dtype=torch.float64, device="cuda")
        mfs.mfs_vmult(h, mfs.MFS_OP_NS_JACOBIAN, mfs.MFS_FP64, 0, y, cuda(d))
        assert relerr(host(y), refJ) <= 1e-12
    finally:
        mfs.mfs_destroy(h)


@pytest.mark.parametrize("prec", [mfs.MFS_FP64, mfs.MFS_FP32])
def test_three_bdf2_steps_match_the_oracle(prec):
    """4^3 Q2Q2 Cartesian cells, Re = 100 (nu = 0.01, unit RMS velocity),
    dt = 1e-2, zero velocity on the boundary, initial velocity the 8-mode
    Fourier field."""
    n, k, nu, dt = [4, 4, 4], 2, 0.01, 0.01
    X = inputs.structured_vertices(3, n)
    tight = prec == mfs.MFS_FP64
    opts = mfs.mfs_default_options(pressure_offset=0, mg_levels=1, precond_precision=prec)
    h = mfs.mfs_setup(3, n, X, k, nu, opts)
    try:
        S = fem.Space(3, n, X, k, k)
        u = inputs.ns_velocity(3, [k * v + 1 for v in n], seed=0)
        states, hists = bdf2.bdf2(S, u, nu, dt, 3, rtol=1e-10)
        nopt = mfs.mfs_default_newton_options(precond_precision=prec, rtol=1e-10 if tight else 1e-8,
                                              linear_rtol=1e-10 if tight else 1e-6)
        mask = ns.ns_dirichlet_mask(S)
        un = cuda(u)
        unm1 = cuda(u)
        p = torch.zeros(S.Nv, dtype=torch.float64, device="cuda")
        for step in range(3):
            x = torch.cat([un, p])
            x[torch.from_numpy(mask).cuda()] = 0.0
            info = mfs.mfs_ns_bdf2_step(h, un, unm1, x, dt, nopt)
            print(f"step {step}: Newton {info.newton_iterations} (oracle {len(hists[step]) - 1}), "
                  f"FGMRES {info.linear_iterations}, ||F|| {info.res0:.3e} -> {info.res:.3e}")
            assert info.status == 0 and info.linear_failures == 0
            err = relerr(host(x), states[step])
            print(f"step {step}: relative difference to the oracle {err:.2e}")
            if tight:
                assert abs(info.newton_iterations - (len(hists[step]) - 1)) <= 1
                assert err <= 1e-8
            else:
                assert err <= 1e-6
            unm1, un, p = un, x[:3 * S.Nv].clone(), x[3 * S.Nv:].clone()
    finally:
        mfs.mfs_destroy(h)

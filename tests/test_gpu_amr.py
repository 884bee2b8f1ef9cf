"""GPU parity of the Navier-Stokes path on locally refined meshes (hanging
nodes) against the CPU oracle, through the C ABI: the constrained Jacobian,
and with multigrid the global-coarsening levels (operators, Jacobi
diagonals, transfers), the V-cycle and the FGMRES solve.

Tolerances as on structured meshes: FP64 operators, diagonals and transfers
within 1e-12 relative (2-norm and max-norm), FP32 Jacobian within 2e-5,
V-cycle within 1e-9 (FP64) and 1e-4 (FP32), solves to the FGMRES tolerance.
The oracle's constrained Jacobian (C^T J_raw C with the Dirichlet rows) and
its multigrid are pinned in test_oracle_amr.py.
"""
import numpy as np
import pytest
import torch

import inputs
import paper_2603_29621_amd as mfs
from oracle import amr

pytestmark = pytest.mark.gpu


def cuda(x, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda", dtype)


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def relerr(y, ref):
    d = y - ref
    return max(np.linalg.norm(d) / np.linalg.norm(ref), np.abs(d).max() / np.abs(ref).max())


MESHES = {
    "n3L2": dict(n=3, seed=0, levels=2, centre=[0.4, 0.5, 0.55], radius=0.3),
    "n4L2seed": dict(n=4, seed=1, levels=2),
    "n6L1": dict(n=6, seed=2, levels=1, radius=0.3),
    # degenerate cases: one base cell refined twice; a mesh refined everywhere
    # (no hanging nodes, the structured mesh of twice the resolution)
    "n1L2": dict(n=1, seed=0, levels=2, centre=[0.3, 0.4, 0.6], radius=0.45),
    "n2all": dict(n=2, seed=0, levels=1, centre=[0.5, 0.5, 0.5], radius=10.0),
}


def _problem(mesh, k, nu):
    h = mfs.mfs_setup_refined(mesh, k, nu)
    S = amr.AmrSpace(mesh, k)
    return h, S


@pytest.mark.parametrize("name", list(MESHES))
@pytest.mark.parametrize("k", [1, 2])
def test_numbering_and_points(name, k):
    mesh = inputs.refined_mesh(**MESHES[name])
    h, S = _problem(mesh, k, 0.01)
    try:
        assert mfs.mfs_n_dofs(h, 0) == (S.N, S.N)
        assert mfs.mfs_n_levels(h) == 1
        assert mfs.mfs_level_info(h, 0) == (k, [mesh["n"]] * 3)
        pts = mfs.mfs_support_points(h, k, S.N, 3)
        assert np.abs(pts - S.true_points()).max() < 1e-15
    finally:
        mfs.mfs_destroy(h)


@pytest.mark.parametrize("name", list(MESHES))
@pytest.mark.parametrize("k,newton", [(1, 1), (2, 1), (2, 0)])
def test_refined_jacobian(name, k, newton):
    mesh = inputs.refined_mesh(**MESHES[name])
    nu, dt = 0.01, 1e-2
    h, S = _problem(mesh, k, nu)
    try:
        u0 = inputs.fourier_field(4)(S.true_points()).T.ravel()
        mfs.mfs_set_linearization(h, cuda(u0), dt, newton)
        N = 4 * S.N
        dx = inputs.uniform_vector(N, 9)
        ref = amr.jacobian_apply(S, dx, u0, nu, dt, bool(newton))
        y = torch.full((N,), 7.0, dtype=torch.float64, device="cuda")
        mfs.mfs_vmult(h, mfs.MFS_OP_NS_JACOBIAN, mfs.MFS_FP64, 0, y, cuda(dx))
        assert relerr(host(y), ref) <= 1e-12
        y32 = torch.full((N,), 7.0, dtype=torch.float32, device="cuda")
        mfs.mfs_vmult(h, mfs.MFS_OP_NS_JACOBIAN, mfs.MFS_FP32, 0, y32, cuda(dx, torch.float32))
        assert relerr(host(y32), ref) <= 2e-5
        # a second application (the E-vectors are reused) gives the same result
        y2 = torch.empty_like(y)
        mfs.mfs_vmult(h, mfs.MFS_OP_NS_JACOBIAN, mfs.MFS_FP64, 0, y2, cuda(dx))
        assert relerr(host(y2), ref) <= 1e-12
    finally:
        mfs.mfs_destroy(h)


def test_refined_matches_assembled_matrix_and_kernel():
    """Against the assembled oracle matrix: several random vectors, and the
    constant pressure in the kernel (up to rounding)."""
    mesh = inputs.refined_mesh(**MESHES["n3L2"])
    nu, dt = 0.02, 5e-3
    h, S = _problem(mesh, 2, nu)
    try:
        u0 = inputs.fourier_field(6)(S.true_points()).T.ravel()
        mfs.mfs_set_linearization(h, cuda(u0), dt, 1)
        J = amr.jacobian_matrix(S, u0, nu, dt, True)
        N = 4 * S.N
        for seed in range(3):
            dx = inputs.uniform_vector(N, 20 + seed)
            y = torch.empty(N, dtype=torch.float64, device="cuda")
            mfs.mfs_vmult(h, mfs.MFS_OP_NS_JACOBIAN, mfs.MFS_FP64, 0, y, cuda(dx))
            assert relerr(host(y), J @ dx) <= 1e-12
        e = np.zeros(N)
        e[3 * S.N:] = 1.0
        y = torch.empty(N, dtype=torch.float64, device="cuda")
        mfs.mfs_vmult(h, mfs.MFS_OP_NS_JACOBIAN, mfs.MFS_FP64, 0, y, cuda(e))
        assert np.abs(host(y)).max() <= 1e-12 * abs(J).max()
    finally:
        mfs.mfs_destroy(h)


def test_refined_jacobian_full_size_properties():
    """128^3 base cells + 2 levels in the bench's sphere (3.97 M cells), Q1Q1,
    in the launch configuration the bench times: the oracle cannot build this
    space, so properties that hold at any size are checked.  The constant
    pressure is in the kernel (the velocity unknowns vanish on the boundary);
    Dirichlet rows are the identity; FP32 agrees with FP64 to 2e-5; a
    second application repeats the first bit for bit (no atomics)."""
    mesh = inputs.refined_mesh(128, seed=0, levels=2, radius=0.15)
    nu, dt = 0.01, 1e-2
    h = mfs.mfs_setup_refined(mesh, 1, nu)
    try:
        n_u, _ = mfs.mfs_n_dofs(h, 0)
        assert n_u == 3969031
        pts = mfs.mfs_support_points(h, 1, n_u, 3)
        u0 = inputs.fourier_field(0)(pts).T.ravel()
        mfs.mfs_set_linearization(h, cuda(u0), dt, 1)
        N = 4 * n_u
        e = torch.zeros(N, dtype=torch.float64, device="cuda")
        e[3 * n_u:] = 1.0
        y = torch.empty_like(e)
        mfs.mfs_vmult(h, mfs.MFS_OP_NS_JACOBIAN, mfs.MFS_FP64, 0, y, e)
        x = cuda(inputs.uniform_vector(N, 5))
        z = torch.empty_like(x)
        mfs.mfs_vmult(h, mfs.MFS_OP_NS_JACOBIAN, mfs.MFS_FP64, 0, z, x)
        scale = float(z.abs().max())
        assert float(y.abs().max()) <= 1e-12 * scale
        bnd = np.any((pts == 0.0) | (pts == 1.0), axis=1)
        zz, xx = host(z), host(x)
        for c in range(3):
            sl = slice(c * n_u, (c + 1) * n_u)
            assert np.array_equal(zz[sl][bnd], xx[sl][bnd])
        z2 = torch.empty_like(x)
        mfs.mfs_vmult(h, mfs.MFS_OP_NS_JACOBIAN, mfs.MFS_FP64, 0, z2, x)
        assert torch.equal(z, z2)
        z32 = torch.empty(N, dtype=torch.float32, device="cuda")
        mfs.mfs_vmult(h, mfs.MFS_OP_NS_JACOBIAN, mfs.MFS_FP32, 0, z32, x.float())
        assert relerr(host(z32), zz) <= 2e-5
    finally:
        mfs.mfs_destroy(h)


def test_refined_multigrid_needs_refinement():
    """Multigrid on a mesh without refined cells is rejected (the structured
    set-up serves it); operators alone are fine."""
    mesh = {"n": 2, "levels": 0, "level": np.zeros(8, dtype=np.int32),
            "idx": np.array([[x, y, z] for z in range(2) for y in range(2) for x in range(2)], dtype=np.int32)}
    with pytest.raises(mfs.MfsError) as e:
        mfs.mfs_setup_refined(mesh, 2, 0.01, mfs.mfs_default_options(pressure_offset=0, mg_levels=1))
    assert e.value.code == mfs.MFS_EINVAL
    h = mfs.mfs_setup_refined(mesh, 2, 0.01)
    try:
        S = amr.AmrSpace(mesh, 2)
        assert mfs.mfs_n_dofs(h, 0) == (S.N, S.N) == (125, 125)
    finally:
        mfs.mfs_destroy(h)


def test_refined_errors():
    mesh = inputs.refined_mesh(**MESHES["n3L2"])
    h, S = _problem(mesh, 1, 0.01)
    try:
        N = 4 * S.N
        x = torch.zeros(N, dtype=torch.float64, device="cuda")
        y = torch.zeros(N, dtype=torch.float64, device="cuda")
        with pytest.raises(mfs.MfsError) as e:  # not linearised yet
            mfs.mfs_vmult(h, mfs.MFS_OP_NS_JACOBIAN, mfs.MFS_FP64, 0, y, x)
        assert e.value.code == mfs.MFS_EINVAL
        mfs.mfs_set_linearization(h, torch.zeros(3 * S.N, dtype=torch.float64, device="cuda"), 0.1, 1)
        with pytest.raises(mfs.MfsError) as e:
            mfs.mfs_vmult(h, mfs.MFS_OP_STOKES, mfs.MFS_FP64, 0, y, x)
        assert e.value.code == mfs.MFS_EUNSUPPORTED
        with pytest.raises(mfs.MfsError) as e:  # set up without multigrid levels
            mfs.mfs_vcycle(h, mfs.MFS_FP64, y, x)
        assert e.value.code == mfs.MFS_EINVAL
        with pytest.raises(mfs.MfsError) as e:
            mfs.mfs_solve(h, x, y)
        assert e.value.code == mfs.MFS_EINVAL
        with pytest.raises(mfs.MfsError) as e:
            mfs.mfs_diagonal(h, 0, y)
        assert e.value.code == mfs.MFS_EUNSUPPORTED
    finally:
        mfs.mfs_destroy(h)


# ------------------------------------------------------------------ multigrid
from oracle import amr_mg  # noqa: E402

MG_CASES = [("n3L2", 1), ("n3L2", 2), ("n4L2seed", 2), ("n6L1", 2), ("n1L2", 2), ("n2all", 1)]


def _mg_problem(name, k, nu=0.01, dt=1e-2, newton=1):
    mesh = inputs.refined_mesh(**MESHES[name])
    S = amr.AmrSpace(mesh, k)
    u0 = inputs.fourier_field(4)(S.true_points()).T.ravel()
    H = amr_mg.AmrNSHierarchy(mesh, k, nu, dt, u0, newton=bool(newton))
    h = mfs.mfs_setup_refined(mesh, k, nu, mfs.mfs_default_options(pressure_offset=0, mg_levels=1))
    mfs.mfs_set_linearization(h, cuda(u0), dt, newton)
    return h, H


@pytest.mark.parametrize("name,k", MG_CASES)
def test_refined_levels_operators_diagonals_transfers(name, k):
    h, H = _mg_problem(name, k)
    try:
        assert mfs.mfs_n_levels(h) == H.nga + len(H.base.spaces)
        for j in range(H.nga):
            Sf, Sc = H.spaces[j], H.spaces[j + 1]
            assert mfs.mfs_n_dofs(h, j) == (Sf.N, Sf.N)
            Nf, Nc = 4 * Sf.N, 4 * Sc.N
            x = inputs.uniform_vector(Nf, 40 + j)
            y = torch.empty(Nf, dtype=torch.float64, device="cuda")
            mfs.mfs_vmult(h, mfs.MFS_OP_NS_JACOBIAN, mfs.MFS_FP64, j, y, cuda(x))
            assert relerr(host(y), H.J[j] @ x) <= 1e-12
            d = torch.empty(Nf, dtype=torch.float64, device="cuda")
            mfs.mfs_diagonal(h, j, d)
            assert relerr(host(d), 1.0 / H.Dinv[j]) <= 1e-12
            xc = inputs.uniform_vector(Nc, 50 + j)
            yf = torch.zeros(Nf, dtype=torch.float64, device="cuda")
            mfs.mfs_prolongate_add(h, mfs.MFS_FP64, j, yf, cuda(xc))
            assert relerr(host(yf), H.P[j] @ xc) <= 1e-12
            yc = torch.empty(Nc, dtype=torch.float64, device="cuda")
            mfs.mfs_restrict(h, mfs.MFS_FP64, j, yc, cuda(x))
            assert relerr(host(yc), H.P[j].T @ x) <= 1e-12
        # the first structured level is the uniform base mesh
        Sb = H.base.spaces[0]
        assert mfs.mfs_n_dofs(h, H.nga) == (Sb.Nv, Sb.Nv)
        xb = inputs.uniform_vector(4 * Sb.Nv, 60)
        yb = torch.empty(4 * Sb.Nv, dtype=torch.float64, device="cuda")
        mfs.mfs_vmult(h, mfs.MFS_OP_NS_JACOBIAN, mfs.MFS_FP64, H.nga, yb, cuda(xb))
        assert relerr(host(yb), H.base.J[0] @ xb) <= 1e-12
    finally:
        mfs.mfs_destroy(h)


@pytest.mark.parametrize("name,k", MG_CASES)
def test_refined_vcycle(name, k):
    """FP64 V-cycle within 1e-9 of the oracle (about 30 operator applications
    and the dense coarse inverse against an LU solve, as on structured
    meshes); FP32 within 1e-4."""
    h, H = _mg_problem(name, k)
    try:
        N = 4 * H.spaces[0].N
        b = inputs.uniform_vector(N, 70)
        ref = H.vcycle(b)
        y = torch.empty(N, dtype=torch.float64, device="cuda")
        mfs.mfs_vcycle(h, mfs.MFS_FP64, y, cuda(b))
        assert relerr(host(y), ref) <= 1e-9
        y32 = torch.empty(N, dtype=torch.float32, device="cuda")
        mfs.mfs_vcycle(h, mfs.MFS_FP32, y32, cuda(b, torch.float32))
        assert relerr(host(y32), ref) <= 1e-4
    finally:
        mfs.mfs_destroy(h)


@pytest.mark.parametrize("name,k", MG_CASES)
def test_refined_solve(name, k):
    h, H = _mg_problem(name, k)
    try:
        N = 4 * H.spaces[0].N
        xt = inputs.uniform_vector(N, 80)
        xt[H.fixed[0]] = 0.0
        b = H.J[0] @ xt
        x_ref, its_ref, _ = H.solve(b, rtol=1e-10)
        for prec in (mfs.MFS_FP64, mfs.MFS_FP32):
            x = torch.zeros(N, dtype=torch.float64, device="cuda")
            info = mfs.mfs_solve(h, cuda(b), x, mfs.mfs_default_options(pressure_offset=0, rtol=1e-10,
                                                                          precond_precision=prec))
            assert info.status == 0 and info.rel_residual <= 1e-10
            xs = host(x)
            assert abs(xs[3 * H.spaces[0].N:].mean()) <= 1e-12 * np.abs(xs).max()
            assert relerr(xs, x_ref) <= 1e-6
            if prec == mfs.MFS_FP64:
                assert abs(info.iterations - its_ref) <= 1
            else:
                assert info.iterations <= its_ref + 3
    finally:
        mfs.mfs_destroy(h)

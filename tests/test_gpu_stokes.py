"""GPU parity of the HIP library against the CPU oracle, through the C ABI.

Tolerances: FP64 results within 1e-12 relative (2-norm and max-norm) of the
oracle for every operator; FP32 operators within 1e-5 relative; transfers
and V-cycles in FP64 within 1e-11 (they chain several operators).
"""
import numpy as np
import pytest
import torch

import inputs
import paper_2603_29621_amd as mfs
from oracle import fem, krylov, mg, solve
from bounds import bordered_error_bound

pytestmark = pytest.mark.gpu


def cuda(x, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda", dtype)


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def relerr(y, ref):
    d = y - ref
    n2 = np.linalg.norm(ref)
    ninf = np.abs(ref).max()
    return max(np.linalg.norm(d) / (n2 if n2 > 0 else 1), np.abs(d).max() / (ninf if ninf > 0 else 1))


# (dim, n, k, noise): several workgroups and ragged tails for every degree
CASES = [
    (2, [16, 16], 2, 0.0),
    (2, [7, 5], 2, 0.2),
    (2, [5, 6], 3, 0.2),
    (2, [3, 4], 4, 0.2),
    (2, [2, 3], 6, 0.1),
    (3, [1, 1, 1], 2, 0.0),
    (3, [4, 4, 4], 2, 0.2),
    (3, [5, 3, 4], 2, 0.2),
    (3, [3, 4, 3], 3, 0.2),
    (3, [3, 2, 3], 4, 0.2),
    (3, [2, 2, 3], 5, 0.1),
    (3, [2, 2, 2], 6, 0.1),
]


def _setup(dim, n, k, noise, nu=0.7, mg_levels=0, **kw):
    X = inputs.structured_vertices(dim, n, noise=noise, seed=3)
    opts = mfs.mfs_default_options(mg_levels=mg_levels, **kw)
    h = mfs.mfs_setup(dim, n, X, k, nu, opts)
    return h, X


@pytest.mark.parametrize("dim,n,k,noise", CASES)
def test_stokes_operators_fp64(dim, n, k, noise):
    nu = 0.7
    h, X = _setup(dim, n, k, noise, nu)
    try:
        S = fem.Space(dim, n, X, k)
        K, mats = fem.stokes_operator(S, nu)
        mask = S.velocity_dirichlet_mask()
        nvel = dim * S.Nv
        assert mfs.mfs_n_dofs(h, 0) == (S.Nv, S.Np)
        x = inputs.uniform_vector(S.n_dofs, 11)
        src = cuda(x)
        dst = torch.empty_like(src)
        mfs.mfs_vmult(h, mfs.MFS_OP_STOKES, mfs.MFS_FP64, 0, dst, src)
        assert relerr(host(dst), K @ x) <= 1e-12
        # blocks
        Z = (~mask[:nvel]).astype(float)
        A = fem.constrain(mats["Avec"], mask[:nvel])
        xu, xp = x[:nvel], x[nvel:]
        du = torch.empty(nvel, dtype=torch.float64, device="cuda")
        dp = torch.empty(S.Np, dtype=torch.float64, device="cuda")
        mfs.mfs_vmult(h, mfs.MFS_OP_A, mfs.MFS_FP64, 0, du, cuda(xu))
        assert relerr(host(du), A @ xu) <= 1e-12
        mfs.mfs_vmult(h, mfs.MFS_OP_B, mfs.MFS_FP64, 0, du, cuda(xp))
        assert relerr(host(du), Z * (mats["B"] @ xp)) <= 1e-12
        mfs.mfs_vmult(h, mfs.MFS_OP_BT, mfs.MFS_FP64, 0, dp, cuda(xu))
        assert relerr(host(dp), mats["B"].T @ (Z * xu)) <= 1e-12
        mfs.mfs_vmult(h, mfs.MFS_OP_MASS_P, mfs.MFS_FP64, 0, dp, cuda(xp))
        assert relerr(host(dp), mats["M"] @ xp) <= 1e-12
        # diagonal of the scalar Laplacian (1 on Dirichlet rows)
        dg = torch.empty(S.Nv, dtype=torch.float64, device="cuda")
        mfs.mfs_diagonal(h, 0, dg)
        ref = fem.constrain(mats["A"], S.dirichlet).diagonal()
        assert relerr(host(dg), ref) <= 1e-12
    finally:
        mfs.mfs_destroy(h)


@pytest.mark.parametrize("dim,n,k,noise", [CASES[1], CASES[6], CASES[8], CASES[9]])
def test_stokes_operators_fp32(dim, n, k, noise):
    nu = 0.7
    h, X = _setup(dim, n, k, noise, nu)
    try:
        S = fem.Space(dim, n, X, k)
        K, mats = fem.stokes_operator(S, nu)
        x = inputs.uniform_vector(S.n_dofs, 12).astype(np.float32).astype(np.float64)
        src = cuda(x, torch.float32)
        dst = torch.empty_like(src)
        mfs.mfs_vmult(h, mfs.MFS_OP_STOKES, mfs.MFS_FP32, 0, dst, src)
        assert relerr(host(dst), K @ x) <= 1e-5
        # gradient block B alone (Dirichlet rows 0)
        nvel = dim * S.Nv
        Z = (~S.velocity_dirichlet_mask()[:nvel]).astype(float)
        du = torch.empty(nvel, dtype=torch.float32, device="cuda")
        mfs.mfs_vmult(h, mfs.MFS_OP_B, mfs.MFS_FP32, 0, du, cuda(x[nvel:], torch.float32))
        assert relerr(host(du), Z * (mats["B"] @ x[nvel:])) <= 1e-5
    finally:
        mfs.mfs_destroy(h)


@pytest.mark.parametrize("k", [2, 3, 4])
def test_stokes_vmult_full_size_sampled(k):
    """64^3 cells, vertex noise 0.2h: sampled rows against the oracle, plus
    symmetry and the pressure null vector at full size."""
    dim, n, nu = 3, [64, 64, 64], 1.0
    X = inputs.structured_vertices(dim, n, noise=0.2, seed=0)
    h = mfs.mfs_setup(dim, n, X, k, nu, mfs.mfs_default_options(mg_levels=0))
    try:
        Nv, Np = mfs.mfs_n_dofs(h, 0)
        N = dim * Nv + Np
        x = inputs.uniform_vector(N, 1)
        src = cuda(x)
        dst = torch.empty_like(src)
        mfs.mfs_vmult(h, mfs.MFS_OP_STOKES, mfs.MFS_FP64, 0, dst, src)
        y = host(dst)
        S = fem.Space(dim, n, X, k)
        rows = np.unique(np.concatenate([
            np.random.default_rng(5).choice(N, 400, replace=False),
            [0, dim * Nv - 1, dim * Nv, N - 1, Nv + Nv // 2, dim * Nv + Np // 2]]))
        ref = fem.sampled_stokes_rows(S, nu, x, rows)
        scale = np.abs(ref).max()
        assert np.abs(y[rows] - ref).max() <= 1e-12 * scale
        # symmetry: <K x, z> = <x, K z> on free rows
        z = inputs.uniform_vector(N, 2)
        dz = torch.empty_like(src)
        mfs.mfs_vmult(h, mfs.MFS_OP_STOKES, mfs.MFS_FP64, 0, dz, cuda(z))
        mask = np.zeros(N, dtype=bool)
        mask[:dim * Nv] = np.tile(S.dirichlet, dim)
        xf, zf = np.where(mask, 0, x), np.where(mask, 0, z)
        a, b = y @ zf, xf @ host(dz)
        assert abs(a - b) <= 1e-11 * (np.abs(y) @ np.abs(zf))
        # (0, 1_p) is in the kernel
        one = np.zeros(N)
        one[dim * Nv:] = 1.0
        mfs.mfs_vmult(h, mfs.MFS_OP_STOKES, mfs.MFS_FP64, 0, dz, cuda(one))
        assert np.abs(host(dz)).max() <= 1e-12 * scale
    finally:
        mfs.mfs_destroy(h)


@pytest.mark.parametrize("k", [2, 3])
def test_solve_full_size_residual_sampled(k):
    """The 64^3 solve of the bench (FP32 multigrid inside FP64 FGMRES to
    1e-8) checked by the oracle at full size: b = K y with y ~ U[-1, 1]
    (b's sampled rows equal the oracle's K y rows to 1e-12), and the oracle's
    rows of b - K x for the GPU solution x are below 1e-8 ||b||_2, the bound
    the 2-norm residual puts on every entry."""
    dim, n, nu = 3, [64, 64, 64], 1.0
    X = inputs.structured_vertices(dim, n, noise=0.2, seed=0)
    opts = mfs.mfs_default_options(rtol=1e-8, precond_precision=mfs.MFS_FP32)
    h = mfs.mfs_setup(dim, n, X, k, nu, opts)
    try:
        Nv, Np = mfs.mfs_n_dofs(h, 0)
        N = dim * Nv + Np
        y = inputs.uniform_vector(N, 11)
        b = torch.empty(N, dtype=torch.float64, device="cuda")
        mfs.mfs_vmult(h, mfs.MFS_OP_STOKES, mfs.MFS_FP64, 0, b, cuda(y))
        x = torch.zeros_like(b)
        info = mfs.mfs_solve(h, b, x, opts)
        assert info.status == 0 and info.rel_residual <= 1e-8
        bh, xh = host(b), host(x)
        S = fem.Space(dim, n, X, k)
        rows = np.unique(np.concatenate([
            np.random.default_rng(6).choice(N, 400, replace=False),
            [0, dim * Nv - 1, dim * Nv, N - 1, Nv + Nv // 2, dim * Nv + Np // 2]]))
        Ky = fem.sampled_stokes_rows(S, nu, y, rows)
        assert np.abs(bh[rows] - Ky).max() <= 1e-12 * np.abs(Ky).max()
        r = Ky - fem.sampled_stokes_rows(S, nu, xh, rows)
        bnorm = np.linalg.norm(bh)
        print(f"64^3 Q{k}: {info.iterations} iterations, max sampled residual {np.abs(r).max() / bnorm:.2e} ||b||")
        assert np.abs(r).max() <= 1e-8 * bnorm
    finally:
        mfs.mfs_destroy(h)


def test_support_and_quadrature_points():
    dim, n, k = 3, [3, 2, 4], 3
    h, X = _setup(dim, n, k, 0.2)
    try:
        S = fem.Space(dim, n, X, k)
        sp_ = mfs.mfs_support_points(h, k, S.Nv, dim)
        assert np.abs(sp_ - S.support_points()).max() < 1e-14
        q = mfs.mfs_quadrature_points(h, S.nc, (k + 1) ** dim, dim)
        assert np.abs(q - S.geometry()[0]).max() < 1e-14
    finally:
        mfs.mfs_destroy(h)


def test_inverted_cell_rejected():
    dim, n = 2, [2, 2]
    X = inputs.structured_vertices(dim, n)
    X[4] = [0.9, 0.9]  # centre vertex pushed past the far corner: cell 0 folds
    with pytest.raises(mfs.MfsError) as e:
        mfs.mfs_setup(dim, n, X, 2, 1.0, mfs.mfs_default_options(mg_levels=0))
    assert e.value.code == mfs.MFS_EINVAL and "cell" in str(e.value)


def test_binding_rejects_short_or_mistyped_vectors():
    """The binding checks every vector against the length and word the call
    reads and writes, before anything is enqueued."""
    dim, n, k = 3, [2, 2, 2], 2
    X = inputs.structured_vertices(dim, n)
    h = mfs.mfs_setup(dim, n, X, k, 1.0, mfs.mfs_default_options(mg_levels=0))
    try:
        nu, np_ = mfs.mfs_n_dofs(h, 0)
        N = dim * nu + np_
        ok = torch.zeros(N, dtype=torch.float64, device="cuda")
        short = torch.zeros(N - 1, dtype=torch.float64, device="cuda")
        with pytest.raises(ValueError, match="needs"):
            mfs.mfs_vmult(h, mfs.MFS_OP_STOKES, mfs.MFS_FP64, 0, short, ok)
        with pytest.raises(ValueError, match="needs"):
            mfs.mfs_vmult(h, mfs.MFS_OP_STOKES, mfs.MFS_FP64, 0, ok, short)
        with pytest.raises(ValueError, match="dtype"):
            mfs.mfs_vmult(h, mfs.MFS_OP_STOKES, mfs.MFS_FP32, 0, ok, ok)
        with pytest.raises(ValueError, match="needs"):
            mfs.mfs_vmult(h, mfs.MFS_OP_A, mfs.MFS_FP64, 0, ok[: dim * nu - 1], ok)
        with pytest.raises(ValueError, match="needs"):
            mfs.mfs_solve(h, ok, short)
        # exact lengths pass
        mfs.mfs_vmult(h, mfs.MFS_OP_BT, mfs.MFS_FP64, 0, torch.zeros(np_, dtype=torch.float64, device="cuda"),
                      ok[: dim * nu])
        torch.cuda.synchronize()
    finally:
        mfs.mfs_destroy(h)


# ------------------------------------------------------------------ multigrid
MG_CASES = [(2, [8, 8], 2, 0.2), (2, [4, 6], 3, 0.1), (3, [4, 4, 4], 2, 0.2), (3, [2, 2, 4], 3, 0.2), (3, [2, 3, 2], 4, 0.1)]


def _oracle_hierarchy(dim, n, X, k, nu, cheb_degree):
    H = mg.Hierarchy(dim, n, X, k, nu, cheb_degree=cheb_degree)
    for l in range(len(H.spaces) - 1):
        H.lam[l] = 1.2 * H.exact_lambda_max(l)
    return H


@pytest.mark.parametrize("dim,n,k,noise", MG_CASES)
def test_levels_transfers_and_lambda(dim, n, k, noise):
    nu = 1.3
    h, X = _setup(dim, n, k, noise, nu, mg_levels=1, cheb_degree=3)
    try:
        H = _oracle_hierarchy(dim, n, X, k, nu, 3)
        assert mfs.mfs_n_levels(h) == len(H.spaces)
        for l, S in enumerate(H.spaces):
            kl, nl = mfs.mfs_level_info(h, l)
            assert kl == S.k and nl[:dim] == S.n
        for l in range(len(H.spaces) - 1):
            Sf, Sc = H.spaces[l], H.spaces[l + 1]
            xc = inputs.uniform_vector(dim * Sc.Nv, 20 + l)
            xf = inputs.uniform_vector(dim * Sf.Nv, 40 + l)
            y = cuda(xf.copy())
            mfs.mfs_prolongate_add(h, mfs.MFS_FP64, l, y, cuda(xc))
            assert relerr(host(y), xf + H.P[l] @ xc) <= 1e-13
            r = torch.empty(dim * Sc.Nv, dtype=torch.float64, device="cuda")
            mfs.mfs_restrict(h, mfs.MFS_FP64, l, r, cuda(xf))
            assert relerr(host(r), H.P[l].T @ xf) <= 1e-13
            # adjointness of the two GPU kernels
            yy = torch.zeros(dim * Sf.Nv, dtype=torch.float64, device="cuda")
            mfs.mfs_prolongate_add(h, mfs.MFS_FP64, l, yy, cuda(xc))
            lhs = host(r) @ xc
            rhs = xf @ host(yy)
            assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1e-30)
            # Lanczos estimate (20 steps) against the exact largest eigenvalue
            lam = mfs.mfs_get_lambda(h, l) / 1.2
            ex = H.exact_lambda_max(l)
            assert 0.85 * ex <= lam <= ex * (1 + 1e-10)
    finally:
        mfs.mfs_destroy(h)


@pytest.mark.parametrize("n,k", [([6, 4, 4], 2), ([4, 2, 4], 3), ([2, 2, 2], 4), ([18, 10, 6], 2)])
def test_transfers_3d_every_level(n, k):
    """3D prolongation and restriction on every level pair (p-transfers from
    degree k down to 1, then degree-1 h-transfers) in FP64 and FP32 against
    the oracle's transfer matrices; FP32 inputs are rounded to FP32 first so
    the reference sees the same values."""
    dim, nu = 3, 1.0
    h, X = _setup(dim, n, k, 0.2, nu, mg_levels=1)
    try:
        H = mg.Hierarchy(dim, n, X, k, nu)
        assert mfs.mfs_n_levels(h) == len(H.spaces)
        for l in range(len(H.spaces) - 1):
            Sf, Sc = H.spaces[l], H.spaces[l + 1]
            for prec, dt, tol in ((mfs.MFS_FP64, torch.float64, 1e-13), (mfs.MFS_FP32, torch.float32, 1e-5)):
                xc = inputs.uniform_vector(dim * Sc.Nv, 20 + l)
                xf = inputs.uniform_vector(dim * Sf.Nv, 40 + l)
                if dt == torch.float32:
                    xc = xc.astype(np.float32).astype(np.float64)
                    xf = xf.astype(np.float32).astype(np.float64)
                y = cuda(xf, dt)
                mfs.mfs_prolongate_add(h, prec, l, y, cuda(xc, dt))
                assert relerr(host(y), xf + H.P[l] @ xc) <= tol, (l, prec)
                r = torch.empty(dim * Sc.Nv, dtype=dt, device="cuda")
                mfs.mfs_restrict(h, prec, l, r, cuda(xf, dt))
                assert relerr(host(r), H.P[l].T @ xf) <= tol, (l, prec)
    finally:
        mfs.mfs_destroy(h)


@pytest.mark.parametrize("n,k,noise", [([12, 10, 6], 2, 0.2), ([16, 8, 4], 2, 0.1), ([2, 2, 2], 2, 0.2),
                                         ([5, 3, 4], 3, 0.2), ([3, 2, 4], 4, 0.1)])
def test_velocity_block_on_every_level(n, k, noise):
    """A on every level of a 3D Taylor-Hood hierarchy (degree k, then the
    lower degrees without a pressure space, then coarser degree-1 meshes)
    against the oracle's level matrices, FP64 and FP32: for k = 2 several
    bricks and ragged brick tails; for k = 3, 4 the column kernel on the
    velocity-only degree-3 level and ragged last workgroups."""
    dim, nu = 3, 0.9
    h, X = _setup(dim, n, k, noise, nu, mg_levels=1)
    try:
        H = _oracle_hierarchy(dim, n, X, k, nu, 5)
        assert mfs.mfs_n_levels(h) == len(H.spaces)
        for l, S in enumerate(H.spaces):
            x = inputs.uniform_vector(dim * S.Nv, 70 + l)
            y = torch.empty(dim * S.Nv, dtype=torch.float64, device="cuda")
            mfs.mfs_vmult(h, mfs.MFS_OP_A, mfs.MFS_FP64, l, y, cuda(x))
            assert relerr(host(y), H.A[l] @ x) <= 1e-12, l
            x32 = x.astype(np.float32).astype(np.float64)
            y32 = torch.empty(dim * S.Nv, dtype=torch.float32, device="cuda")
            mfs.mfs_vmult(h, mfs.MFS_OP_A, mfs.MFS_FP32, l, y32, cuda(x32, torch.float32))
            assert relerr(host(y32), H.A[l] @ x32) <= 1e-5, l
    finally:
        mfs.mfs_destroy(h)


@pytest.mark.parametrize("dim,n,k,noise", MG_CASES)
def test_vcycle_and_block_preconditioner_fp64(dim, n, k, noise):
    nu = 1.3
    h, X = _setup(dim, n, k, noise, nu, mg_levels=1, cheb_degree=3, schur_iterations=7)
    try:
        sysm = krylov.StokesSystem(dim, n, X, k, nu, schur_iterations=7, cheb_degree=3)
        H = sysm.mg
        for l in range(len(H.spaces) - 1):
            H.lam[l] = 1.2 * H.exact_lambda_max(l)
            mfs.mfs_set_lambda(h, l, H.lam[l])
        S = sysm.S
        nvel = dim * S.Nv
        b = inputs.uniform_vector(nvel, 3)
        out = torch.empty(nvel, dtype=torch.float64, device="cuda")
        mfs.mfs_vcycle(h, mfs.MFS_FP64, out, cuda(b))
        assert relerr(host(out), H.vcycle(b)) <= 1e-11
        r = inputs.uniform_vector(S.n_dofs, 4)
        y = torch.empty(S.n_dofs, dtype=torch.float64, device="cuda")
        mfs.mfs_precondition(h, mfs.MFS_FP64, y, cuda(r))
        assert relerr(host(y), sysm.precondition(r)) <= 1e-11
        # FP32 preconditioner: same operator in single precision
        y32 = torch.empty(S.n_dofs, dtype=torch.float32, device="cuda")
        mfs.mfs_precondition(h, mfs.MFS_FP32, y32, cuda(r, torch.float32))
        assert relerr(host(y32), sysm.precondition(r)) <= 1e-4
    finally:
        mfs.mfs_destroy(h)


@pytest.mark.parametrize("n,cheb_degree", [([20, 12, 6], 3), ([16, 8, 4], 5)])
def test_vcycle_several_bricks(n, cheb_degree):
    """3D Q2 V-cycle on meshes of several bricks per direction with a ragged
    brick tail: the Chebyshev steps of the degree-2 and degree-1 levels run
    fused into the brick kernels (iterate updated in place, face nodes in the
    combine), in FP64 and FP32.  lambda_max by a sparse eigensolver, set on
    both sides."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as sla

    dim, k, nu = 3, 2, 1.1
    h, X = _setup(dim, n, k, 0.2, nu, mg_levels=1, cheb_degree=cheb_degree)
    try:
        H = mg.Hierarchy(dim, n, X, k, nu, cheb_degree=cheb_degree)
        assert mfs.mfs_n_levels(h) == len(H.spaces)
        for l in range(len(H.spaces) - 1):
            free = ~H.fixed[l]
            d = sp.diags(np.sqrt(H.Dinv[l][free]))
            B = d @ H.A[l][free][:, free] @ d
            H.lam[l] = 1.2 * float(sla.eigsh(B, k=1, which="LA", tol=1e-8)[0][0])
            mfs.mfs_set_lambda(h, l, H.lam[l])
        nvel = dim * H.spaces[0].Nv
        for seed in (3, 4):
            b = inputs.uniform_vector(nvel, seed)
            ref = H.vcycle(b)
            out = torch.empty(nvel, dtype=torch.float64, device="cuda")
            mfs.mfs_vcycle(h, mfs.MFS_FP64, out, cuda(b))
            assert relerr(host(out), ref) <= 1e-11
            out32 = torch.empty(nvel, dtype=torch.float32, device="cuda")
            mfs.mfs_vcycle(h, mfs.MFS_FP32, out32, cuda(b, torch.float32))
            assert relerr(host(out32), ref) <= 1e-4
    finally:
        mfs.mfs_destroy(h)


# ------------------------------------------------------------------ solves
def _ms_rhs_gpu(h, dim, n, k, S, nu):
    nq = (k + 1) ** dim
    q = mfs.mfs_quadrature_points(h, S.nc, nq, dim)
    ms = inputs.manufactured_2d if dim == 2 else inputs.manufactured_3d
    f = ms(q, nu)[2]
    uD = ms(mfs.mfs_support_points(h, k, S.Nv, dim), nu)[0]
    b = torch.empty(S.n_dofs, dtype=torch.float64, device="cuda")
    mfs.mfs_rhs(h, cuda(f), cuda(uD.T.ravel()), b)
    return b, f, uD


@pytest.mark.parametrize("dim,n,k", [(2, [16, 16], 2), (3, [4, 4, 4], 2), (3, [4, 4, 4], 3)])
def test_rhs_matches_oracle(dim, n, k):
    nu = 0.5
    h, X = _setup(dim, n, k, 0.2, nu, mg_levels=0)
    try:
        S = fem.Space(dim, n, X, k)
        b, f, uD = _ms_rhs_gpu(h, dim, n, k, S, nu)
        ref = solve.stokes_rhs(S, nu, f, uD)
        assert relerr(host(b), ref) <= 1e-12
    finally:
        mfs.mfs_destroy(h)


@pytest.mark.parametrize("prec", [mfs.MFS_FP64, mfs.MFS_FP32])
def test_solve_2d_q2q1_16x16(prec):
    """2D Q2/Q1 on the 16x16 unit square, nu = 1, manufactured solution,
    Chebyshev degree 3, FGMRES to 1e-10: compare with the oracle's exact
    solution and, for the FP64 preconditioner, its FGMRES iteration count."""
    dim, n, k, nu = 2, [16, 16], 2, 1.0
    X = inputs.structured_vertices(dim, n)
    opts = mfs.mfs_default_options(cheb_degree=3, rtol=1e-10, precond_precision=prec)
    h = mfs.mfs_setup(dim, n, X, k, nu, opts)
    try:
        S = fem.Space(dim, n, X, k)
        b, f, uD = _ms_rhs_gpu(h, dim, n, k, S, nu)
        x = torch.zeros_like(b)
        info = mfs.mfs_solve(h, b, x, opts)
        assert info.status == 0 and info.rel_residual <= 1e-10
        xs = host(x)
        mats = fem.assemble_stokes(S, nu)
        bref = solve.stokes_rhs(S, nu, f, uD, mats)
        xd = solve.pressure_mean_free(S, solve.direct_solve(S, nu, bref, mats), mats["M"])
        err = np.linalg.norm(xs - xd) / np.linalg.norm(xd)
        assert err <= 1e-8, err
        assert info.iterations <= 40
        if prec == mfs.MFS_FP64:
            sysm = krylov.StokesSystem(dim, n, X, k, nu, cheb_degree=3)
            for l in range(len(sysm.mg.spaces) - 1):
                sysm.mg.lam[l] = mfs.mfs_get_lambda(h, l)
            _, its, _ = krylov.fgmres(sysm.K, bref, sysm.precondition, krylov.lifting(sysm.mask, bref), rtol=1e-10)
            assert abs(its - info.iterations) <= 1
    finally:
        mfs.mfs_destroy(h)


def test_solve_3d_mixed_precision():
    dim, n, k, nu = 3, [8, 8, 8], 2, 1.0
    X = inputs.structured_vertices(dim, n, noise=0.2, seed=0)
    opts = mfs.mfs_default_options(rtol=1e-8, precond_precision=mfs.MFS_FP32)
    h = mfs.mfs_setup(dim, n, X, k, nu, opts)
    try:
        S = fem.Space(dim, n, X, k)
        b, f, uD = _ms_rhs_gpu(h, dim, n, k, S, nu)
        x = torch.zeros_like(b)
        info = mfs.mfs_solve(h, b, x, opts)
        assert info.status == 0 and info.rel_residual <= 1e-8
        mats = fem.assemble_stokes(S, nu)
        K = fem.constrain(mats["K"], S.velocity_dirichlet_mask())
        bref = solve.stokes_rhs(S, nu, f, uD, mats)
        xs = host(x)
        assert np.linalg.norm(bref - K @ xs) <= 1.01e-8 * np.linalg.norm(bref)
        xd = solve.pressure_mean_free(S, solve.direct_solve(S, nu, bref, mats), mats["M"])
        # error bound from the residual and the smallest eigenvalue of the
        # bordered system, both computed by the oracle
        bound, _ = bordered_error_bound(S, nu, bref, xs, mats)
        err = np.linalg.norm(xs - xd)
        print(f"3D 8^3 Q2/Q1 mixed-precision solve: error {err / np.linalg.norm(xd):.2e}, "
              f"bound {bound / np.linalg.norm(xd):.2e}")
        assert err <= 1.5 * bound + 1e-12 * np.linalg.norm(xd)
    finally:
        mfs.mfs_destroy(h)


def test_setup_in_caller_arena():
    """mfs_setup_arena carves the problem from a caller's uint8 tensor: the
    same operator and solve as mfs_setup, a too small arena is rejected, and
    destroying the problem leaves the arena to its owner."""
    dim, n, k, nu = 3, [4, 4, 4], 2, 0.6
    X = inputs.structured_vertices(dim, n, noise=0.2, seed=2)
    opts = mfs.mfs_default_options(rtol=1e-10, precond_precision=mfs.MFS_FP64)
    fp = mfs.mfs_footprint(dim, n, X, k, opts)
    small = torch.empty(fp - 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(mfs.MfsError) as e:
        mfs.mfs_setup_arena(dim, n, X, k, nu, small, opts)
    assert e.value.code == mfs.MFS_ENOMEM
    arena = torch.full((fp,), 7, dtype=torch.uint8, device="cuda")
    h1 = mfs.mfs_setup(dim, n, X, k, nu, opts)
    h2 = mfs.mfs_setup_arena(dim, n, X, k, nu, arena, opts)
    try:
        nv, np_ = mfs.mfs_n_dofs(h1, 0)
        x = cuda(inputs.uniform_vector(dim * nv + np_, 5))
        y1, y2 = torch.empty_like(x), torch.empty_like(x)
        mfs.mfs_vmult(h1, mfs.MFS_OP_STOKES, mfs.MFS_FP64, 0, y1, x)
        mfs.mfs_vmult(h2, mfs.MFS_OP_STOKES, mfs.MFS_FP64, 0, y2, x)
        torch.cuda.synchronize()
        assert torch.equal(y1, y2)
        s1, s2 = torch.zeros_like(x), torch.zeros_like(x)
        i1 = mfs.mfs_solve(h1, y1, s1, opts)
        i2 = mfs.mfs_solve(h2, y1, s2, opts)
        assert i1.iterations == i2.iterations and torch.equal(s1, s2)
    finally:
        mfs.mfs_destroy(h1)
        mfs.mfs_destroy(h2)
    arena.fill_(1)  # still the caller's memory
    torch.cuda.synchronize()
    assert int(arena.sum()) == fp

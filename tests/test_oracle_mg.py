"""Pins of the oracle's multigrid and Krylov pieces (Sec. 2 eq. (transfer),
Sec. 3 eq. (stokes_block)): polynomial reproduction and the Galerkin identity
of the transfer, the closed-form Chebyshev error polynomial, the two-step
convergence of FGMRES with the exact block preconditioner, and agreement of
the preconditioned FGMRES solution with a sparse direct solve."""
import numpy as np
import pytest
import scipy.linalg as la
import scipy.sparse as sp

import inputs
from oracle import basis, fem, krylov, mg, solve


def _poly_nodes(S, deg_per_dir, rng):
    """Nodal values of a random polynomial of degree deg in each direction."""
    pts = S.support_points()
    C = rng.standard_normal([deg_per_dir + 1] * S.dim)
    val = np.zeros(len(pts))
    for idx in np.ndindex(*C.shape):
        val += C[idx] * np.prod([pts[:, a] ** idx[a] for a in range(S.dim)], axis=0)
    return val


@pytest.mark.parametrize("dim,n,k,h", [(2, [2, 4], 2, True), (2, [3, 2], 3, False), (3, [2, 2, 2], 2, True),
                                       (3, [2, 1, 2], 3, False), (3, [2, 2, 2], 1, True)])
def test_transfer_reproduces_coarse_polynomials(dim, n, k, h):
    rng = np.random.default_rng(0)
    if h:
        Sc = fem.Space(dim, n, inputs.structured_vertices(dim, n), k, 0)
        nf = [2 * v for v in n]
        Sf = fem.Space(dim, nf, inputs.structured_vertices(dim, nf), k, 0)
    else:
        Sc = fem.Space(dim, n, inputs.structured_vertices(dim, n), k - 1, 0)
        Sf = fem.Space(dim, n, inputs.structured_vertices(dim, n), k, 0)
    P = mg.transfer_matrix(Sf, Sc, h, constrained=False)
    # a Q_kc polynomial interpolated on the coarse nodes prolongates exactly
    pts_c, pts_f = Sc.support_points(), Sf.support_points()
    C = rng.standard_normal([Sc.k + 1] * dim)

    def f(pts):
        v = np.zeros(len(pts))
        for idx in np.ndindex(*C.shape):
            v += C[idx] * np.prod([pts[:, a] ** idx[a] for a in range(dim)], axis=0)
        return v

    assert np.abs(P @ f(pts_c) - f(pts_f)).max() < 1e-12
    # constrained version: zero fine Dirichlet rows, zero coarse Dirichlet columns
    Pc = mg.transfer_matrix(Sf, Sc, h)
    assert abs(Pc[Sf.dirichlet]).max() == 0
    assert abs(Pc[:, Sc.dirichlet]).max() == 0


@pytest.mark.parametrize("dim,n,k,h", [(2, [2, 2], 2, True), (2, [2, 3], 3, False), (3, [2, 2, 2], 2, True),
                                       (3, [2, 2, 2], 3, False)])
def test_galerkin_identity_affine(dim, n, k, h):
    """R A_f P = A_c for nested affine meshes with exact quadrature."""
    A_vtx = np.array([[1.3, 0.2, 0.1], [-0.1, 0.9, 0.2], [0.15, -0.2, 1.1]])[:dim, :dim]
    if h:
        nf = [2 * v for v in n]
        Xc = inputs.structured_vertices(dim, n) @ A_vtx.T
        Xf = inputs.structured_vertices(dim, nf) @ A_vtx.T
        Sc, Sf = fem.Space(dim, n, Xc, k, 0), fem.Space(dim, nf, Xf, k, 0)
    else:
        X = inputs.structured_vertices(dim, n) @ A_vtx.T
        Sc, Sf = fem.Space(dim, n, X, k - 1, 0), fem.Space(dim, n, X, k, 0)
    P = mg.transfer_matrix(Sf, Sc, h, constrained=False)
    Af = mg._laplace_only(Sf, 0.7)
    Ac = mg._laplace_only(Sc, 0.7)
    G = (P.T @ Af @ P).toarray()
    assert np.abs(G - Ac.toarray()).max() < 1e-12 * np.abs(Ac.toarray()).max()


def test_chebyshev_closed_form():
    lam = np.linspace(0.05, 1.9, 37)
    A = sp.diags(lam).tocsr()
    x_true = np.random.default_rng(1).standard_normal(len(lam))
    b = A @ x_true
    fixed = np.zeros(len(lam), dtype=bool)
    for deg in (1, 3, 5):
        x = mg.chebyshev_smooth(A, np.ones(len(lam)), fixed, 2.0, 20.0, deg, np.zeros(len(lam)), b, True)
        e = x - x_true
        pd = mg.chebyshev_error_polynomial(lam, 2.0, 20.0, deg)
        assert np.allclose(e, pd * (-x_true), atol=1e-13)


def test_vcycle_contracts():
    dim, n, k = 2, [8, 8], 2
    X = inputs.structured_vertices(dim, n, noise=0.2, seed=4)
    H = mg.Hierarchy(dim, n, X, k, 1.0, cheb_degree=3)
    for l in range(len(H.spaces) - 1):
        H.lam[l] = 1.2 * H.exact_lambda_max(l)
    A = H.A[0]
    rng = np.random.default_rng(0)
    # error propagation of the V-cycle as a stationary iteration
    e = rng.standard_normal(A.shape[0])
    e[H.fixed[0]] = 0
    nrm0 = np.sqrt(e @ (A @ e))
    for _ in range(5):
        e = e - H.vcycle(A @ e)
    assert np.sqrt(e @ (A @ e)) / nrm0 < 0.3 ** 5


def test_exact_block_preconditioner_two_iterations():
    """With exact A^{-1} and S^{-1} (S = B^T A^{-1} B, pseudo-inverse on the
    mean-free pressures), (K P^{-1} - I)^2 = 0: FGMRES stops after 2 steps."""
    dim, n, k = 2, [3, 3], 2
    X = inputs.structured_vertices(dim, n, noise=0.2, seed=2)
    sysm = krylov.StokesSystem(dim, n, X, k, 1.0)
    nu_ = sysm.nvel
    A = sysm.K[:nu_, :nu_].toarray()
    B = sysm.B.toarray()
    Ainv = la.inv(A)
    Sm = B.T @ Ainv @ B
    Sp = la.pinv(Sm, rtol=1e-12)
    pre = lambda r: sysm.precondition(r, vcycle=lambda t: Ainv @ t, schur=lambda rp: -(Sp @ rp))
    xq = sysm.S.geometry()[0]
    _, _, f = inputs.manufactured_2d(xq)
    uD = inputs.manufactured_2d(sysm.S.support_points())[0]
    b = solve.stokes_rhs(sysm.S, 1.0, f, uD, sysm.mats)
    x, its, rel = krylov.fgmres(sysm.K, b, pre, krylov.lifting(sysm.mask, b), rtol=1e-10)
    assert its <= 2 and rel <= 1e-10


@pytest.mark.parametrize("dim,n,k", [(2, [8, 8], 2), (3, [4, 4, 4], 2)])
def test_fgmres_matches_direct_solve(dim, n, k):
    X = inputs.structured_vertices(dim, n, noise=0.2, seed=7)
    sysm = krylov.StokesSystem(dim, n, X, k, 1.0, cheb_degree=3)
    H = sysm.mg
    for l in range(len(H.spaces) - 1):
        H.lam[l] = 1.2 * H.exact_lambda_max(l)
    xq = sysm.S.geometry()[0]
    ms = inputs.manufactured_2d if dim == 2 else inputs.manufactured_3d
    _, _, f = ms(xq)
    uD = ms(sysm.S.support_points())[0]
    b = solve.stokes_rhs(sysm.S, 1.0, f, uD, sysm.mats)
    x, its, rel = krylov.fgmres(sysm.K, b, sysm.precondition, krylov.lifting(sysm.mask, b), rtol=1e-12)
    assert rel <= 1e-12 and its < 80
    x = solve.pressure_mean_free(sysm.S, x, sysm.M)
    xd = solve.pressure_mean_free(sysm.S, solve.direct_solve(sysm.S, 1.0, b, sysm.mats), sysm.M)
    assert np.linalg.norm(x - xd) <= 1e-8 * np.linalg.norm(xd)

"""Pins of the oracle's monolithic Navier-Stokes multigrid (Sec. 5): level
order, interpolation of the linearisation point, unconstrained pressure
transfer, the singular Jacobian and its pinned coarse solve, the smoother's
fixed point, V-cycle contraction and GMRES against a sparse direct solve."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import inputs
from oracle import basis, ns, ns_mg
from oracle.fem import Space
from oracle.mg import transfer_matrix


def _u0(S, seed=3):
    P = S.support_points()
    P3 = np.concatenate([P, np.full((P.shape[0], 3 - S.dim), 0.3)], 1)
    return inputs.fourier_field(seed)(P3)[:, :S.dim].T.ravel()


def _hier(dim, n, k, nu=1e-2, cfl=1.0, noise=0.1, newton=True):
    X = inputs.structured_vertices(dim, [n] * dim, noise=noise, seed=1)
    S = Space(dim, [n] * dim, X, k, k)
    u0 = _u0(S)
    dt = cfl / (n * k) / np.abs(u0).max()
    return ns_mg.NSHierarchy(dim, [n] * dim, X, k, nu, dt, u0, newton=newton), S


def test_level_order_h_then_p():
    assert ns_mg.ns_level_specs([8, 8], 2) == [([8, 8], 2, 0), ([4, 4], 2, 1), ([2, 2], 2, 2), ([2, 2], 1, 2)]
    assert ns_mg.ns_level_specs([6, 4, 4], 1) == [([6, 4, 4], 1, 0), ([3, 2, 2], 1, 1)]


@pytest.mark.parametrize("dim,k", [(2, 1), (2, 2), (3, 2)])
def test_reference_positions_are_support_points_of_the_unit_cube(dim, k):
    S = Space(dim, [3] * dim, inputs.structured_vertices(dim, [3] * dim), k, k)
    np.testing.assert_allclose(ns_mg._reference_positions(S, k), S.support_points(k), atol=1e-15)


@pytest.mark.parametrize("dim,k,h", [(2, 1, True), (2, 2, True), (3, 2, True), (2, 2, False), (3, 2, False)])
def test_interpolation_copies_values_at_shared_nodes(dim, k, h):
    n = [4] * dim
    X = inputs.structured_vertices(dim, n)
    Sf = Space(dim, n, X, k, k)
    Sc = Space(dim, [2] * dim, inputs.coarsen_vertices(dim, n, X, 1), k, k) if h else Space(dim, n, X, k - 1, k - 1)
    f = lambda x: np.stack([np.sin(3 * x[:, 0] + x[:, 1]), np.cos(x.sum(1)), x[:, 0] * x[:, -1]][:dim])  # noqa
    uf = f(Sf.support_points()).ravel()
    uc = ns_mg.interpolate_velocity(Sf, Sc, uf)
    np.testing.assert_allclose(uc, f(Sc.support_points()).ravel(), atol=1e-14)


def test_interpolation_rejects_non_nested_nodes():
    X = inputs.structured_vertices(2, [4, 4])
    with pytest.raises(ValueError):
        ns_mg.interpolate_velocity(Space(2, [4, 4], X, 3, 3), Space(2, [4, 4], X, 2, 2), np.zeros(2 * 13 * 13))


@pytest.mark.parametrize("h", [True, False])
def test_unconstrained_transfer_reproduces_coarse_polynomials_on_the_boundary(h):
    dim, k = 2, 2
    n = [4, 4]
    X = inputs.structured_vertices(dim, n, noise=0.1, seed=2)
    Sf = Space(dim, n, X, k, k)
    Sc = Space(dim, [2, 2], inputs.coarsen_vertices(dim, n, X, 1), k, k) if h else Space(dim, n, X, 1, 1)
    P = transfer_matrix(Sf, Sc, h, constrained=False)
    # a polynomial of the coarse degree in reference coordinates
    pc, pf = ns_mg._reference_positions(Sc, Sc.k), ns_mg._reference_positions(Sf, Sf.k)
    g = lambda x: (1 + x[:, 0] - 2 * x[:, 1] + 3 * x[:, 0] * x[:, 1]) if Sc.k == 1 else (x[:, 0] ** 2 * x[:, 1] - x[:, 1] ** 2)  # noqa
    if h:
        # piecewise polynomial on the coarse cells of width 1/2 is the coarse interpolant itself
        y = P @ g(pc)
        yf = g(pf)
        assert np.abs(y - yf).max() < 1e-13
    else:
        np.testing.assert_allclose(P @ g(pc), g(pf), atol=1e-13)
    bnd = Sf.dirichlet
    assert np.abs((P @ g(pc))[bnd]).max() > 0.1  # boundary rows are not zeroed


def test_constant_pressure_is_the_kernel_and_pressure_rows_sum_to_zero():
    H, S = _hier(2, 6, 2)
    J = H.J[0]
    d = S.dim * S.Nv
    e = np.zeros(J.shape[0])
    e[d:] = 1.0
    assert np.abs(J @ e).max() < 1e-12 * abs(J).max()
    rng = np.random.default_rng(1)
    x = rng.standard_normal(J.shape[0])
    x[H.fixed[0]] = 0.0
    y = J @ x
    assert abs(y[d:].sum()) < 1e-12 * np.abs(y).sum()


def test_pinned_coarse_solve_returns_a_solution_with_zero_pin():
    H, S = _hier(2, 4, 2)
    Jc = H.J[-1]
    rng = np.random.default_rng(4)
    xt = rng.standard_normal(Jc.shape[0])
    xt[H.fixed[-1]] = 0.0
    b = Jc @ xt
    x = H.coarse_solve(b)
    assert abs(x[H.pin]) == 0.0
    d = H.dim * H.spaces[-1].Nv
    np.testing.assert_allclose(x[:d], xt[:d], atol=1e-10)
    np.testing.assert_allclose(x[d:] - x[d:].mean(), xt[d:] - xt[d:].mean(), atol=1e-10)
    np.testing.assert_allclose(Jc @ x, b, atol=1e-10 * np.abs(b).max())


def test_relaxation_fixed_point_and_dirichlet_rows():
    H, S = _hier(2, 4, 1)
    rng = np.random.default_rng(5)
    x = rng.standard_normal(H.J[0].shape[0])
    b = H.J[0] @ x
    np.testing.assert_allclose(H.relax(0, x, b), x, atol=1e-12)
    # Dirichlet rows of the constrained J are identity rows: D = 1 there
    assert np.all(H.Dinv[0][H.fixed[0]] == 1.0)


@pytest.mark.parametrize("dim,n,k", [(2, 16, 1), (2, 8, 2), (3, 4, 2)])
def test_vcycle_contracts(dim, n, k):
    H, S = _hier(dim, n, k, nu=1e-3)
    rng = np.random.default_rng(6)
    xt = rng.standard_normal(H.J[0].shape[0])
    xt[H.fixed[0]] = 0.0
    b = H.J[0] @ xt
    x = np.zeros_like(b)
    d = dim * S.Nv

    def err(x):
        e = x - xt
        e[d:] -= e[d:].mean()
        return np.linalg.norm(e)

    e0 = err(x)
    for _ in range(6):
        x = x + H.vcycle(b - H.J[0] @ x)
    assert err(x) < 0.5 ** 6 * e0


@pytest.mark.parametrize("dim,n,k,newton", [(2, 8, 2, True), (2, 8, 2, False), (3, 4, 1, True), (3, 4, 2, True)])
def test_gmres_matches_direct_solve(dim, n, k, newton):
    H, S = _hier(dim, n, k, nu=2.5e-4, newton=newton)
    J = H.J[0].tolil()
    rng = np.random.default_rng(7)
    xt = rng.standard_normal(J.shape[0])
    xt[H.fixed[0]] = 0.0
    b = H.J[0] @ xt
    x, its, rel = ns_mg.solve(H, b, rtol=1e-12, maxit=100)
    assert rel <= 1e-12 and its <= 40
    # direct: fix pressure node 0 of the finest level, then remove the mean
    p0 = dim * S.Nv
    J[p0, :] = 0.0
    J[:, p0] = 0.0
    J[p0, p0] = 1.0
    bb = b.copy()
    bb[p0] = 0.0
    xd = ns_mg.zero_mean_pressure(S, spla.spsolve(J.tocsc(), bb))
    np.testing.assert_allclose(x, xd, atol=1e-8 * np.abs(xd).max())
    np.testing.assert_allclose(x, ns_mg.zero_mean_pressure(S, xt), atol=1e-8 * np.abs(xt).max())


def test_iterations_bounded_under_refinement():
    its = []
    for n in (8, 16):
        H, S = _hier(2, n, 1, nu=1e-3)
        rng = np.random.default_rng(8)
        xt = rng.standard_normal(H.J[0].shape[0])
        xt[H.fixed[0]] = 0.0
        its.append(ns_mg.solve(H, H.J[0] @ xt, rtol=1e-8)[1])
    assert max(its) <= 15 and its[1] <= its[0] + 3


def test_gll_of_degree_two_is_nested_in_degree_two_children():
    # the injection reading relies on the coarse degree-2 nodes (0, 1/2, 1)
    # being fine nodes of the two children at degree 2
    g = basis.gll_points(2)
    fine = np.concatenate([0.5 * g, 0.5 + 0.5 * g[1:]])
    assert all(np.isclose(fine, v).any() for v in g)

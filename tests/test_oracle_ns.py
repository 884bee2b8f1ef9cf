"""Pins of the oracle's stabilised Navier-Stokes residual and Jacobian
(Sec. 5): central finite differences of the nonlinear residual, the matrix
against the matrix-free application, the u0 = 0 special case against the
Stokes-type blocks built independently, the pressure null vector, and the
vanishing Laplacian of Q1 on affine cells."""
import numpy as np
import pytest

import inputs
from oracle import fem, ns


def _setup(dim, n, k, noise=0.0, seed=1):
    X = inputs.structured_vertices(dim, n, noise=noise, seed=seed)
    S = fem.Space(dim, n, X, k, kp=k)
    rng = np.random.default_rng(seed)
    u0 = np.zeros(dim * S.Nv + S.Nv)
    u0[: dim * S.Nv] = rng.uniform(-1, 1, dim * S.Nv)
    return S, u0


@pytest.mark.parametrize("dim,n,k,noise,newton", [(2, [3, 2], 1, 0.2, True), (2, [2, 2], 2, 0.1, True),
                                                  (3, [2, 2, 1], 1, 0.0, True), (3, [2, 1, 2], 2, 0.1, True)])
def test_jacobian_is_derivative_of_residual(dim, n, k, noise, newton):
    nu, dt = 0.05, 0.1
    S, u0 = _setup(dim, n, k, noise)
    data = ns.linearization_data(S, u0[: dim * S.Nv], nu, dt)
    d = np.random.default_rng(7).uniform(-1, 1, u0.shape)
    J = ns.jacobian_apply(S, d, data, nu, dt, newton)
    errs = []
    for eps in (1e-2, 1e-3):
        fd = (ns.residual(S, u0 + eps * d, u0[: dim * S.Nv], nu, dt, data)
              - ns.residual(S, u0 - eps * d, u0[: dim * S.Nv], nu, dt, data)) / (2 * eps)
        errs.append(np.abs(fd - J).max() / np.abs(J).max())
    # second-order convergence of the central difference (or exact: quadratic residual)
    assert errs[1] < 1e-8 or errs[0] / errs[1] > 50, errs


def test_residual_zero_at_rest_and_matrix_consistency():
    dim, n, k, nu, dt = 3, [2, 2, 2], 2, 0.01, 0.01
    S, u0 = _setup(dim, n, k, 0.1)
    data = ns.linearization_data(S, u0[: dim * S.Nv], nu, dt)
    # u = 0, p = 0 with u0 = 0 is a solution
    z = np.zeros_like(u0)
    d0 = ns.linearization_data(S, z[: dim * S.Nv], nu, dt)
    assert np.abs(ns.residual(S, z, z[: dim * S.Nv], nu, dt, d0)).max() == 0.0
    for newton in (True, False):
        K = ns.jacobian_matrix(S, data, nu, dt, newton)
        x = np.random.default_rng(3).uniform(-1, 1, u0.shape)
        y1 = K @ x
        y2 = ns.constrained_jacobian_apply(S, x, data, nu, dt, newton)
        assert np.abs(y1 - y2).max() <= 1e-12 * np.abs(y2).max()


def test_pressure_constants_in_kernel():
    dim, n, k, nu, dt = 3, [2, 3, 2], 2, 0.01, 0.01
    S, u0 = _setup(dim, n, k, 0.15)
    data = ns.linearization_data(S, u0[: dim * S.Nv], nu, dt)
    one = np.zeros_like(u0)
    one[dim * S.Nv:] = 1.0
    y = ns.constrained_jacobian_apply(S, one, data, nu, dt)
    mask = ns.ns_dirichlet_mask(S)
    assert np.abs(y[~mask]).max() < 1e-12


def test_u0_zero_reduces_to_stokes_blocks():
    """u0 = 0 on a uniform Cartesian mesh: J = [[alpha M + nu A, B], [-B^T, D]]
    plus the PSPG coupling, with D = delta (grad p, grad q) and delta constant."""
    dim, n, k, nu, dt = 2, [3, 3], 2, 0.2, 0.05
    X = inputs.structured_vertices(dim, n)
    S = fem.Space(dim, n, X, k, kp=k)
    z = np.zeros(dim * S.Nv)
    data = ns.linearization_data(S, z, nu, dt)
    delta = data["delta"]
    assert np.ptp(delta) < 1e-14 * delta.max()
    K = ns.jacobian_matrix(S, data, nu, dt)
    mats = fem.assemble_stokes(S, 1.0)  # A (nu = 1), B, M (pressure mass, here = velocity mass)
    mask = ns.ns_dirichlet_mask(S)
    free = ~mask
    nv = dim * S.Nv
    alpha = 1.5 / dt
    Mu = fem.sp.block_diag([mats["M"]] * dim).tocsr()
    Avec = mats["Avec"]
    Kuu = (alpha * Mu + nu * Avec).toarray()
    Kd = K.toarray()
    fu = free[:nv]
    assert np.abs(Kd[:nv, :nv][np.ix_(fu, fu)] - Kuu[np.ix_(fu, fu)]).max() < 1e-12 * np.abs(Kuu).max()
    assert np.abs(Kd[:nv, nv:][fu] - mats["B"].toarray()[fu]).max() < 1e-12
    Dp = delta.max() * mats["A"].toarray()
    assert np.abs(Kd[nv:, nv:] - Dp).max() < 1e-12 * np.abs(Dp).max()


def test_q1_laplacian_vanishes_on_affine_cells():
    X = inputs.structured_vertices(3, [2, 2, 2]) * np.array([1.0, 0.5, 2.0])
    S = fem.Space(3, [2, 2, 2], X, 1, kp=1)
    N, G, L, JxW, vol = ns._qp_data(S)
    assert np.abs(L).max() < 1e-12


def test_sampled_rows_equal_full_evaluation():
    X = inputs.structured_vertices(3, [3, 2, 3], noise=0.2, seed=5)
    S = fem.Space(3, [3, 2, 3], X, 2, 2)
    rng = np.random.default_rng(2)
    u0 = rng.uniform(-1, 1, 3 * S.Nv)
    dx = rng.uniform(-1, 1, 4 * S.Nv)
    data = ns.linearization_data(S, u0, 0.05, 0.1)
    full = ns.constrained_jacobian_apply(S, dx, data, 0.05, 0.1)
    rows = rng.choice(4 * S.Nv, 40, replace=False)
    np.testing.assert_allclose(ns.sampled_jacobian_rows(S, dx, u0, 0.05, 0.1, rows), full[rows], rtol=0,
                               atol=1e-13 * np.abs(full).max())

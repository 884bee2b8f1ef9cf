"""Pins of the oracle's space-time Kronecker operator (Sec. 4
eq. (proceedings-kronecker)): the DG(k) time matrices against the known
stability functions of DG time stepping (the (k, k+1) Pade approximants of
exp(-z), independent of the temporal basis), DG(0) as backward Euler, the
stage-wise application against the assembled Kronecker matrix, and the
temporal transfer against polynomial reproduction."""
import math

import numpy as np
import pytest

import inputs
from oracle import fem, spacetime


def _pade_sub(k, z):
    """(k, k+1) Pade approximant of exp(-z)."""
    m, n = k, k + 1
    num = sum(math.factorial(m + n - j) * math.factorial(m) / (math.factorial(m + n) * math.factorial(j)
                                                                 * math.factorial(m - j)) * (-z) ** j
              for j in range(m + 1))
    den = sum(math.factorial(m + n - j) * math.factorial(n) / (math.factorial(m + n) * math.factorial(j)
                                                                 * math.factorial(n - j)) * z ** j
              for j in range(n + 1))
    return num / den


def test_pade_table_by_hand():
    z = 0.7
    assert abs(_pade_sub(0, z) - 1 / (1 + z)) < 1e-15
    assert abs(_pade_sub(1, z) - (1 - z / 3) / (1 + 2 * z / 3 + z * z / 6)) < 1e-15
    assert abs(_pade_sub(2, z) - (1 - 0.4 * z + 0.05 * z * z) / (1 + 0.6 * z + 0.15 * z * z + z ** 3 / 60)) < 1e-15


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_dg_time_step_stability_function(k):
    """y' = -lambda y over one slab: (G + z I) Y = M_Q^-1 m y0 (z = lambda tau);
    the end value e . Y is the (k, k+1) Pade approximant of exp(-z) times y0."""
    MQ, AQ, m, e = spacetime.time_matrices(k)
    G = spacetime.G_matrix(k)
    assert np.allclose(MQ @ G, AQ, atol=1e-13)
    for z in (0.05, 0.3, 1.0, 4.0):
        Y = np.linalg.solve(G + z * np.eye(k + 1), np.linalg.solve(MQ, m))
        assert abs(e @ Y - _pade_sub(k, z)) < 1e-13


def test_dg0_is_backward_euler():
    MQ, AQ, m, e = spacetime.time_matrices(0)
    assert np.allclose([MQ[0, 0], AQ[0, 0], m[0], e[0]], 1.0)
    n, k, nu, tau = [2, 3], 2, 0.4, 0.05
    S = fem.Space(2, n, inputs.structured_vertices(2, n, noise=0.1, seed=1), k)
    mats = fem.assemble_stokes(S, nu)
    K = spacetime.kron_operator(S, nu, tau, np.array([[1.0]]), mats)
    ref = fem.constrain(spacetime.block_mass(S, mats) + tau * mats["K"], S.velocity_dirichlet_mask())
    assert abs(K - ref).max() < 1e-14


@pytest.mark.parametrize("dim,n,k,q", [(2, [3, 2], 2, 2), (3, [2, 2, 1], 2, 3), (2, [2, 2], 3, 2)])
def test_stagewise_apply_equals_assembled_kronecker(dim, n, k, q):
    nu, tau = 0.3, 0.02
    S = fem.Space(dim, n, inputs.structured_vertices(dim, n, noise=0.15, seed=2), k)
    G = spacetime.G_matrix(q - 1)
    x = inputs.uniform_vector(q * S.n_dofs, 4)
    y = spacetime.kron_apply(S, nu, tau, G, x)
    K = spacetime.kron_operator(S, nu, tau, G)
    assert np.abs(y - K @ x).max() <= 1e-13 * np.abs(y).max()


def test_velocity_mass_integrates_polynomials():
    """1^T M_u 1 is the area; (x, 1) is the first moment (affine cells)."""
    n = [3, 2]
    A = np.array([[1.2, 0.3], [-0.1, 0.9]])
    X = inputs.structured_vertices(2, n) @ A.T
    S = fem.Space(2, n, X, 2)
    M = spacetime.velocity_mass(S)
    one = np.ones(S.Nv)
    assert abs(one @ M @ one - abs(np.linalg.det(A))) < 1e-13
    x = S.support_points()[:, 0]
    centroid_x = (A @ np.array([0.5, 0.5]))[0]
    assert abs(one @ M @ x - abs(np.linalg.det(A)) * centroid_x) < 1e-13


@pytest.mark.parametrize("kf,kc", [(1, 0), (2, 1), (3, 2), (3, 1)])
def test_time_prolongation_reproduces_polynomials(kf, kc):
    P = spacetime.time_prolongation(kf, kc)
    sf, sc = spacetime.time_nodes(kf), spacetime.time_nodes(kc)
    for d in range(kc + 1):
        assert np.allclose(P @ sc ** d, sf ** d, atol=1e-13)


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_package_stage_matrices_equal_the_oracle(k):
    """The host-side DG(k) matrices the package hands to the library."""
    from paper_2603_29621_amd import spacetime as pst

    G, MQ, AQ, m, e = pst.dg_stage_matrices(k)
    MQo, AQo, mo, eo = spacetime.time_matrices(k)
    assert np.allclose(G, spacetime.G_matrix(k), atol=1e-12)
    assert np.allclose(MQ, MQo, atol=1e-14) and np.allclose(AQ, AQo, atol=1e-12)
    assert np.allclose(m, mo, atol=1e-13) and np.allclose(e, eo, atol=1e-13)
    if k > 0:
        assert np.allclose(pst.stage_prolongation(k, k - 1), spacetime.time_prolongation(k, k - 1), atol=1e-13)

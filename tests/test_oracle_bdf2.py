"""Pins of the oracle's BDF2/Newton time stepping (Sec. 5): the BDF2 history
term against the symbolic weak form with distinct u^n and u^{n-1}, the
Jacobian at a general state (nonzero pressure, u != u~) against central
differences of the residual, quadratic convergence of Newton's method, and
the constant-pressure invariance of the residual."""
import numpy as np
import pytest
import sympy

import inputs
from oracle import bdf2, fem, ns
from test_oracle_pins import _cell, _oracle_space, _poly, _weak_form


@pytest.mark.parametrize("dim", [2, 3])
def test_bdf2_history_against_symbolic_weak_form(dim):
    """u in P1, p in P2, u^n and u^{n-1} distinct quadratics, delta_1
    constant: the residual with u~ = (4 u^n - u^{n-1}) / 3 equals the exact
    integral of the weak form with (3 u - 4 u^n + u^{n-1}) / (2 dt)."""
    C = _cell(dim)
    rng = np.random.default_rng(500 + dim)
    nu, dt, dl = 0.21, 0.4, 0.09
    R_ = sympy.Rational
    u = [_poly(C.X, 1, rng) for _ in range(dim)]
    p = _poly(C.X, 2, rng)
    un = [_poly(C.X, 2, rng) for _ in range(dim)]
    unm1 = [_poly(C.X, 2, rng) for _ in range(dim)]
    I, ph = _weak_form(C.X, u, p, un, unm1, u, R_(9, 100), R_(21, 100), R_(2, 5))
    ref = C.element_vector(I, *ph)
    S = _oracle_space(C)
    uh = bdf2.history(np.concatenate([C.nodal(f) for f in un]), np.concatenate([C.nodal(f) for f in unm1]))
    x = np.concatenate([C.nodal(f) for f in u] + [C.nodal(p)])
    data = bdf2.residual_data(S, uh, np.full((1, (3) ** dim), dl), nu, dt)
    got = ns.residual(S, x, None, nu, dt, data)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def _state(dim, n, k, noise, seed):
    X = inputs.structured_vertices(dim, n, noise=noise, seed=seed)
    S = fem.Space(dim, n, X, k, kp=k)
    rng = np.random.default_rng(seed)
    nv = dim * S.Nv
    x = rng.uniform(-1, 1, nv + S.Nv)
    x[ns.ns_dirichlet_mask(S)] = rng.uniform(-0.5, 0.5, int(ns.ns_dirichlet_mask(S).sum()))
    uh = rng.uniform(-1, 1, nv)
    un = rng.uniform(-1, 1, nv)
    return S, x, uh, un


@pytest.mark.parametrize("dim,n,k,noise", [(2, [3, 2], 1, 0.2), (2, [2, 2], 2, 0.1), (3, [2, 1, 2], 2, 0.1),
                                           (3, [2, 2, 1], 1, 0.0)])
def test_jacobian_at_a_general_state_is_the_derivative(dim, n, k, noise):
    nu, dt = 0.03, 0.05
    S, x, uh, un = _state(dim, n, k, noise, 11)
    delta = bdf2.frozen_delta(S, un, nu, dt)
    data = bdf2.point_data(S, x, uh, delta, nu, dt)
    mask = ns.ns_dirichlet_mask(S)
    d = np.random.default_rng(12).uniform(-1, 1, x.shape)
    d[mask] = 0.0  # the Newton update keeps the Dirichlet values
    J = ns.constrained_jacobian_apply(S, d, data, nu, dt, True)
    errs = []
    for eps in (1e-2, 1e-3):
        fd = (bdf2.residual(S, x + eps * d, uh, delta, nu, dt) - bdf2.residual(S, x - eps * d, uh, delta, nu, dt)) / (
            2 * eps)
        errs.append(np.abs(fd - J)[~mask].max() / np.abs(J).max())
    assert errs[1] < 1e-8 or errs[0] / errs[1] > 50, errs


def test_residual_invariant_under_pressure_constants():
    nu, dt = 0.02, 0.1
    S, x, uh, un = _state(3, [2, 2, 2], 2, 0.15, 3)
    delta = bdf2.frozen_delta(S, un, nu, dt)
    y = x.copy()
    y[3 * S.Nv:] += 2.5
    a, b = bdf2.residual(S, x, uh, delta, nu, dt), bdf2.residual(S, y, uh, delta, nu, dt)
    assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()


def test_newton_converges_quadratically_over_three_steps():
    n, k, nu, dt = [3, 3, 3], 2, 0.01, 0.01
    S = fem.Space(3, n, inputs.structured_vertices(3, n), k, kp=k)
    u = inputs.ns_velocity(3, [k * n[0] + 1] * 3, seed=0)
    states, hists = bdf2.bdf2(S, u, nu, dt, 3)
    for h in hists:
        assert h[-1] <= 1e-10 * h[0]
        # quadratic: e_{k+1} <= C e_k^2 once in the basin (C from the first pair)
        for a, b in zip(h[1:-1], h[2:]):
            assert b <= 10.0 * a * a / h[0] + 1e-13 * h[0], h
    for x in states:
        assert abs(x[3 * S.Nv:].mean()) < 1e-12
        assert np.all(x[ns.ns_dirichlet_mask(S)] == 0.0)

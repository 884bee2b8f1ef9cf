"""BDF2 time stepping with Newton's method for the stabilised Navier-Stokes
equations (oracle; test infrastructure only), Sec. 5.

Each time step solves F(u, p) = 0 for the new state, where F is the SUPG/PSPG
residual of `ns.residual` with the BDF2 time derivative
    (3 u - 4 u^n + u^{n-1}) / (2 dt) = alpha (u - u~),
    alpha = 3 / (2 dt),  u~ = (4 u^n - u^{n-1}) / 3,
by Newton's method: x_{k+1} = x_k - J(x_k)^{-1} F(x_k), J the Gateaux
derivative of F (`ns.jacobian_apply` at the point x_k, with the full strong
residual R(u_k, p_k) = alpha (u_k - u~) + u_k . grad u_k + grad p_k
- nu Lap u_k in its streamline term).

Readings where the paper is silent:
* delta_1 is frozen for the whole time step at the velocity u^n of the last
  step (the Tezduyar form of `ns.linearization_data`), so the Jacobian is the
  exact derivative of the residual the step solves;
* velocity Dirichlet values on the whole boundary are those of the iterate
  (the caller puts the boundary data of the new time level there); the
  Newton update vanishes on them and F is 0 on their rows;
* the pressure is fixed by a zero nodal mean;
* the first step uses u^{n-1} = u^n (no earlier state).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import ns
from .fem import Space


def history(u_n: np.ndarray, u_nm1: np.ndarray) -> np.ndarray:
    """u~ = (4 u^n - u^{n-1}) / 3, so that the BDF2 derivative is alpha (u - u~)."""
    return (4.0 * u_n - u_nm1) / 3.0


def frozen_delta(S: Space, u: np.ndarray, nu: float, dt: float, cells=None) -> np.ndarray:
    """delta_1 per Gauss point from the velocity u (blocked nodal, dim*Nv)."""
    return ns.linearization_data(S, u, nu, dt, cells)["delta"]


def residual_data(S: Space, u_hist: np.ndarray, delta: np.ndarray, nu: float, dt: float, cells=None):
    """Data for `ns.residual`: the history u~ at the Gauss points (its time
    term reads "u") and the frozen delta_1."""
    d = ns.linearization_data(S, u_hist, nu, dt, cells)
    d["delta"] = delta
    return d


def point_data(S: Space, x: np.ndarray, u_hist: np.ndarray, delta: np.ndarray, nu: float, dt: float):
    """Linearisation data at the state x = [u; p]: u, grad u and the full
    strong residual R(u, p) at the Gauss points, and the frozen delta_1."""
    d = ns.linearization_data(S, x[: S.dim * S.Nv], nu, dt)
    hist = ns.linearization_data(S, u_hist, nu, dt)["u"]
    _, _, _, _, gp = ns._local_fields(S, d, x)
    alpha = 1.5 / dt
    # linearization_data's R0 is u . grad u - nu Lap u; add the time and pressure terms
    d["R0"] = d["R0"] + alpha * (d["u"] - hist) + gp
    d["delta"] = delta
    return d


def residual(S: Space, x, u_hist, delta, nu, dt):
    """F(x) with Dirichlet rows 0 (the constrained nonlinear residual)."""
    F = ns.residual(S, x, None, nu, dt, residual_data(S, u_hist, delta, nu, dt))
    F[ns.ns_dirichlet_mask(S)] = 0.0
    return F


def _pinned_solve(K, rhs, pin):
    """Solve the singular Jacobian system with pressure unknown `pin` fixed to
    0 (its row and column replaced by the identity); the pressure rows of the
    right-hand side sum to zero, so this is a solution of the full system."""
    K = K.tolil()
    K[pin, :] = 0.0
    K[:, pin] = 0.0
    K[pin, pin] = 1.0
    r = rhs.copy()
    r[pin] = 0.0
    return spla.spsolve(K.tocsc(), r)


def newton(S: Space, x0, u_hist, delta, nu, dt, rtol=1e-10, maxit=20, newton=True):
    """Newton's method for F(x) = 0 from x0 (whose Dirichlet rows are kept):
    returns (x, [||F(x_k)||_2 for every iterate])."""
    x = x0.copy()
    nv = S.dim * S.Nv
    norms = []
    for _ in range(maxit + 1):
        F = residual(S, x, u_hist, delta, nu, dt)
        norms.append(float(np.linalg.norm(F)))
        if norms[-1] <= rtol * norms[0] or norms[-1] == 0.0 or len(norms) > maxit:
            break
        J = ns.jacobian_matrix(S, point_data(S, x, u_hist, delta, nu, dt), nu, dt, newton)
        dx = _pinned_solve(J, -F, nv)
        x = x + dx
    x[nv:] -= x[nv:].mean()
    return x, norms


def bdf2(S: Space, u_start, nu, dt, steps, boundary=None, rtol=1e-10, maxit=20):
    """`steps` BDF2 steps from the velocity u_start (u^{-1} = u^0 = u_start,
    pressure 0).  boundary: velocity values on the Dirichlet rows of every new
    state (default 0).  Returns the states [u; p] after each step and the
    residual histories of the Newton iterations."""
    nv = S.dim * S.Nv
    mask = ns.ns_dirichlet_mask(S)
    u_nm1 = u_start.copy()
    u_n = u_start.copy()
    p_n = np.zeros(S.Nv)
    bfull = np.zeros(nv + S.Nv)
    if boundary is not None:
        bfull[:nv] = boundary
    states, hists = [], []
    for _ in range(steps):
        delta = frozen_delta(S, u_n, nu, dt)
        uh = history(u_n, u_nm1)
        x0 = np.concatenate([u_n, p_n])
        x0[mask] = bfull[mask]
        x, norms = newton(S, x0, uh, delta, nu, dt, rtol, maxit)
        states.append(x)
        hists.append(norms)
        u_nm1, u_n, p_n = u_n, x[:nv].copy(), x[nv:].copy()
    return states, hists

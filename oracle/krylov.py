"""Block preconditioner, Schur PCG and FGMRES of the oracle (test
infrastructure only), Sec. 3 eq. (stokes_block).

Readings where the paper gives method names only:
* S ~ nu^{-1} M_p; its inverse applied by a fixed number of Jacobi-PCG steps
  (z0 = 0), so y_p = -nu z with M_p z ~ r_p;
* y_u = one V-cycle applied to r_u - B y_p (B = constrained gradient block);
* FGMRES(m) with right preconditioning, classical Gram-Schmidt applied
  twice, x0 = the lifting of the Dirichlet rows of b, stop when
  ||b - K x||_2 <= rtol ||b||_2 (estimated from the Givens-rotated
  Hessenberg system, confirmed with the true residual at every restart);
* the pressure is returned with zero mass-weighted mean.
"""
from __future__ import annotations

import numpy as np

from .fem import Space, assemble_stokes, constrain
from .mg import Hierarchy


def pcg_fixed(M, dinv, r, iterations):
    """Jacobi-preconditioned CG for M z = r from z = 0, a fixed number of steps."""
    z = np.zeros_like(r)
    res = r.copy()
    s = dinv * res
    p = s.copy()
    rho = res @ s
    for _ in range(iterations):
        q = M @ p
        pq = p @ q
        alpha = rho / pq if pq != 0 else 0.0
        z += alpha * p
        res -= alpha * q
        s = dinv * res
        rho_new = res @ s
        beta = rho_new / rho if rho != 0 else 0.0
        p = s + beta * p
        rho = rho_new
    return z


class StokesSystem:
    """Constrained Stokes matrix, its blocks and the multigrid hierarchy."""

    def __init__(self, dim, n, X, k, nu, schur_iterations=10, **mg_kw):
        self.S = Space(dim, n, X, k)
        self.nu = nu
        self.dim = dim
        self.mats = assemble_stokes(self.S, nu)
        self.mask = self.S.velocity_dirichlet_mask()
        self.K = constrain(self.mats["K"], self.mask)
        nu_ = dim * self.S.Nv
        self.nvel = nu_
        self.B = self.K[:nu_, nu_:]  # constrained gradient block
        self.M = self.mats["M"]
        self.Mdinv = 1.0 / self.M.diagonal()
        self.schur_iterations = schur_iterations
        self.mg = Hierarchy(dim, n, X, k, nu, **mg_kw)

    def precondition(self, r, vcycle=None, schur=None):
        nu_ = self.nvel
        rp = r[nu_:]
        if schur is None:
            yp = -self.nu * pcg_fixed(self.M, self.Mdinv, rp, self.schur_iterations)
        else:
            yp = schur(rp)
        t = r[:nu_] - self.B @ yp
        yu = self.mg.vcycle(t) if vcycle is None else vcycle(t)
        return np.concatenate([yu, yp])


def fgmres(K, b, precond, x0, rtol=1e-8, restart=30, maxit=200):
    """Right-preconditioned flexible GMRES; returns (x, iterations, rel_res)."""
    x = x0.copy()
    bnorm = np.linalg.norm(b)
    bnorm = bnorm if bnorm > 0 else 1.0
    its = 0
    r = b - K @ x
    beta = np.linalg.norm(r)
    while beta / bnorm > rtol and its < maxit:
        m = restart
        V = np.zeros((m + 1, len(b)))
        Z = np.zeros((m, len(b)))
        H = np.zeros((m + 1, m))
        cs, sn = np.zeros(m), np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        j = 0
        while j < m:
            Z[j] = precond(V[j])
            w = K @ Z[j]
            h = V[: j + 1] @ w
            w = w - V[: j + 1].T @ h
            h2 = V[: j + 1] @ w
            w = w - V[: j + 1].T @ h2
            h = h + h2
            hn = np.linalg.norm(w)
            V[j + 1] = w / hn if hn > 0 else 0.0
            col = np.concatenate([h, [hn]])
            for i in range(j):
                t = cs[i] * col[i] + sn[i] * col[i + 1]
                col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1]
                col[i] = t
            den = np.hypot(col[j], col[j + 1])
            cs[j] = col[j] / den if den > 0 else 1.0
            sn[j] = col[j + 1] / den if den > 0 else 0.0
            col[j] = den
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            H[: j + 1, j] = col[: j + 1]
            j += 1
            its += 1
            if abs(g[j]) / bnorm <= rtol or its >= maxit or hn == 0:
                break
        y = np.zeros(j)
        for i in range(j - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1: j] @ y[i + 1:]) / H[i, i]
        x = x + Z[:j].T @ y
        r = b - K @ x
        beta = np.linalg.norm(r)
    return x, its, beta / bnorm


def lifting(mask, b):
    return np.where(mask, b, 0.0)

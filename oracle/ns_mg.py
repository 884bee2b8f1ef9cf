"""Monolithic multigrid and GMRES for the stabilised Navier-Stokes Jacobian
(oracle; test infrastructure only), Sec. 5.

The Jacobian J of the SUPG/PSPG system (equal order Q_k/Q_k) is
preconditioned by one V-cycle of a hybrid multigrid acting on all d+1
components at once: first global coarsening of the mesh (h-levels), then
lowering of the degree (p-levels), relaxation around point Jacobi as the
smoother and a direct solve on the coarsest level; the outer solver is
(flexible) GMRES.

Readings where the paper gives only the method names:
* h-levels halve n while every n is even and larger than ``coarse_min``;
  then the degree drops one by one to ``p_min``.  Every level is equal order.
* Coarse-level operators are rediscretisations: J on a coarse level is built
  from the linearisation point interpolated at the coarse nodes (nodal
  interpolation of the fine velocity), with delta_1 recomputed from the
  coarse cells.  For k <= 2 every coarse node is a fine node, so the
  interpolation is an injection; these are the degrees the monolithic
  multigrid supports.
* Transfers: eq. (transfer) per component; the velocity components carry the
  Dirichlet constraints, the pressure is unconstrained.
* Smoother: ``relax_steps`` sweeps of damped point Jacobi
  x <- x + omega D^{-1} (b - J x), before and after the coarse correction,
  with D the diagonal of the constrained J (1 on Dirichlet rows); reading
  omega = 0.5 and 5 sweeps (the paper states 5 relaxation iterations).
  With ``smoother="asm"`` the sweeps use the additive Schwarz operator of
  ``oracle/asm.py`` in place of D^{-1} (the paper's Exp. 4: 2 sweeps).
* The constrained J is singular: a constant pressure lies in its kernel (the
  velocity vanishes on the whole boundary, so the pressure terms see only its
  gradient or integrate to a boundary flux).  The direct coarse solve fixes
  the pressure at pressure node 0 of the coarsest level: that row and column
  become the identity and the right-hand side entry is replaced by 0.
* GMRES: the FGMRES of the Stokes solver (right preconditioning, classical
  Gram-Schmidt twice), x0 = the Dirichlet rows of b; the pressure is
  returned with zero nodal mean (the kernel of J is the constant pressure).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as la
import scipy.sparse as sp

import inputs

from . import asm, basis, ns
from .fem import Space
from .krylov import fgmres
from .mg import transfer_matrix


def ns_level_specs(n, k, p_min=1, coarse_min=2):
    """[(n_list, k, h_level_index)] fine to coarse: h-levels first, then p."""
    n = list(n)
    out = [(list(n), k, 0)]
    hl = 0
    while all(v % 2 == 0 and v > max(1, coarse_min) for v in n):
        n = [v // 2 for v in n]
        hl += 1
        out.append((list(n), k, hl))
    kk = k
    while kk > max(1, p_min):
        kk -= 1
        out.append((list(n), kk, hl))
    return out


def _reference_positions(S: Space, deg: int) -> np.ndarray:
    """Global reference coordinates in [0, 1]^d of the scalar nodes of degree
    ``deg`` (the structured mesh seen as the unit cube; coarse meshes keep
    every second fine vertex, so transfers act in these coordinates)."""
    g = basis.gll_points(deg)
    axes = []
    for na in S.n:
        idx = np.arange(deg * na + 1)
        c = np.minimum(idx // deg, na - 1)
        axes.append((c + g[idx - deg * c]) / na)
    grids = np.meshgrid(*axes[::-1], indexing="ij")  # slowest axis first
    return np.stack([a.ravel() for a in grids[::-1]], axis=-1)


def interpolate_velocity(Sf: Space, Sc: Space, uf: np.ndarray) -> np.ndarray:
    """Nodal interpolation of the fine velocity at the coarse nodes.  Every
    coarse node must coincide with a fine node in reference coordinates
    (true for k <= 2); the fine value there is copied."""
    d = Sf.dim
    pf = _reference_positions(Sf, Sf.k)
    pc = _reference_positions(Sc, Sc.k)
    key = lambda p: np.round(p * 2 ** 30).astype(np.int64)  # noqa: E731
    kf = {tuple(v): i for i, v in enumerate(key(pf))}
    idx = np.array([kf.get(tuple(v), -1) for v in key(pc)])
    if (idx < 0).any() or np.abs(pf[np.maximum(idx, 0)] - pc).max() > 1e-12:
        raise ValueError("coarse nodes are not a subset of the fine nodes (k > 2 needs interpolation)")
    return np.concatenate([uf[c * Sf.Nv:(c + 1) * Sf.Nv][idx] for c in range(d)])


class NSHierarchy:
    """Levels, rediscretised constrained Jacobians, transfers and the pinned
    coarse factorisation."""

    def __init__(self, dim, n, X, k, nu, dt, u0, newton=True, p_min=1, coarse_min=2, relax_steps=5,
                 omega=0.5, smoother="jacobi"):
        self.dim, self.nu, self.dt, self.newton = dim, nu, dt, newton
        self.relax_steps, self.omega, self.smoother = relax_steps, omega, smoother
        specs = ns_level_specs(n, k, p_min, coarse_min)
        self.spaces, self.u0 = [], []
        for nl, kl, hl in specs:
            Xl = inputs.coarsen_vertices(dim, n, X, hl) if hl > 0 else X
            self.spaces.append(Space(dim, nl, Xl, kl, kl))
        self.u0.append(np.asarray(u0, dtype=np.float64))
        for l in range(1, len(self.spaces)):
            self.u0.append(interpolate_velocity(self.spaces[l - 1], self.spaces[l], self.u0[-1]))
        self.J, self.Dinv, self.fixed, self.P = [], [], [], []
        for S, u in zip(self.spaces, self.u0):
            data = ns.linearization_data(S, u, nu, dt)
            J = ns.jacobian_matrix(S, data, nu, dt, newton)
            self.J.append(J)
            self.Dinv.append(1.0 / J.diagonal())
            self.fixed.append(ns.ns_dirichlet_mask(S))
        self.B = []
        if smoother == "asm":
            for l in range(len(self.spaces) - 1):
                self.B.append(asm.ASM(self.J[l], asm.patches(self.spaces[l], self.fixed[l])))
        elif smoother != "jacobi":
            raise ValueError(smoother)
        for l in range(len(self.spaces) - 1):
            Sf, Sc = self.spaces[l], self.spaces[l + 1]
            h = Sf.n != Sc.n
            Pu = transfer_matrix(Sf, Sc, h, constrained=True)
            Pp = transfer_matrix(Sf, Sc, h, constrained=False)
            self.P.append(sp.block_diag([Pu] * dim + [Pp], format="csr"))
        Jc = self.J[-1].toarray()
        self.pin = dim * self.spaces[-1].Nv  # pressure node 0 of the coarsest level
        Jc[self.pin, :] = 0.0
        Jc[:, self.pin] = 0.0
        Jc[self.pin, self.pin] = 1.0
        self.coarse_lu = la.lu_factor(Jc)

    def coarse_solve(self, b):
        b = b.copy()
        b[self.pin] = 0.0
        return la.lu_solve(self.coarse_lu, b)

    def relax(self, l, x, b):
        if self.smoother == "asm":
            return asm.relax(self.J[l], self.B[l], x, b, self.relax_steps, self.omega)
        for _ in range(self.relax_steps):
            x = x + self.omega * self.Dinv[l] * (b - self.J[l] @ x)
        return x

    def vcycle(self, b, l=0):
        if l == len(self.spaces) - 1:
            return self.coarse_solve(b)
        x = np.where(self.fixed[l], b, 0.0)
        x = self.relax(l, x, b)
        r = b - self.J[l] @ x
        xc = self.vcycle(self.P[l].T @ r, l + 1)
        x = x + self.P[l] @ xc
        return self.relax(l, x, b)


def zero_mean_pressure(S: Space, x: np.ndarray) -> np.ndarray:
    y = x.copy()
    p = y[S.dim * S.Nv:]
    y[S.dim * S.Nv:] = p - p.mean()
    return y


def solve(H: NSHierarchy, b, rtol=1e-8, restart=30, maxit=200):
    """FGMRES on the constrained Jacobian of the finest level with one V-cycle
    as the preconditioner; returns (x, iterations, relative residual)."""
    S = H.spaces[0]
    x0 = np.where(H.fixed[0], b, 0.0)
    x, its, rel = fgmres(H.J[0], b, H.vcycle, x0, rtol, restart, maxit)
    return zero_mean_pressure(S, x), its, rel

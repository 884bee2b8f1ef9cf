"""Monolithic multigrid for the stabilised Navier-Stokes Jacobian on locally
refined meshes (oracle; test infrastructure only), Sec. 5.

Levels: global coarsening (GC) first, then the structured hierarchy of the
uniform base mesh (h-levels, then p-levels, as in ``ns_mg``).  A GC level is
the previous mesh with every family of eight leaf children replaced by its
parent, so the finest level present drops by one per step; after L steps
the mesh is the uniform base mesh.

Readings where the paper gives only the method names:
* The GC levels carry the same hanging-node constraints as the finest level
  (``amr.AmrSpace``), and each has its own rediscretised Jacobian with the
  linearisation point copied at the coarse unknowns (every coarse node of
  degree k <= 2 is a fine node position, and a coarse unknown is never a
  hanging node of the finer mesh).
* Transfers: the coarse space is a subspace of the fine one, so the
  prolongation is the coarse field evaluated at the fine unknowns (the
  interpolation of eq. (transfer) through the constraints); velocity rows and
  columns of Dirichlet unknowns are zero, the pressure is unconstrained.
  Restriction is the transpose.
* Smoother, coarse solve and V-cycle as in ``ns_mg``.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

import inputs

from . import amr, ns_mg
from .krylov import fgmres


def coarsen(mesh: dict) -> dict:
    """Replace every family of eight leaves by its parent."""
    lev = np.asarray(mesh["level"], dtype=np.int64)
    idx = np.asarray(mesh["idx"], dtype=np.int64)
    keep = np.ones(len(lev), dtype=bool)
    parents = []
    for l in range(1, lev.max() + 1):
        sel = np.nonzero(lev == l)[0]
        par = idx[sel] // 2
        key = par[:, 0] + (mesh["n"] << l) * (par[:, 1] + (mesh["n"] << l) * par[:, 2])
        uk, inv, cnt = np.unique(key, return_inverse=True, return_counts=True)
        full = cnt[inv] == 8
        keep[sel[full]] = False
        pk = np.unique(key[full])
        m2 = mesh["n"] << l
        pp = np.stack([pk % m2, (pk // m2) % m2, pk // (m2 * m2)], 1)  # parent indices
        parents.append((np.full(len(pk), l - 1), pp.reshape(-1, 3)))
    lev2 = np.concatenate([lev[keep]] + [p[0] for p in parents])
    idx2 = np.concatenate([idx[keep]] + [p[1] for p in parents])
    order = np.lexsort((idx2[:, 0], idx2[:, 1], idx2[:, 2], lev2))
    return {"n": mesh["n"], "levels": int(lev2.max()), "level": lev2[order], "idx": idx2[order]}


def copy_at_positions(Sf: amr.AmrSpace, Sc: amr.AmrSpace, uf: np.ndarray, ncomp: int) -> np.ndarray:
    """Coarse unknown values taken from the fine unknowns at the same
    positions (each coarse unknown is a fine unknown)."""
    scale = Sf.R // Sc.R
    key = lambda p: p[:, 0] + (Sf.R + 1) * (p[:, 1] + (Sf.R + 1) * p[:, 2])  # noqa: E731
    kf = key(Sf.true_pos)
    kc = key(Sc.true_pos * scale)
    pos = np.searchsorted(kf, kc)
    if np.any(pos >= len(kf)) or np.any(kf[np.minimum(pos, len(kf) - 1)] != kc):
        raise ValueError("a coarse unknown is not a fine unknown")
    return np.concatenate([uf[c * Sf.N:(c + 1) * Sf.N][pos] for c in range(ncomp)])


def transfer(Sf: amr.AmrSpace, Sc: amr.AmrSpace) -> sp.csr_matrix:
    """Prolongation of the 4-component vector: coarse field at the fine
    unknowns, Dirichlet velocity rows and columns zero."""
    E = Sc.evaluation_matrix(Sf.true_points())
    E.data[np.abs(E.data) < 1e-14] = 0.0
    E.eliminate_zeros()
    zf = sp.diags((~Sf.true_dirichlet).astype(np.float64))
    zc = sp.diags((~Sc.true_dirichlet).astype(np.float64))
    Ev = (zf @ E @ zc).tocsr()
    return sp.block_diag([Ev] * 3 + [E], format="csr")


class AmrNSHierarchy:
    def __init__(self, mesh, k, nu, dt, u0, newton=True, p_min=1, coarse_min=2, relax_steps=5, omega=0.5):
        self.relax_steps, self.omega = relax_steps, omega
        meshes = [mesh]
        while meshes[-1]["level"].max() > 0:
            meshes.append(coarsen(meshes[-1]))
        self.meshes = meshes
        self.spaces = [amr.AmrSpace(m, k) for m in meshes]  # the last one is uniform
        self.nga = len(meshes) - 1  # GC levels with their own operator
        self.u0 = [np.asarray(u0, dtype=np.float64)]
        for j in range(self.nga):
            self.u0.append(copy_at_positions(self.spaces[j], self.spaces[j + 1], self.u0[-1], 3))
        self.J, self.Dinv, self.fixed, self.P = [], [], [], []
        for j in range(self.nga):
            S = self.spaces[j]
            J = amr.jacobian_matrix(S, self.u0[j], nu, dt, newton)
            self.J.append(J)
            self.Dinv.append(1.0 / J.diagonal())
            self.fixed.append(S.ns_dirichlet_true())
            self.P.append(transfer(S, self.spaces[j + 1]))
        n = mesh["n"]
        self.base = ns_mg.NSHierarchy(3, [n] * 3, inputs.structured_vertices(3, [n] * 3), k, nu, dt,
                                      self.u0[self.nga], newton, p_min, coarse_min, relax_steps, omega)

    def relax(self, j, x, b):
        for _ in range(self.relax_steps):
            x = x + self.omega * self.Dinv[j] * (b - self.J[j] @ x)
        return x

    def vcycle(self, b, j=0):
        if j == self.nga:
            return self.base.vcycle(b)
        x = np.where(self.fixed[j], b, 0.0)
        x = self.relax(j, x, b)
        r = b - self.J[j] @ x
        xc = self.vcycle(self.P[j].T @ r, j + 1)
        x = x + self.P[j] @ xc
        return self.relax(j, x, b)

    def solve(self, b, rtol=1e-8, restart=30, maxit=200):
        """FGMRES on the finest Jacobian with one V-cycle as the preconditioner;
        the pressure is returned with zero nodal mean."""
        x0 = np.where(self.fixed[0], b, 0.0)
        x, its, rel = fgmres(self.J[0], b, self.vcycle, x0, rtol, restart, maxit)
        N = self.spaces[0].N
        x = x.copy()
        x[3 * N:] -= x[3 * N:].mean()
        return x, its, rel

"""Additive Schwarz (ASM) relaxation for the monolithic Navier-Stokes
multigrid (oracle; test infrastructure only): Sec. 2 (point Jacobi or ASM as
the ingredient of a relaxation smoother) and Sec. 5 (Exp. 4: two relaxation
steps around ASM on every level).

Readings where the paper names the method only:
* Patches: one per mesh vertex v.  Patch v holds every unknown (the d
  velocity components and the pressure) at the scalar nodes that lie
  strictly within one cell of v along every axis of the structured node
  lattice: node index i_a with |i_a - k v_a| < k.  For an interior vertex
  these are the nodes inside the union of the 2^d cells at v (its vertex
  star); at the domain boundary the star is clipped and keeps its nodes on
  the boundary.  Dirichlet unknowns (boundary velocity) are left out.  For
  Q1 a patch is the d + 1 unknowns of its vertex (point-block Jacobi); for
  Q2 it has 3^d nodes.
* Local matrices: A_P = R_P J R_P^T, the principal submatrix of the
  constrained Jacobian on the patch's unknowns, inverted exactly.
* Weighting: B = sum_P R_P^T W A_P^{-1} R_P with W = diag(1 / m_i), m_i the
  number of patches that hold unknown i (a partition of unity).
* Relaxation: x <- x + omega B (b - J x), ``steps`` times; reading omega = 1
  and 2 steps (the paper's Exp. 4).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as la

from .fem import Space, _multi_index


def node_multi_index(S: Space) -> np.ndarray:
    """[Nv, dim] lattice indices of the scalar nodes (x fastest)."""
    return _multi_index([a - 1 for a in S.vaxes], inclusive=True)


def vertex_multi_index(S: Space) -> np.ndarray:
    """[n_vertices, dim] vertex indices, lexicographic (x fastest)."""
    return _multi_index(S.n, inclusive=True)


def patches(S: Space, fixed: np.ndarray):
    """Unknown indices of every vertex patch (vertex order), Dirichlet
    unknowns (``fixed``) removed; unknown = field * Nv + node."""
    nodes = node_multi_index(S)
    out = []
    for v in vertex_multi_index(S):
        inside = np.flatnonzero(np.all(np.abs(nodes - S.k * v[None, :]) < S.k, axis=1))
        dofs = np.concatenate([f * S.Nv + inside for f in range(S.dim + 1)])
        out.append(np.sort(dofs[~fixed[dofs]]))
    return out


def multiplicity(n_unknowns: int, patch_list) -> np.ndarray:
    m = np.zeros(n_unknowns, dtype=np.int64)
    for I in patch_list:
        m[I] += 1
    return m


class ASM:
    """B = sum_P R_P^T W A_P^{-1} R_P for the sparse matrix J."""

    def __init__(self, J, patch_list):
        self.patches = [np.asarray(I) for I in patch_list]
        self.m = multiplicity(J.shape[0], self.patches)
        Jc = J.tocsr()
        self.inv = [la.inv(Jc[I][:, I].toarray()) for I in self.patches]

    def apply(self, r: np.ndarray) -> np.ndarray:
        y = np.zeros_like(r)
        for I, Ai in zip(self.patches, self.inv):
            y[I] += (Ai @ r[I]) / self.m[I]
        return y

    def matrix(self) -> np.ndarray:
        """B as a dense matrix (small cases)."""
        n = len(self.m)
        B = np.zeros((n, n))
        for I, Ai in zip(self.patches, self.inv):
            B[np.ix_(I, I)] += Ai / self.m[I][:, None]
        return B


def relax(J, B: ASM, x, b, steps, omega):
    for _ in range(steps):
        x = x + omega * B.apply(b - J @ x)
    return x

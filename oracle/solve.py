"""Right-hand side, direct solves and error norms for the oracle (test
infrastructure only).

Readings: inhomogeneous Dirichlet data enters by lifting.  b_i = (f, phi_i)
minus the unconstrained operator applied to the lifting on free rows, and
b_i = u_D(x_i) on Dirichlet rows, so the solution vector carries the boundary
values.  The pressure is fixed by a zero mean (the constrained operator
annihilates (0, 1_p)).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import basis
from .fem import Space, assemble_stokes, constrain, velocity_l2g


def load_vector(S: Space, f_qp: np.ndarray) -> np.ndarray:
    """(f, phi_i) for each velocity DoF, f given at the physical Gauss points
    of every cell as [nc, nq, dim]."""
    _, _, _, _, JxW = S.geometry()
    q1 = basis.gauss_rule(S.k + 1)[0]
    N, _, _ = basis.tensor_basis(S.dim, S.k, q1)
    out = np.zeros(S.dim * S.Nv)
    for c in range(S.dim):
        loc = np.einsum("eq,qi->ei", JxW * f_qp[:, :, c], N)
        np.add.at(out, (S.vdofs + c * S.Nv).ravel(), loc.ravel())
    return out


def stokes_rhs(S: Space, nu: float, f_qp: np.ndarray, uD_nodes: np.ndarray, mats=None):
    """Right-hand side of the constrained Stokes system.

    f_qp: [nc, nq, dim] forcing at the Gauss points; uD_nodes: [Nv, dim]
    velocity values at the velocity support points (only Dirichlet entries
    are used)."""
    mats = assemble_stokes(S, nu) if mats is None else mats
    mask = S.velocity_dirichlet_mask()
    lift = np.zeros(S.n_dofs)
    lift[: S.dim * S.Nv] = uD_nodes.T.ravel()
    lift[~mask] = 0.0
    b = np.zeros(S.n_dofs)
    b[: S.dim * S.Nv] = load_vector(S, f_qp)
    b -= mats["K"] @ lift
    b[mask] = lift[mask]
    return b


def pressure_mean_free(S: Space, x: np.ndarray, M=None) -> np.ndarray:
    """Shift the pressure block to zero mass-weighted mean."""
    if M is None:
        M = assemble_stokes(S, 1.0)["M"]
    y = x.copy()
    p = y[S.dim * S.Nv:]
    one = np.ones(S.Np)
    p -= (one @ (M @ p)) / (one @ (M @ one))
    return y


def direct_solve(S: Space, nu: float, b: np.ndarray, mats=None) -> np.ndarray:
    """Exact solution of the constrained (singular) Stokes system by a
    bordered sparse LU: [[K, e], [e^T, 0]] with e = (0, M_p 1)."""
    mats = assemble_stokes(S, nu) if mats is None else mats
    K = constrain(mats["K"], S.velocity_dirichlet_mask())
    e = np.zeros(S.n_dofs)
    e[S.dim * S.Nv:] = mats["M"] @ np.ones(S.Np)
    Kb = sp.bmat([[K, sp.csr_matrix(e[:, None])], [sp.csr_matrix(e[None, :]), None]], format="csc")
    xb = spla.spsolve(Kb, np.concatenate([b, [0.0]]))
    return xb[:-1]


def evaluate(S: Space, x: np.ndarray, q: int):
    """FE velocity, velocity gradient and pressure at the tensor Gauss points
    of a q-point rule in every cell, plus the physical points and JxW."""
    pts, W = basis.tensor_quadrature(S.dim, q)
    x1 = basis.gauss_rule(q)[0]
    N1, dN1, _ = basis.tensor_basis(S.dim, 1, x1)
    Xc = S.X[S.cell_vertices]
    xq = np.einsum("qv,cva->cqa", N1, Xc)
    J = np.einsum("qvb,cva->cqab", dN1, Xc)
    det = np.linalg.det(J)
    invJ = np.linalg.inv(J)
    N, dN, _ = basis.tensor_basis(S.dim, S.k, x1)
    u = np.zeros(xq.shape)
    gu = np.zeros(xq.shape + (S.dim,))
    for c in range(S.dim):
        loc = x[S.vdofs + c * S.Nv]
        u[:, :, c] = loc @ N.T
        gref = np.einsum("ei,qib->eqb", loc, dN)
        gu[:, :, c, :] = np.einsum("eqb,eqba->eqa", gref, invJ)
    Np_, _, _ = basis.tensor_basis(S.dim, S.kp, x1)
    p = x[S.dim * S.Nv:][S.pdofs] @ Np_.T
    return xq, det * W[None, :], u, gu, p

"""Space-time Kronecker operator of the transient Stokes equations (oracle;
test infrastructure only), Sec. 4 eq. (proceedings-kronecker).

On a time slab of length tau with a Q-stage DG(k) discretisation in time
(Q = k + 1) and the stage-major vector x = (x_1, .., x_Q), x_q = [u_q; p_q]:
    K x = (G_Q (x) M + tau I_Q (x) A) x,   G_Q = M_Q^{-1} A_Q^tau,
with M the Stokes block mass (velocity mass, zero pressure block) and A the
Stokes operator of eq. (stokes_block).  The temporal matrices come from the
nodal basis phi_1..phi_Q of P_k on the reference slab [0, 1]:
    M_Q[i, j] = int_0^1 phi_j phi_i ds,
    A_Q^tau[i, j] = int_0^1 phi_j' phi_i ds + phi_j(0) phi_i(0)   (the upwind jump),
    m_Q[i] = phi_i(0)   (the previous slab's end value enters b = f + (m_Q (x) M) x_{n-1}).

Readings where the paper is silent:
* temporal nodes: the Q Gauss-Legendre points of [0, 1] (the paper leaves the
  DG(k) basis to its references); the slab's end value is sum_j phi_j(1) x_j;
* constraints: every stage carries the spatial constraints: identity on the
  velocity Dirichlet rows of every stage, Dirichlet source values ignored in
  the other rows;
* temporal transfers between DG(k_f) and DG(k_c) (p-coarsening in time):
  P_tau[i, j] = phi^c_j(s^f_i), the coarse polynomial evaluated at the fine
  nodes, applied per spatial unknown; R_tau = P_tau^T.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import basis
from .fem import Space, assemble_stokes, constrain


def time_nodes(k: int) -> np.ndarray:
    return basis.gauss_rule(k + 1)[0]


def time_matrices(k: int):
    """M_Q, A_Q^tau, m_Q and the end-value weights e_Q (phi_j(1)) of DG(k)."""
    s = time_nodes(k)
    xq, wq = basis.gauss_rule(k + 2)  # exact for the degree-2k integrands
    V = basis.lagrange_values(s, xq)  # [point, j]
    D = basis.lagrange_derivatives(s, xq)
    MQ = np.einsum("p,pi,pj->ij", wq, V, V)
    v0 = basis.lagrange_values(s, np.array([0.0]))[0]
    v1 = basis.lagrange_values(s, np.array([1.0]))[0]
    AQ = np.einsum("p,pi,pj->ij", wq, V, D) + np.outer(v0, v0)
    return MQ, AQ, v0, v1


def G_matrix(k: int) -> np.ndarray:
    MQ, AQ, _, _ = time_matrices(k)
    return np.linalg.solve(MQ, AQ)


def block_mass(S: Space, mats=None):
    """Stokes block mass: velocity mass per component, zero pressure block."""
    mats = assemble_stokes(S, 1.0) if mats is None else mats
    Mu = mats["Mu"] if "Mu" in mats else None
    if Mu is None:
        Mu = velocity_mass(S)
    blocks = [Mu] * S.dim + [sp.csr_matrix((S.Np, S.Np))]
    return sp.block_diag(blocks, format="csr")


def velocity_mass(S: Space):
    """Scalar mass matrix of the velocity basis, full quadrature."""
    _, _, _, _, JxW = S.geometry()
    q1 = basis.gauss_rule(S.k + 1)[0]
    N, _, _ = basis.tensor_basis(S.dim, S.k, q1)
    Me = np.einsum("cq,qi,qj->cij", JxW, N, N)
    nb = N.shape[1]
    r = np.broadcast_to(S.vdofs[:, :, None], (S.nc, nb, nb)).ravel()
    c = np.broadcast_to(S.vdofs[:, None, :], (S.nc, nb, nb)).ravel()
    return sp.coo_matrix((Me.ravel(), (r, c)), shape=(S.Nv, S.Nv)).tocsr()


def kron_operator(S: Space, nu: float, tau: float, G: np.ndarray, mats=None):
    """Assembled constrained K = G (x) M + tau I (x) A (stage-major)."""
    mats = assemble_stokes(S, nu) if mats is None else mats
    mask = S.velocity_dirichlet_mask()
    M = block_mass(S, mats)
    K = (sp.kron(sp.csr_matrix(G), M) + tau * sp.kron(sp.identity(G.shape[0]), mats["K"])).tocsr()
    return constrain(K, np.tile(mask, G.shape[0]))


def kron_apply(S: Space, nu, tau, G, x, mats=None):
    """K x stage by stage: y_q = sum_r G[q, r] M x_r + tau A x_q on free rows,
    y_q = x_q on Dirichlet rows."""
    mats = assemble_stokes(S, nu) if mats is None else mats
    mask = S.velocity_dirichlet_mask()
    M = block_mass(S, mats)
    Q = G.shape[0]
    N = S.n_dofs
    X = x.reshape(Q, N)
    Xf = np.where(mask[None, :], 0.0, X)
    MX = np.array([M @ Xf[r] for r in range(Q)])
    Y = np.array([G[q] @ MX + tau * (mats["K"] @ Xf[q]) for q in range(Q)])
    Y[:, mask] = X[:, mask]
    return Y.ravel()


def time_prolongation(kf: int, kc: int) -> np.ndarray:
    """P_tau [Q_f, Q_c]: the coarse DG(kc) polynomial at the fine nodes."""
    return basis.lagrange_values(time_nodes(kc), time_nodes(kf))

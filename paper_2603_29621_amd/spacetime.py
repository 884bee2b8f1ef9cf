"""Host-side time discretisation for the space-time operator of Sec. 4
(eq. (proceedings-kronecker)): the DG(k) stage matrices on one slab, which
the caller hands to ``mfs_st_vmult`` (G) and ``mfs_st_stage_transfer``
(P_tau).  Small dense Q x Q arithmetic, Q = k + 1 <= 8.

Temporal nodal basis: Lagrange polynomials on the Q Gauss-Legendre points of
the reference slab [0, 1].  M_Q = (phi_j, phi_i), A_Q = (phi_j', phi_i) +
phi_j(0) phi_i(0) (upwind jump), G_Q = M_Q^{-1} A_Q; the previous slab's end
value enters the right-hand side through m_Q = (phi_i(0)); the end value of a
slab is sum_j phi_j(1) x_j.
"""
from __future__ import annotations

import numpy as np


def _nodes(k: int) -> np.ndarray:
    t, _ = np.polynomial.legendre.leggauss(k + 1)
    return 0.5 * (np.sort(t) + 1.0)


def _lagrange(nodes: np.ndarray, x: np.ndarray):
    """values [len(x), Q] and derivatives of the Lagrange basis of `nodes`."""
    Q = len(nodes)
    x = np.atleast_1d(x)
    val = np.ones((len(x), Q))
    der = np.zeros((len(x), Q))
    for j in range(Q):
        others = [nodes[m] for m in range(Q) if m != j]
        den = np.prod([nodes[j] - o for o in others]) if others else 1.0
        poly = np.poly1d(others, r=True) if others else np.poly1d([1.0])
        val[:, j] = poly(x) / den
        der[:, j] = poly.deriv()(x) / den if others else 0.0
    return val, der


def dg_stage_matrices(k: int):
    """(G_Q, M_Q, A_Q, m_Q, e_Q) of DG(k) on the reference slab."""
    s = _nodes(k)
    t, w = np.polynomial.legendre.leggauss(k + 2)
    t, w = 0.5 * (t + 1.0), 0.5 * w
    V, D = _lagrange(s, t)
    MQ = (V * w[:, None]).T @ V
    v0 = _lagrange(s, np.array([0.0]))[0][0]
    v1 = _lagrange(s, np.array([1.0]))[0][0]
    AQ = (V * w[:, None]).T @ D + np.outer(v0, v0)
    return np.linalg.solve(MQ, AQ), MQ, AQ, v0, v1


def stage_prolongation(kf: int, kc: int) -> np.ndarray:
    """P_tau [kf+1, kc+1]: the DG(kc) stage polynomial at the DG(kf) nodes."""
    return _lagrange(_nodes(kc), _nodes(kf))[0]

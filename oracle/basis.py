"""1D nodal bases and quadrature for the oracle (test infrastructure only).

The paper fixes the element pairs (Taylor-Hood Q_k/Q_{k-1}, Sec. 3; equal
order Q_kQ_k with PSPG, Sec. 5) but not the node set or the quadrature.
Reading used here (and by the HIP library, which implements it separately):

* nodal Lagrange basis on the Gauss-Lobatto-Legendre (GLL) points of [0, 1];
* tensor-product Gauss-Legendre quadrature with k+1 points per direction,
  k = velocity degree, for every term.

Everything is evaluated directly from the product formula of the Lagrange
polynomials; nothing is tabulated by a fast algorithm.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as L


def gll_points(k: int) -> np.ndarray:
    """k+1 Gauss-Lobatto-Legendre points on [0, 1]: the end points and the
    roots of P_k' mapped from [-1, 1]."""
    if k < 1:
        raise ValueError("degree must be >= 1")
    if k == 1:
        return np.array([0.0, 1.0])
    dP = L.Legendre.basis(k).deriv()
    inner = np.sort(np.real(dP.roots()))
    t = np.concatenate([[-1.0], inner, [1.0]])
    return 0.5 * (t + 1.0)


def gauss_rule(q: int):
    """q-point Gauss-Legendre rule on [0, 1] -> (points, weights)."""
    t, w = L.leggauss(q)
    return 0.5 * (t + 1.0), 0.5 * w


def lagrange_values(nodes: np.ndarray, x: np.ndarray) -> np.ndarray:
    """V[i, j] = phi_j(x_i) with phi_j the Lagrange polynomial of ``nodes``."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    V = np.ones((len(x), n))
    for j in range(n):
        for m in range(n):
            if m != j:
                V[:, j] *= (x - nodes[m]) / (nodes[j] - nodes[m])
    return V


def lagrange_derivatives(nodes: np.ndarray, x: np.ndarray) -> np.ndarray:
    """D[i, j] = phi_j'(x_i) by the product rule."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    D = np.zeros((len(x), n))
    for j in range(n):
        for l in range(n):
            if l == j:
                continue
            term = np.full(len(x), 1.0 / (nodes[j] - nodes[l]))
            for m in range(n):
                if m != j and m != l:
                    term *= (x - nodes[m]) / (nodes[j] - nodes[m])
            D[:, j] += term
    return D


def lagrange_second_derivatives(nodes: np.ndarray, x: np.ndarray) -> np.ndarray:
    """H[i, j] = phi_j''(x_i) by the product rule."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    H = np.zeros((len(x), n))
    for j in range(n):
        for l in range(n):
            if l == j:
                continue
            for r in range(n):
                if r == j or r == l:
                    continue
                term = np.full(len(x), 1.0 / ((nodes[j] - nodes[l]) * (nodes[j] - nodes[r])))
                for m in range(n):
                    if m not in (j, l, r):
                        term *= (x - nodes[m]) / (nodes[j] - nodes[m])
                H[:, j] += term
    return H


def tensor_index(dim: int, n1: int) -> np.ndarray:
    """Local multi-indices [n1^dim, dim] in lexicographic order, x fastest."""
    idx = np.stack(np.meshgrid(*[np.arange(n1)] * dim, indexing="ij"), 0)
    return idx.reshape(dim, -1, order="F").T.copy()


def tensor_basis(dim: int, k: int, pts1d: np.ndarray):
    """Values and reference gradients of the Q_k GLL basis at the tensor points
    of ``pts1d`` (also lexicographic, x fastest).

    Returns (N [nq, nb], dN [nq, nb, dim], H [nq, nb, dim, dim]) where H is the
    reference Hessian."""
    nodes = gll_points(k)
    V = lagrange_values(nodes, pts1d)
    D = lagrange_derivatives(nodes, pts1d)
    S = lagrange_second_derivatives(nodes, pts1d)
    qi = tensor_index(dim, len(pts1d))
    bi = tensor_index(dim, k + 1)
    nq, nb = len(qi), len(bi)
    N = np.ones((nq, nb))
    dN = np.ones((nq, nb, dim))
    H = np.ones((nq, nb, dim, dim))
    for a in range(dim):
        va = V[qi[:, a]][:, bi[:, a]]  # [nq, nb]
        da = D[qi[:, a]][:, bi[:, a]]
        sa = S[qi[:, a]][:, bi[:, a]]
        N *= va
        for b in range(dim):
            dN[:, :, b] *= da if a == b else va
            for c in range(dim):
                if a == b == c:
                    H[:, :, b, c] *= sa
                elif a == b or a == c:
                    H[:, :, b, c] *= da
                else:
                    H[:, :, b, c] *= va
    return N, dN, H


def tensor_quadrature(dim: int, q: int):
    """Tensor Gauss rule on [0,1]^dim: (points [nq, dim], weights [nq]),
    lexicographic with x fastest."""
    x, w = gauss_rule(q)
    qi = tensor_index(dim, q)
    P = x[qi]
    W = np.prod(w[qi], axis=1)
    return P, W

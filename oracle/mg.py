"""Multigrid pieces of the oracle, matrix-based (test infrastructure only).

* Level hierarchy of Sec. 3: the polynomial degree is lowered one by one
  (p-levels) down to ``p_min``, then the mesh is coarsened globally
  (h-levels).  Reading: h-coarsening halves n while every n is even and
  larger than ``coarse_min``; a coarse mesh keeps the fine vertices whose
  indices are divisible by 2 (reference-space transfer).
* Transfer, Sec. 2 eq. (transfer): P = sum_e S_e W_e P_e C_e G_e, assembled
  here as a sparse matrix.  P_e[i, j] is the coarse Lagrange basis function j
  evaluated at fine node i of the coarse cell (reference coordinates).
  Reading of "some weighting": W = 1/m_i with m_i the number of coarse cells
  containing fine node i.  C_e: coarse Dirichlet values are zero; fine
  Dirichlet rows of P are zero.  Restriction is P^T.
* Chebyshev semi-iteration around point Jacobi (Sec. 2 and 3) on the interval
  [lambda/range, lambda] (reading: range 20, lambda = 1.2 times the largest
  eigenvalue estimate of D^{-1} A).
* V-cycle: pre-smoothing from x = (b on Dirichlet rows, 0 elsewhere),
  residual, restriction, recursion, prolongation, post-smoothing; exact
  solve on the coarsest level.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as la
import scipy.sparse as sp

import inputs

from . import basis
from .fem import Space, assemble_stokes, constrain


def level_specs(n, k, p_min=1, coarse_min=2):
    """[(n_list, k, h_level_index)] from fine to coarse."""
    n = list(n)
    out = [(list(n), k, 0)]
    kk, hl = k, 0
    while kk > max(1, p_min):
        kk -= 1
        out.append((list(n), kk, hl))
    while all(v % 2 == 0 and v > max(1, coarse_min) for v in n):
        n = [v // 2 for v in n]
        hl += 1
        out.append((list(n), kk, hl))
    return out


def build_spaces(dim, n, X, k, p_min=1, coarse_min=2):
    specs = level_specs(n, k, p_min, coarse_min)
    spaces = []
    for i, (nl, kl, hl) in enumerate(specs):
        Xl = inputs.coarsen_vertices(dim, n, X, hl) if hl > 0 else X
        kp = (kl - 1) if i == 0 and kl >= 2 else 0
        spaces.append(Space(dim, nl, Xl, kl, kp if kp > 0 else 0))
    return spaces


def _fine_positions_h(k):
    """1D reference positions (in the coarse cell) of the 2k+1 fine nodes of
    the two children."""
    g = basis.gll_points(k)
    return np.concatenate([0.5 * g, 0.5 + 0.5 * g[1:]])


def transfer_matrix(Sf: Space, Sc: Space, h: bool, constrained: bool = True) -> sp.csr_matrix:
    """Scalar prolongation (coarse -> fine), with the Dirichlet constraints
    unless ``constrained`` is False, as a CSR matrix."""
    dim = Sf.dim
    kc = Sc.k
    if h:
        pos = _fine_positions_h(kc)
        F = 2 * kc
        assert Sf.k == kc and all(a == 2 * b for a, b in zip(Sf.n, Sc.n))
    else:
        pos = basis.gll_points(Sf.k)
        F = Sf.k
        assert Sf.n == Sc.n
    E = basis.lagrange_values(basis.gll_points(kc), pos)  # [F+1, kc+1]
    floc = basis.tensor_index(dim, F + 1)  # fine local multi-indices
    cloc = basis.tensor_index(dim, kc + 1)
    # P_e = product over directions of E
    Pe = np.ones((len(floc), len(cloc)))
    for a in range(dim):
        Pe *= E[floc[:, a]][:, cloc[:, a]]
    # global fine / coarse indices per coarse cell
    fstr = np.cumprod([1] + Sf.vaxes[:-1])
    cstr = np.cumprod([1] + Sc.vaxes[:-1])
    C = Sc.cidx  # [nc, dim]
    fg = ((C[:, None, :] * F + floc[None, :, :]) * fstr[None, None, :]).sum(-1)  # [nc, nf_loc]
    cg = ((C[:, None, :] * kc + cloc[None, :, :]) * cstr[None, None, :]).sum(-1)
    mult = np.bincount(fg.ravel(), minlength=Sf.Nv).astype(np.float64)
    nc = C.shape[0]
    rows = np.broadcast_to(fg[:, :, None], (nc, fg.shape[1], cg.shape[1])).ravel()
    cols = np.broadcast_to(cg[:, None, :], (nc, fg.shape[1], cg.shape[1])).ravel()
    vals = np.broadcast_to(Pe[None], (nc,) + Pe.shape).ravel() / mult[rows]
    P = sp.coo_matrix((vals, (rows, cols)), shape=(Sf.Nv, Sc.Nv)).tocsr()
    if not constrained:
        return P
    zf = sp.diags((~Sf.dirichlet).astype(np.float64))
    zc = sp.diags((~Sc.dirichlet).astype(np.float64))
    return (zf @ P @ zc).tocsr()


def vector_op(M: sp.spmatrix, dim: int) -> sp.csr_matrix:
    """Block-diagonal copy of a scalar operator for every velocity component."""
    return sp.block_diag([M] * dim, format="csr")


class Hierarchy:
    """Matrix-based multigrid on the velocity block A (vector Laplacian)."""

    def __init__(self, dim, n, X, k, nu, p_min=1, coarse_min=2, cheb_degree=5, cheb_range=20.0):
        self.dim = dim
        self.nu = nu
        self.spaces = build_spaces(dim, n, X, k, p_min, coarse_min)
        self.A, self.Dinv, self.P, self.fixed = [], [], [], []
        for S in self.spaces:
            A = assemble_stokes(S, nu)["A"] if S.kp > 0 else _laplace_only(S, nu)
            Ac = constrain(A, S.dirichlet)
            self.A.append(vector_op(Ac, dim))
            d = Ac.diagonal()
            self.Dinv.append(np.tile(1.0 / d, dim))
            self.fixed.append(np.tile(S.dirichlet, dim))
        for l in range(len(self.spaces) - 1):
            Sf, Sc = self.spaces[l], self.spaces[l + 1]
            h = Sf.n != Sc.n
            self.P.append(vector_op(transfer_matrix(Sf, Sc, h), dim))
        self.cheb_degree = cheb_degree
        self.cheb_range = cheb_range
        self.lam = [None] * len(self.spaces)
        Ac = self.A[-1].toarray()
        self.coarse_factor = la.cho_factor(Ac)

    def exact_lambda_max(self, l):
        """Largest eigenvalue of D^{-1} A on the free rows (dense, small)."""
        A = self.A[l].toarray()
        free = ~self.fixed[l]
        d = np.sqrt(self.Dinv[l][free])
        B = d[:, None] * A[np.ix_(free, free)] * d[None, :]
        return float(la.eigvalsh(B)[-1])

    def chebyshev(self, l, x, b, zero_start):
        return chebyshev_smooth(self.A[l], self.Dinv[l], self.fixed[l], self.lam[l], self.cheb_range,
                                self.cheb_degree, x, b, zero_start)

    def vcycle(self, b, l=0):
        if l == len(self.spaces) - 1:
            return la.cho_solve(self.coarse_factor, b)
        x = np.where(self.fixed[l], b, 0.0)
        x = self.chebyshev(l, x, b, True)
        r = b - self.A[l] @ x
        bc = self.P[l].T @ r
        xc = self.vcycle(bc, l + 1)
        x = x + self.P[l] @ xc
        return self.chebyshev(l, x, b, False)


def chebyshev_smooth(A, Dinv, fixed, lmax, rng, degree, x, b, zero_start):
    """``degree`` steps of the Chebyshev semi-iteration for A x = b with
    Jacobi scaling Dinv on [lmax/rng, lmax]; rows in ``fixed`` keep x."""
    lmin = lmax / rng
    theta, delta = 0.5 * (lmax + lmin), 0.5 * (lmax - lmin)
    sigma = theta / delta
    rho_old = 1.0 / sigma
    x = x.copy()
    r = Dinv * (b if zero_start else b - A @ x)
    r[fixed] = 0.0
    d = r / theta
    x += d
    for _ in range(1, degree):
        rho = 1.0 / (2.0 * sigma - rho_old)
        r = Dinv * (b - A @ x)
        r[fixed] = 0.0
        d = rho * rho_old * d + (2.0 * rho / delta) * r
        x += d
        rho_old = rho
    return x


def _laplace_only(S: Space, nu: float):
    from .fem import _assemble, stokes_element_matrices

    em = stokes_element_matrices(S, nu)
    return _assemble(S.vdofs, S.vdofs, em["A"], (S.Nv, S.Nv))


def chebyshev_error_polynomial(lam, lmax, rng, degree):
    """Closed form of the Chebyshev error polynomial p_d(lambda) =
    T_d((b+a-2 lambda)/(b-a)) / T_d((b+a)/(b-a)) on [a, b] = [lmax/rng, lmax]."""
    a, b = lmax / rng, lmax

    def T(d, t):
        t = np.asarray(t, dtype=np.float64)
        out = np.where(np.abs(t) <= 1, np.cos(d * np.arccos(np.clip(t, -1, 1))),
                       np.cosh(d * np.arccosh(np.maximum(np.abs(t), 1.0))) * np.sign(t) ** d)
        return out

    return T(degree, (b + a - 2 * lam) / (b - a)) / T(degree, (b + a) / (b - a))

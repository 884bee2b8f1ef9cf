"""Structured hexahedral meshes, DoF numbering, geometry and Stokes element
matrices by full quadrature (oracle; test infrastructure only).

Follows Sec. 1, eq. (stokes), and the block system of Sec. 3,
eq. (stokes_block).  Readings where the paper is silent:

* Sign of the divergence rows: the block matrix [[A, B], [B^T, 0]] of
  eq. (stokes_block) is symmetric, so the pressure rows carry B^T u with
  B_ij = -(psi_j, div phi_i); the +(div u, q) of eq. (stokes) differs only by
  the sign of the pressure rows and gives the same discrete solution.
* A_ij = nu (grad phi_j, grad phi_i) with the full gradient, one scalar block
  per velocity component.
* Geometry: the Q1 (bilinear / trilinear) map of the cell's 2^d vertices.
* Constraints: every velocity node on the boundary is a Dirichlet node.  The
  constrained operator acts as the identity on those rows and ignores the
  source values there in every other row.

DoF layout (shared with the HIP library as an interface, not as code):
blocked vector [u_0 | u_1 | (u_2) | p]; on the structured grid with n[a]
cells and degree k the scalar nodes form a (k n0 + 1) x (k n1 + 1) (x ...)
lexicographic grid, x fastest.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import basis


class Space:
    """Structured Q_k / Q_kp space on a (possibly perturbed) structured mesh."""

    def __init__(self, dim: int, n, X: np.ndarray, k: int, kp: int | None = None):
        self.dim = dim
        self.n = [int(v) for v in (n if hasattr(n, "__len__") else [n] * dim)]
        self.X = np.asarray(X, dtype=np.float64).reshape(-1, dim)
        self.k = int(k)
        self.kp = int(k - 1 if kp is None else kp)
        self.nc = int(np.prod(self.n))
        assert self.X.shape[0] == int(np.prod([na + 1 for na in self.n]))
        # cell multi-indices, lexicographic x fastest
        self.cidx = _multi_index(self.n)
        self.vaxes = [self.k * na + 1 for na in self.n]
        self.Nv = int(np.prod(self.vaxes))
        self.paxes = [self.kp * na + 1 for na in self.n] if self.kp > 0 else None
        self.Np = int(np.prod(self.paxes)) if self.kp > 0 else 0
        self.cell_vertices = self._local_to_global([na + 1 for na in self.n], 1)
        self.vdofs = self._local_to_global(self.vaxes, self.k)
        self.pdofs = self._local_to_global(self.paxes, self.kp) if self.kp > 0 else None
        self.dirichlet = self._boundary_mask(self.vaxes)

    # -- numbering ---------------------------------------------------------
    def _local_to_global(self, axes, deg):
        loc = basis.tensor_index(self.dim, deg + 1)  # [nb, dim]
        g = self.cidx[:, None, :] * deg + loc[None, :, :]  # [nc, nb, dim]
        strides = np.cumprod([1] + list(axes[:-1]))
        return (g * np.array(strides)[None, None, :]).sum(-1)

    def _boundary_mask(self, axes):
        idx = _multi_index([a - 1 for a in axes], inclusive=True)
        m = np.zeros(len(idx), dtype=bool)
        for a in range(self.dim):
            m |= (idx[:, a] == 0) | (idx[:, a] == axes[a] - 1)
        return m

    def node_coords_reference(self, axes, deg):
        """Global node multi-indices [N, dim] of a scalar grid."""
        return _multi_index([a - 1 for a in axes], inclusive=True)

    @property
    def n_dofs(self):
        return self.dim * self.Nv + self.Np

    def velocity_dirichlet_mask(self):
        """Boolean mask over the full blocked vector: True on Dirichlet rows."""
        m = np.zeros(self.n_dofs, dtype=bool)
        for c in range(self.dim):
            m[c * self.Nv:(c + 1) * self.Nv] = self.dirichlet
        return m

    # -- geometry ----------------------------------------------------------
    def geometry(self, cells=None):
        """Physical quadrature points, Jacobians, determinants, inverses and
        JxW at the (k+1)^d Gauss points of the given cells."""
        cells = np.arange(self.nc) if cells is None else np.asarray(cells)
        Pq, Wq = basis.tensor_quadrature(self.dim, self.k + 1)
        N1, dN1, _ = basis.tensor_basis(self.dim, 1, basis.gauss_rule(self.k + 1)[0])
        Xc = self.X[self.cell_vertices[cells]]  # [c, 2^d, dim]
        xq = np.einsum("qv,cva->cqa", N1, Xc)
        J = np.einsum("qvb,cva->cqab", dN1, Xc)  # J[a,b] = dx_a/dxi_b
        det = np.linalg.det(J)
        if np.any(det <= 0):
            raise ValueError("non-positive Jacobian determinant")
        invJ = np.linalg.inv(J)
        return xq, J, det, invJ, det * Wq[None, :]

    def support_points(self, deg=None):
        """Physical coordinates of the scalar nodes of degree ``deg`` (velocity
        degree by default), by the Q1 map of the cell containing them."""
        deg = self.k if deg is None else deg
        axes = [deg * na + 1 for na in self.n]
        N = int(np.prod(axes))
        out = np.zeros((N, self.dim))
        nodes = basis.gll_points(deg)
        N1 = basis.tensor_basis(self.dim, 1, nodes)[0]  # [nb, 2^d]
        g = self._local_to_global(axes, deg)
        Xc = self.X[self.cell_vertices]
        out[g.ravel()] = np.einsum("bv,cva->cba", N1, Xc).reshape(-1, self.dim)
        return out


def _multi_index(n, inclusive=False):
    """[prod(n(+1)), dim] lexicographic multi-indices (x fastest)."""
    ext = [na + 1 for na in n] if inclusive else list(n)
    idx = np.stack(np.meshgrid(*[np.arange(e) for e in ext], indexing="ij"), 0)
    return idx.reshape(len(ext), -1, order="F").T.copy()


# ---------------------------------------------------------------------------
# Element matrices (full quadrature, dense)
# ---------------------------------------------------------------------------
def stokes_element_matrices(S: Space, nu: float, cells=None):
    """Per-cell dense matrices:
    A[c, i, j] = nu sum_q JxW grad(phi_i) . grad(phi_j)          (scalar block)
    B[c, comp*nv + i, j] = - sum_q JxW psi_j d(phi_i)/dx_comp
    M[c, i, j] = sum_q JxW psi_i psi_j                            (pressure mass)
    """
    xq, J, det, invJ, JxW = S.geometry(cells)
    q1 = basis.gauss_rule(S.k + 1)[0]
    _, dN, _ = basis.tensor_basis(S.dim, S.k, q1)
    G = np.einsum("qib,cqba->cqia", dN, invJ)  # physical gradients
    A = nu * np.einsum("cq,cqia,cqja->cij", JxW, G, G)
    out = {"A": A}
    if S.kp > 0:
        Np_, _, _ = basis.tensor_basis(S.dim, S.kp, q1)
        B = -np.einsum("cq,qj,cqia->caij", JxW, Np_, G)  # [c, comp, i, j]
        out["B"] = B.reshape(B.shape[0], -1, B.shape[-1])
        out["M"] = np.einsum("cq,qi,qj->cij", JxW, Np_, Np_)
    return out


def _assemble(rows_l2g, cols_l2g, blocks, shape):
    nc, nr = rows_l2g.shape
    ncol = cols_l2g.shape[1]
    r = np.broadcast_to(rows_l2g[:, :, None], (nc, nr, ncol)).ravel()
    c = np.broadcast_to(cols_l2g[:, None, :], (nc, nr, ncol)).ravel()
    return sp.coo_matrix((blocks.ravel(), (r, c)), shape=shape).tocsr()


def velocity_l2g(S: Space):
    """[nc, dim*nv] global indices of the local velocity DoFs, component-major."""
    return np.concatenate([S.vdofs + c * S.Nv for c in range(S.dim)], axis=1)


def assemble_stokes(S: Space, nu: float):
    """Unconstrained CSR matrices (A_scalar, A_vec, B, M_p, K)."""
    em = stokes_element_matrices(S, nu)
    A = _assemble(S.vdofs, S.vdofs, em["A"], (S.Nv, S.Nv))
    Avec = sp.block_diag([A] * S.dim, format="csr")
    B = _assemble(velocity_l2g(S), S.pdofs, em["B"], (S.dim * S.Nv, S.Np))
    M = _assemble(S.pdofs, S.pdofs, em["M"], (S.Np, S.Np))
    K = sp.bmat([[Avec, B], [B.T, None]], format="csr")
    return {"A": A, "Avec": Avec, "B": B, "M": M, "K": K}


def constrain(K: sp.spmatrix, mask: np.ndarray) -> sp.csr_matrix:
    """Z K Z + I_D: zero the rows and columns of the masked DoFs and put 1 on
    their diagonal."""
    z = sp.diags((~mask).astype(np.float64))
    return (z @ K @ z + sp.diags(mask.astype(np.float64))).tocsr()


def stokes_operator(S: Space, nu: float):
    """Constrained Stokes matrix (CSR)."""
    mats = assemble_stokes(S, nu)
    return constrain(mats["K"], S.velocity_dirichlet_mask()), mats


def element_loop_stokes_vmult(S: Space, nu: float, x: np.ndarray, chunk: int = 4096, cells=None) -> np.ndarray:
    """Constrained Stokes matvec by an explicit loop over cells (chunks of
    cells), each cell multiplying its dense element matrix.  With ``cells``
    only those cells contribute (rows they do not fully cover are partial)."""
    mask = S.velocity_dirichlet_mask()
    xz = np.where(mask, 0.0, x)
    y = np.zeros_like(x)
    ul2g = velocity_l2g(S)
    nv = S.vdofs.shape[1]
    all_cells = np.arange(S.nc) if cells is None else np.asarray(cells)
    for c0 in range(0, len(all_cells), chunk):
        cells = all_cells[c0:c0 + chunk]
        em = stokes_element_matrices(S, nu, cells)
        ug = ul2g[cells]
        pg = S.pdofs[cells] + S.dim * S.Nv
        xu = xz[ug]
        xp = xz[pg]
        yu = np.empty_like(xu)
        for c in range(S.dim):
            yu[:, c * nv:(c + 1) * nv] = np.einsum("eij,ej->ei", em["A"], xu[:, c * nv:(c + 1) * nv])
        yu += np.einsum("eij,ej->ei", em["B"], xp)
        yp = np.einsum("eij,ei->ej", em["B"], xu)
        np.add.at(y, ug.ravel(), yu.ravel())
        np.add.at(y, pg.ravel(), yp.ravel())
    y[mask] = x[mask]
    return y


def cells_containing(S: Space, rows: np.ndarray) -> np.ndarray:
    """Cells whose local DoFs include the given rows of the blocked vector."""
    out = set()
    for r in np.asarray(rows):
        if r < S.dim * S.Nv:
            node, axes, deg = r % S.Nv, S.vaxes, S.k
        else:
            node, axes, deg = r - S.dim * S.Nv, S.paxes, S.kp
        g = []
        for a in range(S.dim):
            g.append(node % axes[a])
            node //= axes[a]
        per_dir = []
        for a in range(S.dim):
            c = g[a] // deg
            opts = [v for v in (c, c - 1 if g[a] % deg == 0 else None) if v is not None and 0 <= v < S.n[a]]
            per_dir.append(opts)
        for combo in np.array(np.meshgrid(*per_dir, indexing="ij")).reshape(S.dim, -1).T:
            cid = 0
            for a in reversed(range(S.dim)):
                cid = cid * S.n[a] + combo[a]
            out.add(int(cid))
    return np.array(sorted(out), dtype=np.int64)


def sampled_stokes_rows(S: Space, nu: float, x: np.ndarray, rows: np.ndarray) -> np.ndarray:
    """(K x)_i of the constrained Stokes operator for the given rows, from the
    element matrices of the cells containing them."""
    cells = cells_containing(S, rows)
    y = element_loop_stokes_vmult(S, nu, x, cells=cells)
    mask = S.velocity_dirichlet_mask()
    y[mask] = x[mask]
    return y[np.asarray(rows)]

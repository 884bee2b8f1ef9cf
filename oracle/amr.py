"""Locally refined meshes with hanging nodes (oracle; test infrastructure
only): the conforming Q_k space, its constraints, and the SUPG/PSPG
Navier-Stokes Jacobian on it (Sec. 5, locally refined meshes; the hanging-
node constraints C_e of eq. (transfer) and Sec. 2).

Mesh: leaves of an octree over n^3 Cartesian cells of the unit cube, 2:1
balanced over faces and edges (``inputs.refined_mesh``).  Cell (l, i, j, m)
has side 1 / (n 2^l).

Space (k = 1, 2, whose GLL nodes are equispaced): every cell carries the
(k+1)^3 tensor nodes.  Node positions live on the integer lattice of
spacing 1 / (k n 2^L) (L the finest level), so equal positions are found
exactly.  The raw nodes are the distinct positions.  A raw node that lies in
the closed region of a coarser leaf without being one of its nodes is
hanging: its value is that leaf's Q_k interpolant at the node (the trace on
the shared face or edge), expanded recursively when a master is hanging
itself; the coarsest such leaf is used.  The remaining raw nodes are the
unknowns.  C maps unknowns to raw nodes (identity on unknowns, the
interpolation weights on hanging nodes), and the constrained operator is
C^T A_raw C with A_raw assembled cell by cell over raw nodes.

Numbering (an interface shared with the HIP library, not code): unknowns in
lexicographic order of their lattice position, x fastest; vectors are
blocked by component as on structured meshes.  Velocity unknowns on the
boundary of the cube are Dirichlet unknowns; the pressure has none.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import basis, ns
from .fem import Space, constrain


class AmrSpace(Space):
    """Conforming Q_k space (equal order for Navier-Stokes) on a refined mesh."""

    def __init__(self, mesh: dict, k: int):
        if k not in (1, 2):
            raise ValueError("refined meshes support k = 1, 2")
        self.dim, self.k, self.kp = 3, int(k), int(k)
        n, L = int(mesh["n"]), int(mesh["levels"])
        self.n = [n] * 3
        self.L = L
        self.lev = np.asarray(mesh["level"], dtype=np.int64)
        self.idx = np.asarray(mesh["idx"], dtype=np.int64)
        self.nc = len(self.lev)
        self.R = k * n * 2 ** L  # lattice extent
        self.unit = 2 ** (L - self.lev)  # node spacing of each cell
        self.origin = self.idx * (k * self.unit)[:, None]
        self.loc = basis.tensor_index(3, k + 1)
        pos = self.origin[:, None, :] + self.loc[None] * self.unit[:, None, None]
        key = self._key(pos)
        ukeys, inv = np.unique(key.ravel(), return_inverse=True)
        self.raw_pos = self._decode(ukeys)
        self.vdofs = inv.reshape(self.nc, -1)
        self.Nv = len(ukeys)
        # geometry: the 8 corners of every cell (Q1 map of fem.Space)
        h = 1.0 / (n * 2.0 ** self.lev)
        corners = basis.tensor_index(3, 2)
        self.X = ((self.idx[:, None, :] + corners[None]) * h[:, None, None]).reshape(-1, 3)
        self.cell_vertices = np.arange(self.nc * 8).reshape(self.nc, 8)
        self.dirichlet = np.zeros(self.Nv, dtype=bool)  # raw assembly is unconstrained
        self._constraints()

    def _key(self, p):
        R1 = self.R + 1
        return p[..., 0] + R1 * (p[..., 1] + R1 * p[..., 2])

    def _decode(self, key):
        R1 = self.R + 1
        return np.stack([key % R1, (key // R1) % R1, key // (R1 * R1)], -1)

    def _constraints(self):
        k = self.k
        master = np.full(self.Nv, -1, dtype=np.int64)
        for c in np.argsort(self.lev, kind="stable"):  # coarsest cells first
            lo = self.origin[c]
            hi = lo + k * self.unit[c]
            inside = np.all((self.raw_pos >= lo) & (self.raw_pos <= hi), axis=1)
            off_lattice = np.any((self.raw_pos - lo) % self.unit[c] != 0, axis=1)
            sel = inside & off_lattice & (master < 0)
            master[sel] = c
        self.master = master
        self.hanging = master >= 0
        self.true_of = np.cumsum(~self.hanging) - 1
        self.N = int((~self.hanging).sum())
        self.true_pos = self.raw_pos[~self.hanging]
        gll = basis.gll_points(k)
        memo = {}

        def expand(r):
            if not self.hanging[r]:
                return {int(self.true_of[r]): 1.0}
            if r in memo:
                return memo[r]
            c = master[r]
            xi = (self.raw_pos[r] - self.origin[c]) / float(k * self.unit[c])
            w1 = [basis.lagrange_values(gll, xi[a])[0] for a in range(3)]
            out = {}
            for t, (i, j, l) in enumerate(self.loc):
                w = w1[0][i] * w1[1][j] * w1[2][l]
                if abs(w) < 1e-14:
                    continue
                for g, v in expand(int(self.vdofs[c, t])).items():
                    out[g] = out.get(g, 0.0) + w * v
            memo[r] = out
            return out

        rows, cols, vals = [], [], []
        for r in range(self.Nv):
            for g, v in expand(r).items():
                rows.append(r)
                cols.append(g)
                vals.append(v)
        self.C = sp.csr_matrix((vals, (rows, cols)), shape=(self.Nv, self.N))
        on_bnd = np.any((self.true_pos == 0) | (self.true_pos == self.R), axis=1)
        self.true_dirichlet = on_bnd

    # -- helpers -------------------------------------------------------------
    def true_points(self):
        """Physical coordinates of the unknowns [N, 3]."""
        return self.true_pos / float(self.R)

    def expand(self, x, ncomp):
        """Unknown values (ncomp blocks of N) -> raw node values (blocks of Nv)."""
        return np.concatenate([self.C @ x[c * self.N:(c + 1) * self.N] for c in range(ncomp)])

    def restrict(self, y, ncomp):
        """Transpose of expand."""
        return np.concatenate([self.C.T @ y[c * self.Nv:(c + 1) * self.Nv] for c in range(ncomp)])

    def ns_dirichlet_true(self):
        m = np.zeros(4 * self.N, dtype=bool)
        for c in range(3):
            m[c * self.N:(c + 1) * self.N] = self.true_dirichlet
        return m

    def evaluation_matrix(self, pts):
        """Sparse [m, N]: values of the unknowns' basis functions at physical
        points [m, 3] (each point in the first leaf of the list whose closed
        region contains it; the space is continuous, so any such leaf gives
        the same values)."""
        gll = basis.gll_points(self.k)
        lat = np.asarray(pts, dtype=np.float64) * self.R
        side = (self.k * self.unit).astype(np.float64)
        rows, cols, vals = [], [], []
        for m, p in enumerate(lat):
            inside = np.all((p >= self.origin - 1e-9) & (p <= self.origin + side[:, None] + 1e-9), axis=1)
            c = int(np.nonzero(inside)[0][0])
            xi = (p - self.origin[c]) / side[c]
            w1 = [basis.lagrange_values(gll, xi[a])[0] for a in range(3)]
            w = w1[0][self.loc[:, 0]] * w1[1][self.loc[:, 1]] * w1[2][self.loc[:, 2]]
            rows.extend([m] * len(w))
            cols.extend(self.vdofs[c].tolist())
            vals.extend(w.tolist())
        Eraw = sp.csr_matrix((vals, (rows, cols)), shape=(len(lat), self.Nv))
        return (Eraw @ self.C).tocsr()


def scalar_matrices(S: Space):
    """Raw (unconstrained) scalar mass and stiffness matrices by full
    quadrature, for any Space-like object."""
    _, J, det, invJ, JxW = S.geometry()
    q1 = basis.gauss_rule(S.k + 1)[0]
    N, dN, _ = basis.tensor_basis(3, S.k, q1)
    G = np.einsum("qib,cqba->cqia", dN, invJ)
    Me = np.einsum("cq,qi,qj->cij", JxW, N, N)
    Ke = np.einsum("cq,cqia,cqja->cij", JxW, G, G)
    nb = N.shape[1]
    r = np.broadcast_to(S.vdofs[:, :, None], (S.nc, nb, nb)).ravel()
    c = np.broadcast_to(S.vdofs[:, None, :], (S.nc, nb, nb)).ravel()
    M = sp.coo_matrix((Me.ravel(), (r, c)), shape=(S.Nv, S.Nv)).tocsr()
    K = sp.coo_matrix((Ke.ravel(), (r, c)), shape=(S.Nv, S.Nv)).tocsr()
    return M, K


def linearization(S: AmrSpace, u0, nu, dt):
    """Point data of the linearisation point (unknown values u0, 3 blocks)."""
    return ns.linearization_data(S, S.expand(u0, 3), nu, dt)


def jacobian_matrix(S: AmrSpace, u0, nu, dt, newton=True):
    """Constrained SUPG/PSPG Jacobian on the unknowns: C^T J_raw C per
    component block, then identity on the velocity Dirichlet rows."""
    data = linearization(S, u0, nu, dt)
    Jraw = ns.jacobian_matrix(S, data, nu, dt, newton)  # S.dirichlet is empty: unconstrained
    C4 = sp.block_diag([S.C] * 4, format="csr")
    return constrain((C4.T @ Jraw @ C4).tocsr(), S.ns_dirichlet_true())


def jacobian_apply(S: AmrSpace, dx, u0, nu, dt, newton=True, data=None):
    """Constrained Jacobian applied to dx by the element loop (Dirichlet
    source values ignored, identity on Dirichlet rows)."""
    if data is None:
        data = linearization(S, u0, nu, dt)
    mask = S.ns_dirichlet_true()
    y = S.restrict(ns.jacobian_apply(S, S.expand(np.where(mask, 0.0, dx), 4), data, nu, dt, newton), 4)
    y[mask] = dx[mask]
    return y

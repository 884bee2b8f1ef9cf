"""hp Taylor-Hood spaces with the minimum rule (oracle; test infrastructure
only), Sec. 3.

A structured 3D mesh carries one velocity degree k_K per cell (pressure
k_K - 1).  The conforming space is the set of continuous functions that are
Q_{k_K} on every cell; on a face or edge shared by cells of different degree,
continuity forces the trace to the lowest of those degrees (the minimum rule
the paper cites for its hp-multigrid).

Global unknowns, one set per mesh entity (this ordering is the interface
shared with the library):
  1. vertices, lexicographic over the (n0+1)(n1+1)(n2+1) grid (x fastest);
  2. edges along x, then along y, then along z, each set lexicographic over
     its index box (an edge along axis a at (i, j, l) starts at vertex
     (i, j, l)), with m_e - 1 unknowns at the interior points of the
     degree-m_e GLL rule, in increasing order; m_e = the lowest degree of the
     cells that contain the edge;
  3. faces normal to x, then y, then z, lexicographic over their index box,
     with (m_f - 1)^2 unknowns at the interior tensor GLL points of degree
     m_f, the lower free axis fastest; m_f = the lowest degree of the (one or
     two) cells that contain the face;
  4. cell interiors, lexicographic, (k - 1)^3 unknowns each, x fastest.
The function on a face is the degree-m_f tensor interpolant of its vertex
values, of its edge functions evaluated at the degree-m_f GLL points, and of
its interior unknowns; an edge function is the degree-m_e interpolant of its
two vertices and interior unknowns.  A cell's local nodal values (tensor GLL
of degree k, x fastest) are these entity functions evaluated at the cell's
nodes, so every cell operator is C_K^T A_K C_K with the cell's dense element
matrix A_K (full quadrature, oracle.fem) and its sparse map C_K.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.linalg as la
import scipy.sparse as sp

import inputs

from . import basis
from .fem import Space, stokes_element_matrices
from .krylov import fgmres, pcg_fixed
from .mg import chebyshev_smooth


class HpSpace:
    """Scalar continuous space, degree deg[c] on cell c (lexicographic cells)."""

    def __init__(self, n, deg):
        self.n = [int(v) for v in n]
        assert len(self.n) == 3
        n0, n1, n2 = self.n
        self.deg = np.asarray(deg, dtype=np.int64).reshape(-1)
        assert self.deg.size == n0 * n1 * n2 and self.deg.min() >= 1
        self.D = self.deg.reshape(n2, n1, n0)  # [z, y, x]
        self.nvert = (n0 + 1) * (n1 + 1) * (n2 + 1)
        off = self.nvert
        self.edge_deg, self.edge_off, self.edge_box = [], [], []
        for a in range(3):
            box = [self.n[b] + (0 if b == a else 1) for b in range(3)]
            m = np.zeros(box[::-1], dtype=np.int64)  # [z, y, x]
            for idx in itertools.product(*[range(v) for v in box]):
                m[idx[::-1]] = min(self.D[c[::-1]] for c in self._cells_of(idx, [b for b in range(3) if b != a]))
            cnt = (m - 1).ravel()  # x fastest when raveled from [z, y, x]
            o = off + np.concatenate([[0], np.cumsum(cnt)[:-1]])
            self.edge_deg.append(m)
            self.edge_off.append(o.reshape(m.shape))
            self.edge_box.append(box)
            off += int(cnt.sum())
        self.face_deg, self.face_off, self.face_box = [], [], []
        for a in range(3):
            box = [self.n[b] + (1 if b == a else 0) for b in range(3)]
            m = np.zeros(box[::-1], dtype=np.int64)
            for idx in itertools.product(*[range(v) for v in box]):
                m[idx[::-1]] = min(self.D[c[::-1]] for c in self._cells_of(idx, [a]))
            cnt = ((m - 1) ** 2).ravel()
            o = off + np.concatenate([[0], np.cumsum(cnt)[:-1]])
            self.face_deg.append(m)
            self.face_off.append(o.reshape(m.shape))
            self.face_box.append(box)
            off += int(cnt.sum())
        cnt = (self.deg - 1) ** 3
        self.cell_off = off + np.concatenate([[0], np.cumsum(cnt)[:-1]])
        off += int(cnt.sum())
        self.N = off
        self._gll = {}
        self._rows = {}
        self.dirichlet = self._dirichlet_mask()

    # -- helpers -------------------------------------------------------------
    def _cells_of(self, idx, fixed_axes):
        """Cells (x, y, z) containing the entity at index idx whose position is
        fixed (on a grid plane) along fixed_axes."""
        ranges = []
        for b in range(3):
            if b in fixed_axes:
                ranges.append([c for c in (idx[b] - 1, idx[b]) if 0 <= c < self.n[b]])
            else:
                ranges.append([idx[b]])
        return [tuple(c) for c in itertools.product(*ranges)]

    def gll(self, m):
        if m not in self._gll:
            self._gll[m] = basis.gll_points(m)
        return self._gll[m]

    def vertex(self, v):
        n0, n1, _ = self.n
        return int(v[0] + (n0 + 1) * (v[1] + (n1 + 1) * v[2]))

    def _edge(self, a, e, t):
        """{global: weight} of the edge function along axis a at index e,
        evaluated at reference position t in [0, 1]."""
        m = int(self.edge_deg[a][e[::-1]])
        L = basis.lagrange_values(self.gll(m), np.array([t]))[0]
        out = {}
        end = list(e)
        end[a] += 1
        for j in range(m + 1):
            w = L[j]
            if w == 0.0:
                continue
            if j == 0:
                g = self.vertex(e)
            elif j == m:
                g = self.vertex(end)
            else:
                g = int(self.edge_off[a][e[::-1]]) + j - 1
            out[g] = out.get(g, 0.0) + w
        return out

    def _face(self, a, f, s, t):
        """{global: weight} of the face function normal to a at index f, at the
        reference position (s, t) along its free axes (lower axis first)."""
        a1, a2 = [b for b in range(3) if b != a]
        m = int(self.face_deg[a][f[::-1]])
        x = self.gll(m)
        Ls = basis.lagrange_values(x, np.array([s]))[0]
        Lt = basis.lagrange_values(x, np.array([t]))[0]
        out = {}

        def add(d, w):
            for g, v in d.items():
                out[g] = out.get(g, 0.0) + w * v

        for p in range(m + 1):
            for q in range(m + 1):
                w = Ls[p] * Lt[q]
                if w == 0.0:
                    continue
                pe, qe = p in (0, m), q in (0, m)
                shift = list(f)
                if p == m:
                    shift[a1] += 1
                if q == m:
                    shift[a2] += 1
                if pe and qe:
                    add({self.vertex(shift): 1.0}, w)
                elif pe:  # on the edge along a2 at a1 = 0 or 1
                    e = list(f)
                    if p == m:
                        e[a1] += 1
                    add(self._edge(a2, tuple(e), x[q]), w)
                elif qe:
                    e = list(f)
                    if q == m:
                        e[a2] += 1
                    add(self._edge(a1, tuple(e), x[p]), w)
                else:
                    g = int(self.face_off[a][f[::-1]]) + (p - 1) + (m - 1) * (q - 1)
                    add({g: 1.0}, w)
        return out

    def cell_rows(self, c):
        """Sparse local->global map of cell c: CSR matrix [(k+1)^3, N]."""
        if c in self._rows:
            return self._rows[c]
        n0, n1, _ = self.n
        cx, cy, cz = c % n0, (c // n0) % n1, c // (n0 * n1)
        cc = (cx, cy, cz)
        k = int(self.deg[c])
        x = self.gll(k)
        rows, cols, vals = [], [], []
        loc = basis.tensor_index(3, k + 1)
        for r, li in enumerate(loc):
            fixed = [b for b in range(3) if li[b] in (0, k)]
            pos = [cc[b] + (1 if li[b] == k else 0) if b in fixed else cc[b] for b in range(3)]
            if len(fixed) == 3:
                d = {self.vertex(pos): 1.0}
            elif len(fixed) == 2:
                a = [b for b in range(3) if b not in fixed][0]
                d = self._edge(a, tuple(pos), x[li[a]])
            elif len(fixed) == 1:
                a = fixed[0]
                a1, a2 = [b for b in range(3) if b != a]
                d = self._face(a, tuple(pos), x[li[a1]], x[li[a2]])
            else:
                d = {int(self.cell_off[c]) + (li[0] - 1) + (k - 1) * ((li[1] - 1) + (k - 1) * (li[2] - 1)): 1.0}
            for g, w in d.items():
                rows.append(r)
                cols.append(g)
                vals.append(w)
        C = sp.csr_matrix((vals, (rows, cols)), shape=(len(loc), self.N))
        self._rows[c] = C
        return C

    def _dirichlet_mask(self):
        m = np.zeros(self.N, dtype=bool)
        n0, n1, n2 = self.n
        for v in itertools.product(range(n0 + 1), range(n1 + 1), range(n2 + 1)):
            if any(v[b] in (0, self.n[b]) for b in range(3)):
                m[self.vertex(v)] = True
        for a in range(3):
            for idx in itertools.product(*[range(v) for v in self.edge_box[a]]):
                if any(idx[b] in (0, self.n[b]) for b in range(3) if b != a):
                    o = int(self.edge_off[a][idx[::-1]])
                    m[o:o + int(self.edge_deg[a][idx[::-1]]) - 1] = True
            for idx in itertools.product(*[range(v) for v in self.face_box[a]]):
                if idx[a] in (0, self.n[a]):
                    o = int(self.face_off[a][idx[::-1]])
                    m[o:o + (int(self.face_deg[a][idx[::-1]]) - 1) ** 2] = True
        return m

    def reference_points(self):
        """Global reference coordinates ([0, n_a] per axis) of every unknown."""
        P = np.zeros((self.N, 3))
        n0, n1, n2 = self.n
        for v in itertools.product(range(n0 + 1), range(n1 + 1), range(n2 + 1)):
            P[self.vertex(v)] = v
        for a in range(3):
            for idx in itertools.product(*[range(v) for v in self.edge_box[a]]):
                m = int(self.edge_deg[a][idx[::-1]])
                o = int(self.edge_off[a][idx[::-1]])
                for j in range(1, m):
                    p = np.array(idx, dtype=float)
                    p[a] += self.gll(m)[j]
                    P[o + j - 1] = p
            a1, a2 = [b for b in range(3) if b != a]
            for idx in itertools.product(*[range(v) for v in self.face_box[a]]):
                m = int(self.face_deg[a][idx[::-1]])
                o = int(self.face_off[a][idx[::-1]])
                x = self.gll(m)
                for q in range(1, m):
                    for p_ in range(1, m):
                        p = np.array(idx, dtype=float)
                        p[a1] += x[p_]
                        p[a2] += x[q]
                        P[o + (p_ - 1) + (m - 1) * (q - 1)] = p
        for c in range(self.deg.size):
            k = int(self.deg[c])
            cc = np.array([c % n0, (c // n0) % n1, c // (n0 * n1)], dtype=float)
            x = self.gll(k)
            o = int(self.cell_off[c])
            for l in range(1, k):
                for j in range(1, k):
                    for i in range(1, k):
                        P[o + (i - 1) + (k - 1) * ((j - 1) + (k - 1) * (l - 1))] = cc + [x[i], x[j], x[l]]
        return P

    def evaluate(self, x, c, xi):
        """The function with unknowns x on cell c at reference points xi [q, 3]."""
        return _tensor_values(int(self.deg[c]), xi) @ (self.cell_rows(c) @ x)


def _tensor_values(k, xi):
    """[q, (k+1)^3] values of the tensor GLL Lagrange basis at points xi [q, 3]."""
    g = basis.gll_points(k)
    Lx = basis.lagrange_values(g, xi[:, 0])
    Ly = basis.lagrange_values(g, xi[:, 1])
    Lz = basis.lagrange_values(g, xi[:, 2])
    return np.einsum("qi,qj,ql->qlji", Lx, Ly, Lz).reshape(xi.shape[0], -1)


# ---------------------------------------------------------------------------
# hp Stokes system
# ---------------------------------------------------------------------------
class HpStokes:
    """Constrained hp Taylor-Hood Stokes matrix: velocity degree deg[c],
    pressure deg[c] - 1 on every cell, blocked [u_0 | u_1 | u_2 | p]."""

    def __init__(self, n, X, deg, nu):
        self.n = [int(v) for v in n]
        self.X = X
        self.deg = np.asarray(deg, dtype=np.int64).reshape(-1)
        self.nu = nu
        self.V = HpSpace(n, self.deg)
        self.Pspace = HpSpace(n, self.deg - 1)
        Nu, Np = self.V.N, self.Pspace.N
        self.Nu, self.Np = Nu, Np
        Ablk, Bblk, Mblk = [], [], []
        Cu, Cp = [], []
        order = []
        for k in sorted(set(self.deg.tolist())):
            cells = np.nonzero(self.deg == k)[0]
            S = Space(3, self.n, X, int(k), int(k) - 1)
            em = stokes_element_matrices(S, nu, cells)
            for i, c in enumerate(cells):
                order.append(c)
                Ablk.append(em["A"][i])
                Bblk.append(em["B"][i])
                Mblk.append(em["M"][i])
                Cu.append(self.V.cell_rows(int(c)))
                Cp.append(self.Pspace.cell_rows(int(c)))
        CU = sp.vstack(Cu).tocsr()
        CP = sp.vstack(Cp).tocsr()
        A = (CU.T @ sp.block_diag(Ablk) @ CU).tocsr()
        # B element blocks are [comp*nb + i, j]; expand the velocity map per component
        CU3 = sp.vstack([sp.block_diag([C] * 3) for C in Cu]).tocsr()
        B = (CU3.T @ sp.block_diag(Bblk) @ CP).tocsr()
        M = (CP.T @ sp.block_diag(Mblk) @ CP).tocsr()
        self.A, self.B, self.M = A, B, M
        self.Avec = sp.block_diag([A] * 3, format="csr")
        mask_u = np.tile(self.V.dirichlet, 3)
        self.mask = np.concatenate([mask_u, np.zeros(Np, dtype=bool)])
        K = sp.bmat([[self.Avec, B], [B.T, None]], format="csr")
        z = sp.diags((~self.mask).astype(np.float64))
        self.K = (z @ K @ z + sp.diags(self.mask.astype(np.float64))).tocsr()
        self.nvel = 3 * Nu


def sampled_stokes_rows(n, X, deg, nu, x, rows, V=None, Pspace=None):
    """Rows ``rows`` of the constrained hp Stokes operator (the matrix of
    ``HpStokes``) applied to x = [u_0 | u_1 | u_2 | p], each from the cells
    whose local maps reference the row's unknown: element matrices of those
    cells by full quadrature, C_K^T (A_K, B_K) C_K.  For sizes too large to
    assemble; V and Pspace may be passed in (the velocity and pressure spaces)."""
    n = [int(v) for v in n]
    deg = np.asarray(deg, dtype=np.int64).reshape(-1)
    V = HpSpace(n, deg) if V is None else V
    Pspace = HpSpace(n, deg - 1) if Pspace is None else Pspace
    Nu, Np = V.N, Pspace.N
    nv = 3 * Nu
    xu = np.where(np.tile(V.dirichlet, 3), 0.0, x[:nv])
    xp = x[nv:]
    refV, refP = V.reference_points(), Pspace.reference_points()
    n0, n1, n2 = n
    cache, spaces = {}, {}

    def cell_data(c):
        if c not in cache:
            k = int(deg[c])
            if k not in spaces:
                spaces[k] = Space(3, n, X, k, k - 1)
            S = spaces[k]
            CU, CP = V.cell_rows(c), Pspace.cell_rows(c)
            u_loc = np.stack([CU @ xu[a * Nu:(a + 1) * Nu] for a in range(3)])  # [3, nb]
            p_loc = CP @ xp
            # the element matrices of the cell (full quadrature, as in
            # stokes_element_matrices) applied to its local values:
            # A_ij = nu sum_q JxW grad phi_i . grad phi_j,
            # B_(a i) j = - sum_q JxW psi_j d phi_i / dx_a
            _, _, _, invJ, JxW = S.geometry(np.array([c]))
            q1 = basis.gauss_rule(k + 1)[0]
            _, dN, _ = basis.tensor_basis(3, k, q1)
            Np_, _, _ = basis.tensor_basis(3, k - 1, q1)
            G = np.einsum("qib,qba->qia", dN, invJ[0])  # physical gradients [q, i, a]
            w = JxW[0]
            gu = np.einsum("qja,cj->cqa", G, u_loc)  # gradients of the 3 components at the points
            pq = Np_ @ p_loc
            ru = np.stack([nu * np.einsum("q,qia,qa->i", w, G, gu[a]) - np.einsum("q,q,qi->i", w, pq, G[:, :, a])
                           for a in range(3)])
            div = gu[0, :, 0] + gu[1, :, 1] + gu[2, :, 2]
            rp = -np.einsum("q,q,qj->j", w, div, Np_)
            cache[c] = (CU, CP, ru, rp)
        return cache[c]

    def cells_at(pt):
        ranges = []
        for b in range(3):
            f = int(np.floor(pt[b] + 1e-12))
            cand = [f - 1, f] if abs(pt[b] - round(pt[b])) < 1e-12 else [f]
            ranges.append([c for c in cand if 0 <= c < n[b]])
        return [cx + n0 * (cy + n1 * cz) for cz in ranges[2] for cy in ranges[1] for cx in ranges[0]]

    out = np.zeros(len(rows))
    for t, r in enumerate(rows):
        r = int(r)
        if r < nv:
            a, g = divmod(r, Nu)
            if V.dirichlet[g]:
                out[t] = x[r]
                continue
            for c in cells_at(refV[g]):
                CU, _, ru, _ = cell_data(c)
                out[t] += CU[:, g].toarray().ravel() @ ru[a]
        else:
            g = r - nv
            for c in cells_at(refP[g]):
                _, CP, _, rp = cell_data(c)
                out[t] += CP[:, g].toarray().ravel() @ rp
    return out


def random_block_degrees(n, seed, block=4, lo=2, hi=6):
    """Per-cell degrees constant on block^3 cell blocks, uniform in [lo, hi]
    per block (input recipe of the hp workload)."""
    return inputs.block_degrees(n, seed, block, lo, hi)


# ---------------------------------------------------------------------------
# hp multigrid (velocity block): p-levels k_K <- max(k_K - 1, p_low), then
# h-levels on the uniform-degree mesh
# ---------------------------------------------------------------------------
def hp_transfer(Vf: HpSpace, Vc: HpSpace, constrained=True):
    """Prolongation coarse -> fine on the same mesh: every fine unknown takes
    the coarse function's value at its point (the coarse space is contained
    in the fine one).  Dirichlet rows / columns zero when constrained."""
    n0, n1, _ = Vf.n
    Pf = Vf.reference_points()
    rows, cols, vals = [], [], []
    # the cell containing each point (lowest index on shared boundaries)
    cell_idx = np.minimum(np.floor(Pf).astype(np.int64), np.array(Vf.n) - 1)
    cid = cell_idx[:, 0] + n0 * (cell_idx[:, 1] + n1 * cell_idx[:, 2])
    for c in np.unique(cid):
        sel = np.nonzero(cid == c)[0]
        xi = Pf[sel] - cell_idx[sel]
        Nc = _tensor_values(int(Vc.deg[c]), xi) @ Vc.cell_rows(int(c))
        Nc = sp.csr_matrix(Nc)
        r, cc = Nc.nonzero()
        rows.extend(sel[r].tolist())
        cols.extend(cc.tolist())
        vals.extend(np.asarray(Nc[r, cc]).ravel().tolist())
    P = sp.csr_matrix((vals, (rows, cols)), shape=(Vf.N, Vc.N))
    if constrained:
        P = sp.diags((~Vf.dirichlet).astype(float)) @ P @ sp.diags((~Vc.dirichlet).astype(float))
    return P.tocsr()


def structured_permutation(V: HpSpace, S: Space):
    """Matrix Pi with x_hp = Pi x_struct for a uniform-degree hp space and the
    structured space of the same degree (same functions, other numbering);
    points matched by reference coordinates."""
    k = S.k
    g = basis.gll_points(k)
    axes = []
    for na in S.n:
        idx = np.arange(k * na + 1)
        c = np.minimum(idx // k, na - 1)
        axes.append(c + g[idx - k * c])
    zz, yy, xx = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    ps = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], -1)
    ph = V.reference_points()
    key = lambda p: [tuple(v) for v in np.round(p * 2 ** 30).astype(np.int64)]  # noqa: E731
    pos = {v: i for i, v in enumerate(key(ps))}
    cols = np.array([pos[v] for v in key(ph)])
    return sp.csr_matrix((np.ones(V.N), (np.arange(V.N), cols)), shape=(V.N, S.Nv))


class HpHierarchy:
    """Velocity-block multigrid of the hp Stokes solver: hp p-levels with
    k_K <- max(k_K - 1, 2) until every degree is 2, then the structured
    degree-2 h-hierarchy (oracle.mg) down to coarse_min cells per direction."""

    def __init__(self, n, X, deg, nu, coarse_min=2, cheb_degree=5, cheb_range=20.0):
        from .mg import Hierarchy

        self.nu = nu
        degs = [np.asarray(deg, dtype=np.int64).reshape(-1)]
        while degs[-1].max() > 2:
            degs.append(np.maximum(degs[-1] - 1, 2))
        if len(degs) > 1:
            degs.pop()  # the uniform degree-2 level is the structured one
        self.hp = []
        for d in degs:
            V = HpSpace(n, d)
            A = self._scalar_A(n, X, d, V, nu)
            self.hp.append((V, A))
        self.mg = Hierarchy(3, n, X, 2, nu, p_min=2, coarse_min=coarse_min, cheb_degree=cheb_degree,
                            cheb_range=cheb_range)
        self.A, self.Dinv, self.fixed, self.P = [], [], [], []
        for V, A in self.hp:
            z = sp.diags((~V.dirichlet).astype(float))
            Ac = (z @ A @ z + sp.diags(V.dirichlet.astype(float))).tocsr()
            self.A.append(sp.block_diag([Ac] * 3, format="csr"))
            self.Dinv.append(np.tile(1.0 / Ac.diagonal(), 3))
            self.fixed.append(np.tile(V.dirichlet, 3))
        for l in range(len(self.hp) - 1):
            self.P.append(sp.block_diag([hp_transfer(self.hp[l][0], self.hp[l + 1][0])] * 3, format="csr"))
        # last hp level -> structured degree-2 level: evaluate, then renumber
        Vl = self.hp[-1][0]
        S0 = self.mg.spaces[0]
        V2 = HpSpace(n, np.full(Vl.deg.size, 2))
        Pi = structured_permutation(V2, S0)
        T = hp_transfer(Vl, V2, constrained=False) @ Pi
        z = sp.diags((~Vl.dirichlet).astype(float))
        zc = sp.diags((~S0.dirichlet).astype(float))
        self.P.append(sp.block_diag([(z @ T @ zc).tocsr()] * 3, format="csr"))
        self.cheb_degree, self.cheb_range = cheb_degree, cheb_range
        self.lam = [None] * len(self.hp)

    @staticmethod
    def _scalar_A(n, X, d, V, nu):
        blocks, C = [], []
        for k in sorted(set(d.tolist())):
            cells = np.nonzero(d == k)[0]
            S = Space(3, n, X, int(k), int(k) - 1)
            em = stokes_element_matrices(S, nu, cells)
            for i, c in enumerate(cells):
                blocks.append(em["A"][i])
                C.append(V.cell_rows(int(c)))
        CC = sp.vstack(C).tocsr()
        return (CC.T @ sp.block_diag(blocks) @ CC).tocsr()

    def exact_lambda_max(self, l):
        A = self.A[l].toarray()
        free = ~self.fixed[l]
        d = np.sqrt(self.Dinv[l][free])
        return float(la.eigvalsh(d[:, None] * A[np.ix_(free, free)] * d[None, :])[-1])

    def vcycle(self, b, l=0):
        if l == len(self.hp):
            return self.mg.vcycle(b, 0)
        x = np.where(self.fixed[l], b, 0.0)
        x = chebyshev_smooth(self.A[l], self.Dinv[l], self.fixed[l], self.lam[l], self.cheb_range,
                             self.cheb_degree, x, b, True)
        r = b - self.A[l] @ x
        xc = self.vcycle(self.P[l].T @ r, l + 1)
        x = x + self.P[l] @ xc
        return chebyshev_smooth(self.A[l], self.Dinv[l], self.fixed[l], self.lam[l], self.cheb_range,
                                self.cheb_degree, x, b, False)


class HpStokesSolver:
    """Block preconditioner (Sec. 3 eq. (stokes_block)) and FGMRES on the hp
    Stokes system, as for the structured solver."""

    def __init__(self, n, X, deg, nu, schur_iterations=10, **mg_kw):
        self.sys = HpStokes(n, X, deg, nu)
        self.mg = HpHierarchy(n, X, deg, nu, **mg_kw)
        self.nu = nu
        self.schur_iterations = schur_iterations
        s = self.sys
        self.Bc = s.K[:s.nvel, s.nvel:]
        self.Mdinv = 1.0 / s.M.diagonal()

    def precondition(self, r):
        s = self.sys
        z = pcg_fixed(s.M, self.Mdinv, r[s.nvel:], self.schur_iterations)
        yp = -self.nu * z
        yu = self.mg.vcycle(r[:s.nvel] - self.Bc @ yp)
        return np.concatenate([yu, yp])

    def solve(self, b, rtol=1e-8, restart=30, maxit=200):
        s = self.sys
        x0 = np.where(s.mask, b, 0.0)
        x, its, rel = fgmres(s.K, b, self.precondition, x0, rtol, restart, maxit)
        # zero mass-weighted pressure mean
        p = x[s.nvel:]
        one = np.ones(s.Np)
        x[s.nvel:] = p - (one @ (s.M @ p)) / (one @ (s.M @ one))
        return x, its, rel

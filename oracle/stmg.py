"""hp space-time multigrid (hp-STMG) for the transient Stokes stage system
(oracle; test infrastructure only), Sec. 4: GMRES preconditioned by one
V-cycle on the Kronecker operator of eq. (proceedings-kronecker), levels
coarsened polynomially and geometrically in space and polynomially in time,
tensor-product transfers applied one factor at a time, a space-time additive
Schwarz smoother on vertex-star patches, a direct solve on the coarsest level.

Readings where the paper is silent:
* Spaces: Taylor-Hood Q_k / Q_{k-1} (continuous pressure) on every level, the
  pair the spatial operators here are built for (the paper names the
  discontinuous-pressure pair as one option among others).
* Level order, by the two rules of Sec. 4 (space before time; polynomial
  before geometric) with no geometric coarsening in time (time marching):
  all of space first, the spatial degree k -> k-1 -> ... -> 2 and then h
  (n halved while every n is even and larger than ``coarse_min``; a coarse
  mesh keeps the fine vertices of even index), all at the temporal degree
  kt; then on the coarsest mesh the temporal degree kt -> ... -> 0 (DG(0),
  one stage).  Lowering the temporal degree on the fine mesh instead (space
  p, time p, then h) leaves the modes that are smooth in space and of high
  degree in time to neither the spatially local smoother nor a coarse level:
  on 2D Q2/Q1 with DG(1) it took 34, 87 and 150 FGMRES iterations on 16^2,
  32^2 and 64^2 cells (nu = 1) where this order takes 12, 14 and 17.
* Spatial transfer, per stage: the constrained Lagrange transfer of the
  velocity multigrid for every component, and the same transfer without
  constraints for the pressure of degree k-1.  Temporal transfer: the coarse
  DG polynomial at the fine temporal nodes per spatial unknown (P_tau).
  Restriction: the transpose in space; in time M_c^{-1} P_tau^T M_f, the L2
  projection onto the coarse temporal space, because the stage rows are
  mass-scaled (M_Q^{-1} from the left).  With it the coarse temporal operator
  is the Galerkin one.  (With the level order above the plain transpose
  takes the same iteration counts within one on small cases; with time
  coarsened on the fine mesh it took up to 4x more.)
* Smoother: additive Schwarz over vertex-star patches with the temporal
  direction whole (the paper names cell patches and vertex-star patches;
  with the continuous pressure here the cell patches share every pressure
  node, and their smoother diverged undamped and needed 19-53 iterations
  damped, against 10-15 for these patches, on five small 2D and 3D cases).  Patch v holds, in every stage, every velocity component at the
  velocity nodes i with |i_a - k v_a| < k and the pressure at the pressure
  nodes j with |j_a - (k-1) v_a| < k-1 (the open vertex star), Dirichlet
  rows left out; its matrix is the principal submatrix of the level
  operator, inverted exactly; the corrections are weighted by 1/m_i, m_i the
  number of patches holding unknown i.  ``steps`` relaxation steps
  x <- x + omega B (b - K x) before and after the coarse correction; reading
  steps = 2, omega = 0.5 (omega = 1 diverges on 16^2 cells).
* Every level starts from x = b on the Dirichlet rows, 0 elsewhere.
* Coarsest level: the constrained operator has the constant pressure of each
  stage in its kernel (all boundary velocity is Dirichlet), so the direct
  solve pins the first pressure node of every stage to zero: its row and
  column are replaced by the identity and its right-hand side entry by 0
  (for a consistent right-hand side this solves the singular system).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as la
import scipy.sparse as sp

import inputs

from . import asm, krylov, spacetime
from .fem import Space, _multi_index
from .mg import transfer_matrix


def level_specs(n, k, kt, coarse_min=2):
    """[(n_list, k, kt, h_index)] from fine to coarse."""
    n = list(n)
    out = [(list(n), k, kt, 0)]
    kk, tt, hl = k, kt, 0
    while kk > 2:
        kk -= 1
        out.append((list(n), kk, tt, hl))
    while all(v % 2 == 0 and v > max(1, coarse_min) for v in n):
        n = [v // 2 for v in n]
        hl += 1
        out.append((list(n), kk, tt, hl))
    while tt > 0:
        tt -= 1
        out.append((list(n), kk, tt, hl))
    return out


def spatial_transfer(Sf: Space, Sc: Space) -> sp.csr_matrix:
    """Prolongation of one stage [u_0 | .. | p]: constrained velocity
    components, unconstrained pressure of degree k-1."""
    h = Sf.n != Sc.n
    Pv = transfer_matrix(Sf, Sc, h)
    pf = Space(Sf.dim, Sf.n, Sf.X, Sf.kp, 0)
    pc = Space(Sc.dim, Sc.n, Sc.X, Sc.kp, 0)
    Pp = transfer_matrix(pf, pc, h, constrained=False)
    return sp.block_diag([Pv] * Sf.dim + [Pp], format="csr")


def vertex_patches(S: Space, Q: int):
    """Unknown indices of every vertex-star patch over Q stages
    (stage-major, vertex-lexicographic order), the Dirichlet rows left out."""
    mask = S.velocity_dirichlet_mask()
    N = S.n_dofs
    vn = _multi_index([a - 1 for a in S.vaxes], inclusive=True)
    pn = _multi_index([a - 1 for a in S.paxes], inclusive=True)
    out = []
    for v in _multi_index(S.n, inclusive=True):
        iv = np.flatnonzero(np.all(np.abs(vn - S.k * v[None, :]) < S.k, axis=1))
        ip = np.flatnonzero(np.all(np.abs(pn - S.kp * v[None, :]) < S.kp, axis=1))
        dofs = np.concatenate([f * S.Nv + iv for f in range(S.dim)] + [S.dim * S.Nv + ip])
        dofs = dofs[~mask[dofs]]
        out.append(np.sort(np.concatenate([q * N + dofs for q in range(Q)])))
    return out


def time_restriction(kf: int, kc: int) -> np.ndarray:
    """R_tau [Q_c, Q_f] = M_c^{-1} P_tau^T M_f: the stage rows are
    mass-scaled, so the restriction is the L2 projection onto the coarse
    temporal space, under which the coarse operator is the Galerkin one."""
    Mf = spacetime.time_matrices(kf)[0]
    Mc = spacetime.time_matrices(kc)[0]
    return np.linalg.solve(Mc, spacetime.time_prolongation(kf, kc).T @ Mf)


def pinned_coarse_matrix(K: np.ndarray, S: Space, Q: int) -> np.ndarray:
    """Dense K with the first pressure node of every stage pinned."""
    A = K.copy()
    N = S.n_dofs
    for q in range(Q):
        i = q * N + S.dim * S.Nv
        A[i, :] = 0.0
        A[:, i] = 0.0
        A[i, i] = 1.0
    return A


class STMG:
    """Levels, operators, transfers, smoothers and the V-cycle."""

    def __init__(self, dim, n, X, k, kt, nu, tau, coarse_min=2, steps=2, omega=0.5):
        self.specs = level_specs(n, k, kt, coarse_min)
        self.nu, self.tau, self.steps, self.omega = nu, tau, steps, omega
        self.spaces, self.Q, self.K, self.fixed, self.smoother = [], [], [], [], []
        for nl, kl, tl, hl in self.specs:
            Xl = inputs.coarsen_vertices(dim, n, X, hl) if hl > 0 else X
            S = Space(dim, nl, Xl, kl, kl - 1)
            Q = tl + 1
            K = spacetime.kron_operator(S, nu, tau, spacetime.G_matrix(tl))
            self.spaces.append(S)
            self.Q.append(Q)
            self.K.append(K)
            self.fixed.append(np.tile(S.velocity_dirichlet_mask(), Q))
        for l in range(len(self.spaces) - 1):
            self.smoother.append(asm.ASM(self.K[l], vertex_patches(self.spaces[l], self.Q[l])))
        self.P, self.R = [], []
        for l in range(len(self.spaces) - 1):
            Sf, Sc = self.spaces[l], self.spaces[l + 1]
            if self.Q[l] != self.Q[l + 1]:
                Pt = spacetime.time_prolongation(self.specs[l][2], self.specs[l + 1][2])
                Rt = time_restriction(self.specs[l][2], self.specs[l + 1][2])
                I = sp.identity(Sf.n_dofs)
                self.P.append(sp.kron(sp.csr_matrix(Pt), I, format="csr"))
                self.R.append(sp.kron(sp.csr_matrix(Rt), I, format="csr"))
            else:
                self.P.append(sp.kron(sp.identity(self.Q[l]), spatial_transfer(Sf, Sc), format="csr"))
                self.R.append(self.P[-1].T.tocsr())
        Sc = self.spaces[-1]
        self.coarse = la.lu_factor(pinned_coarse_matrix(self.K[-1].toarray(), Sc, self.Q[-1]))
        self.pinned = np.array([q * Sc.n_dofs + Sc.dim * Sc.Nv for q in range(self.Q[-1])])

    @property
    def n_levels(self):
        return len(self.spaces)

    def relax(self, l, x, b):
        return asm.relax(self.K[l], self.smoother[l], x, b, self.steps, self.omega)

    def vcycle(self, b, l=0):
        if l == self.n_levels - 1:
            b = b.copy()
            b[self.pinned] = 0.0
            return la.lu_solve(self.coarse, b)
        x = np.where(self.fixed[l], b, 0.0)
        x = self.relax(l, x, b)
        r = b - self.K[l] @ x
        xc = self.vcycle(self.R[l] @ r, l + 1)
        x = x + self.P[l] @ xc
        return self.relax(l, x, b)

    def solve(self, b, rtol=1e-8, restart=30, maxit=200):
        """FGMRES on the finest level, one V-cycle per iteration, from x = 0."""
        return krylov.fgmres(self.K[0], b, self.vcycle, np.zeros_like(b), rtol, restart, maxit)

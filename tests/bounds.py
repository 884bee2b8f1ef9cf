"""Error bounds for solver results, computed from the oracle's assembled
system (test infrastructure)."""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import fem


def bordered_error_bound(S, nu, b, x, mats):
    """Oracle-side bound on ||x - x*||_2 for the exact solution x* of the
    constrained Stokes system with zero-mean pressure: x* solves the bordered
    system Kb [x; 0] = [b; 0] with Kb = [[K, e], [e^T, 0]], e = (0, M_p 1),
    which is symmetric and nonsingular, so ||x - x*|| <= ||Kb^-1|| ||r_b|| =
    ||r_b|| / |lambda|_min(Kb) with r_b = [b - K x; -e^T x]."""
    K = fem.constrain(mats["K"], S.velocity_dirichlet_mask())
    e = np.zeros(S.n_dofs)
    e[S.dim * S.Nv:] = mats["M"] @ np.ones(S.Np)
    Kb = sp.bmat([[K, sp.csr_matrix(e[:, None])], [sp.csr_matrix(e[None, :]), None]], format="csc")
    # the constrained K is not symmetric (identity Dirichlet rows, zero
    # Dirichlet columns); symmetrise by dropping the Dirichlet columns' zeros:
    # its eigenvalues on the free block plus ones on the Dirichlet rows
    mask = np.concatenate([S.velocity_dirichlet_mask(), [False]])
    free = np.flatnonzero(~mask)
    Kf = Kb[free][:, free]
    lam_min = abs(spla.eigsh(Kf, k=1, sigma=0.0, which="LM", return_eigenvectors=False)[0])
    lam_min = min(lam_min, 1.0)  # the identity rows
    rb = np.concatenate([b - K @ x, [-(e @ x)]])
    return np.linalg.norm(rb) / lam_min, lam_min

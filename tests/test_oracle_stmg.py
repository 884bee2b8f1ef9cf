"""Pins of the oracle's hp space-time multigrid (Sec. 4): the level order of
the two coarsening rules, the temporal transfers against the polynomial
exactness that fixes them (the restriction of the mass-scaled stage rows
makes the coarse temporal operator the Galerkin one), the spatial
Taylor-Hood transfers against the Galerkin identity of nested Cartesian
spaces, the vertex-star patches against their closed-form sizes and the
Kronecker structure of their matrices, the coarse correction of the V-cycle
on a Galerkin hierarchy, and the contraction of the whole V-cycle."""
import numpy as np
import pytest

import inputs
from oracle import spacetime, stmg
from oracle.fem import Space, assemble_stokes, constrain


def test_level_order():
    """Space first (p, then h), then the temporal degree on the coarsest mesh
    (no geometric coarsening in time); written out by hand from the two
    rules."""
    got = [(tuple(n), k, kt) for n, k, kt, _ in stmg.level_specs([8, 4], 4, 2)]
    # h stops once a direction has coarse_min = 2 cells; time on the coarsest mesh
    assert got == [((8, 4), 4, 2), ((8, 4), 3, 2), ((8, 4), 2, 2), ((4, 2), 2, 2), ((4, 2), 2, 1),
                   ((4, 2), 2, 0)]
    assert [(tuple(n), k, kt) for n, k, kt, _ in stmg.level_specs([3, 3], 2, 0)] == [((3, 3), 2, 0)]


@pytest.mark.parametrize("kf,kc", [(1, 0), (2, 1), (3, 2), (3, 1), (2, 0)])
def test_time_transfers(kf, kc):
    """P_tau carries the coarse polynomial to the fine nodes, R_tau P_tau = I
    (projection), and R_tau G_f P_tau = G_c: the fine temporal operator on
    coarse polynomials is the coarse one (exact integration of the mass,
    derivative and upwind jump of nested polynomial spaces)."""
    P = spacetime.time_prolongation(kf, kc)
    R = stmg.time_restriction(kf, kc)
    sc, sf = spacetime.time_nodes(kc), spacetime.time_nodes(kf)
    for d in range(kc + 1):
        assert np.allclose(P @ sc ** d, sf ** d, atol=1e-13)
    assert np.allclose(R @ P, np.eye(kc + 1), atol=1e-12)
    assert np.allclose(R @ spacetime.G_matrix(kf) @ P, spacetime.G_matrix(kc), atol=1e-11)
    # the plain transpose is not a projection once the coarse space has
    # more than the constants (the reading this restriction replaces)
    if kc >= 1:
        assert not np.allclose(P.T @ spacetime.G_matrix(kf) @ P, spacetime.G_matrix(kc), atol=1e-3)


@pytest.mark.parametrize("dim,nf,nc,kf,kc", [(2, [4, 6], [4, 6], 3, 2), (2, [4, 6], [2, 3], 2, 2),
                                            (3, [2, 2, 2], [2, 2, 2], 3, 2), (3, [4, 2, 2], [2, 1, 1], 2, 2)])
def test_spatial_transfer_galerkin(dim, nf, nc, kf, kc):
    """On nested Cartesian meshes with exact quadrature the restricted fine
    Stokes operator and block mass are the coarse ones on the free unknowns:
    R K_f P = K_c, with R = P^T over velocity (constrained) and pressure
    (degree k - 1, unconstrained)."""
    Xf = inputs.structured_vertices(dim, nf, noise=0.0)
    Xc = inputs.structured_vertices(dim, nc, noise=0.0)
    Sf, Sc = Space(dim, nf, Xf, kf, kf - 1), Space(dim, nc, Xc, kc, kc - 1)
    P = stmg.spatial_transfer(Sf, Sc)
    free = ~Sc.velocity_dirichlet_mask()
    for op in ("K", "M"):
        if op == "K":
            Kf = constrain(assemble_stokes(Sf, 0.7)["K"], Sf.velocity_dirichlet_mask())
            Kc = constrain(assemble_stokes(Sc, 0.7)["K"], Sc.velocity_dirichlet_mask())
        else:
            Kf, Kc = spacetime.block_mass(Sf), spacetime.block_mass(Sc)
        RKP = (P.T @ Kf @ P).toarray()
        ref = Kc.toarray()
        assert np.allclose(RKP[np.ix_(free, free)], ref[np.ix_(free, free)], atol=1e-12)
    # the pressure part reproduces the coarse pressure field at the fine
    # pressure nodes (linear fields are in every pressure space here)
    pf = Sf.support_points(Sf.kp)
    pc = Sc.support_points(Sc.kp)
    f = lambda x: 0.3 + x @ np.arange(1, dim + 1)
    xc = np.zeros(Sc.n_dofs)
    xc[dim * Sc.Nv:] = f(pc)
    assert np.allclose((P @ xc)[dim * Sf.Nv:], f(pf), atol=1e-13)


@pytest.mark.parametrize("dim,n,k", [(2, [4, 3], 2), (2, [4, 4], 3), (3, [2, 3, 2], 2)])
def test_vertex_patches(dim, n, k):
    """An interior vertex's patch holds (2k-1)^d velocity nodes per component
    and (2k-3)^d pressure nodes (the open star); every free unknown lies in
    some patch; and a patch matrix over Q stages is G (x) M_J + tau I (x) A_J
    on the patch's spatial unknowns J (stage-major index layout)."""
    X = inputs.structured_vertices(dim, n, noise=0.1, seed=2)
    S = Space(dim, n, X, k, k - 1)
    Q, tau = 2, 0.3
    N = S.n_dofs
    P = stmg.vertex_patches(S, Q)
    assert len(P) == int(np.prod([a + 1 for a in n]))
    vidx = np.stack(np.meshgrid(*[np.arange(a + 1) for a in n], indexing="ij"), 0).reshape(dim, -1, order="F").T
    nvel, npres = (2 * k - 1) ** dim, (2 * k - 3) ** dim
    for v, I in zip(vidx, P):
        if np.all((v > 0) & (v < np.array(n))):
            J = I[I < N]
            assert len(J) == dim * nvel + npres
    covered = np.zeros(Q * N, dtype=bool)
    for I in P:
        covered[I] = True
    assert np.array_equal(covered, ~np.tile(S.velocity_dirichlet_mask(), Q))
    G = spacetime.G_matrix(Q - 1)
    K = spacetime.kron_operator(S, 1.3, tau, G)
    M = spacetime.block_mass(S)
    A = constrain(assemble_stokes(S, 1.3)["K"], S.velocity_dirichlet_mask())
    for I in P[:: max(1, len(P) // 5)]:
        J = I[I < N]
        assert np.array_equal(I, np.concatenate([q * N + J for q in range(Q)]))
        ref = np.kron(G, M[J][:, J].toarray()) + tau * np.kron(np.eye(Q), A[J][:, J].toarray())
        assert np.allclose(K[I][:, I].toarray(), ref, atol=1e-13)


def test_coarse_correction_galerkin():
    """Without smoothing the V-cycle is the coarse correction P_tot x_c; on a
    Cartesian hierarchy (Galerkin in space and time) the restricted residual
    after it vanishes: R_tot (b - K P_tot x_c) = 0."""
    H = stmg.STMG(2, [4, 4], inputs.structured_vertices(2, [4, 4], noise=0.0), 3, 1, nu=0.9, tau=0.2, steps=0)
    assert [(s[0], s[1], s[2]) for s in H.specs] == [([4, 4], 3, 1), ([4, 4], 2, 1), ([2, 2], 2, 1), ([2, 2], 2, 0)]
    rng = np.random.default_rng(4)
    N = H.K[0].shape[0]
    xt = rng.uniform(-1, 1, N)
    xt[H.fixed[0]] = 0.0
    b = H.K[0] @ xt
    x = H.vcycle(b)
    r = b - H.K[0] @ x
    for R in H.R:
        r = R @ r
    assert np.abs(r).max() <= 1e-11 * np.abs(b).max()


@pytest.mark.parametrize("dim,n,k,kt", [(2, [8, 8], 2, 1), (2, [8, 8], 3, 1), (3, [4, 4, 4], 2, 1)])
def test_vcycle_contracts_and_solves(dim, n, k, kt):
    """Three V-cycles as a stationary iteration cut the residual at least 20x,
    and FGMRES with one V-cycle per iteration reaches 1e-10 in at most 40
    iterations, with K x = b (the pressure up to its constant per stage)."""
    X = inputs.structured_vertices(dim, n, noise=0.1, seed=3)
    H = stmg.STMG(dim, n, X, k, kt, nu=1.0, tau=0.05)
    K = H.K[0]
    N = K.shape[0]
    rng = np.random.default_rng(0)
    xt = rng.uniform(-1, 1, N)
    xt[H.fixed[0]] = 0.0
    b = K @ xt
    x = np.zeros(N)
    for _ in range(3):
        x = x + H.vcycle(b - K @ x)
    assert np.linalg.norm(b - K @ x) <= np.linalg.norm(b) / 20
    x, its, rel = H.solve(b, rtol=1e-10)
    assert rel <= 1e-10 and its <= 40
    assert np.linalg.norm(b - K @ x) <= 1e-9 * np.linalg.norm(b)

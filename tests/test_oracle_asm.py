"""Pins of the oracle's additive Schwarz relaxation (Sec. 2, Sec. 5 Exp. 4):
the vertex patches against the combinatorial vertex star, the multiplicity
against its closed form, the weighted sum of local inverses against a
hand-computed 3 x 3 case, point-block Jacobi for Q1, the exact solve of a
single all-covering patch, and the smoother inside the monolithic V-cycle."""
import numpy as np
import pytest
import scipy.sparse as sp

import inputs
from oracle import asm, ns, ns_mg
from oracle.fem import Space


def _space(dim, n, k, noise=0.1, seed=0):
    return Space(dim, n, inputs.structured_vertices(dim, n, noise=noise, seed=seed), k, k)


@pytest.mark.parametrize("dim,n,k", [(2, [3, 4], 2), (3, [3, 2, 3], 2), (3, [2, 3, 2], 1), (2, [3, 3], 3)])
def test_patches_are_vertex_star_interiors(dim, n, k):
    """Patch of vertex v = the nodes of the cells at v that no other cell
    holds, with the mesh surrounded by one layer of ghost cells (so that a
    boundary vertex's star keeps its domain-boundary nodes, and the star of a
    vertex next to the boundary does not reach past it), restricted to the
    domain's nodes.  Built on the ghost mesh from cell-to-node and
    cell-to-vertex maps only."""
    S = _space(dim, n, k)
    fixed = ns.ns_dirichlet_mask(S)
    P = asm.patches(S, fixed)
    assert len(P) == S.cell_vertices.max() + 1
    G = Space(dim, [a + 2 for a in n], inputs.structured_vertices(dim, [a + 2 for a in n]), k, k)
    gnode = asm.node_multi_index(G) - k  # ghost-mesh node -> domain lattice index
    inside = np.all((gnode >= 0) & (gnode <= k * np.array(n)), axis=1)
    strides = np.cumprod([1] + [k * a + 1 for a in n[:-1]])
    dnode = (gnode * strides).sum(1)
    gvert = asm.vertex_multi_index(G) - 1
    vstrides = np.cumprod([1] + [a + 1 for a in n[:-1]])
    for gv in np.flatnonzero(np.all((gvert >= 0) & (gvert <= np.array(n)), axis=1)):
        v = int((gvert[gv] * vstrides).sum())
        star = np.flatnonzero((G.cell_vertices == gv).any(1))
        other = np.setdiff1d(np.arange(G.nc), star)
        gn = np.setdiff1d(np.unique(G.vdofs[star]), np.unique(G.vdofs[other]))
        nodes = dnode[gn[inside[gn]]]
        dofs = np.concatenate([f * S.Nv + nodes for f in range(dim + 1)])
        assert np.array_equal(P[v], np.sort(dofs[~fixed[dofs]]))


@pytest.mark.parametrize("dim,n,k", [(3, [3, 2, 3], 2), (2, [3, 3], 3), (3, [2, 2, 2], 1)])
def test_multiplicity_closed_form(dim, n, k):
    """Every free unknown is covered; a node with lattice index i lies in 2
    patches along each axis where i is not a multiple of k, else in 1."""
    S = _space(dim, n, k)
    fixed = ns.ns_dirichlet_mask(S)
    m = asm.multiplicity(len(fixed), asm.patches(S, fixed))
    idx = asm.node_multi_index(S)
    per_node = np.prod(np.where(idx % k != 0, 2, 1), axis=1)
    expect = np.tile(per_node, dim + 1)
    assert np.array_equal(m[~fixed], expect[~fixed])
    assert (m[fixed] == 0).all()


def test_weighted_sum_by_hand():
    """J = [[2, -1, 0], [-0.5, 2, -1], [0, -0.5, 2]], patches {0, 1}, {1, 2}:
    A1^-1 = [[2, 1], [0.5, 2]] / 3.5, A2^-1 = [[2, 1], [0.5, 2]] / 3.5,
    unknown 1 is shared (weight 1/2)."""
    J = sp.csr_matrix(np.array([[2, -1, 0], [-0.5, 2, -1], [0, -0.5, 2]], dtype=float))
    B = asm.ASM(J, [np.array([0, 1]), np.array([1, 2])])
    a = 1 / 3.5
    expect = np.array([
        [2 * a, 1 * a, 0],
        [0.5 * 0.5 * a, 0.5 * 2 * a + 0.5 * 2 * a, 0.5 * 1 * a],
        [0, 0.5 * a, 2 * a],
    ])
    assert np.allclose(B.matrix(), expect, atol=1e-15)
    r = np.array([1.0, -2.0, 0.5])
    assert np.allclose(B.apply(r), expect @ r, atol=1e-15)


def test_single_patch_is_the_exact_solve():
    rng = np.random.default_rng(3)
    A = sp.random(40, 40, density=0.2, random_state=4) + 5 * sp.identity(40)
    B = asm.ASM(A, [np.arange(40)])
    b = rng.standard_normal(40)
    x = asm.relax(A.tocsr(), B, np.zeros(40), b, 1, 1.0)
    assert np.abs(A @ x - b).max() < 1e-12


def test_q1_patches_are_point_blocks():
    """k = 1: every patch is one vertex's free unknowns (no overlap), so B
    inverts the diagonal (d+1) x (d+1) node blocks of J exactly."""
    dim, n = 3, [3, 2, 2]
    S = _space(dim, n, 1)
    u0 = inputs.uniform_vector(dim * S.Nv, 5)
    data = ns.linearization_data(S, u0, 0.05, 0.1)
    J = ns.jacobian_matrix(S, data, 0.05, 0.1)
    fixed = ns.ns_dirichlet_mask(S)
    P = asm.patches(S, fixed)
    for v, I in enumerate(P):
        nodes = np.unique(I % S.Nv)
        assert np.array_equal(nodes, [v])
    B = asm.ASM(J, P).matrix()
    BJ = B @ J.toarray()
    for I in P:
        assert np.allclose(BJ[np.ix_(I, I)], np.eye(len(I)), atol=1e-12)


def test_asm_smoother_in_the_vcycle():
    """Steady-like regime (dt = 1): two ASM sweeps need fewer FGMRES
    iterations than five Jacobi sweeps, and both reach the tolerance."""
    dim, n, k = 3, [4, 4, 4], 2
    X = inputs.structured_vertices(dim, n, noise=0.1, seed=0)
    S = Space(dim, n, X, k, k)
    u0 = inputs.fourier_field(0)(S.support_points()).T.ravel()
    its = {}
    for sm, st, om in (("jacobi", 5, 0.5), ("asm", 2, 1.0)):
        H = ns_mg.NSHierarchy(dim, n, X, k, 0.01, 1.0, u0, smoother=sm, relax_steps=st, omega=om)
        y = np.random.default_rng(0).standard_normal(H.J[0].shape[0])
        b = H.J[0] @ y
        x, its[sm], rel = ns_mg.solve(H, b, rtol=1e-8)
        assert rel <= 1e-8
    assert its["asm"] < its["jacobi"], its

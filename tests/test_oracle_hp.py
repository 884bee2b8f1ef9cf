"""Pins of the oracle's hp spaces and hp Stokes solver (Sec. 3, minimum rule):
dimension of the conforming space against the null space of the continuity
jumps, continuity across faces and edges, polynomial reproduction, the
uniform-degree case against the structured oracle, symmetry and kernels,
patch test, transfers, V-cycle and FGMRES against a direct solve."""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp

import inputs
from oracle import basis, fem, hp


def _poly(p, deg=2):
    x, y, z = p[:, 0], p[:, 1], p[:, 2]
    if deg == 1:
        return 0.3 + x - 2 * y + 0.5 * z + x * y * z
    return 1 + x * x * y - 0.5 * y * z * z + 0.25 * x * y * z + z * z * x * y


def _jumps(V: hp.HpSpace, pts_per_dir=7):
    """Rows that take the difference of the broken cell functions at points of
    every interior face (broken space = concatenated local nodal vectors)."""
    n0, n1, n2 = V.n
    offs = np.concatenate([[0], np.cumsum((V.deg + 1) ** 3)])
    rows = []
    t = np.linspace(0.05, 0.95, pts_per_dir)
    for c in range(V.deg.size):
        cc = np.array([c % n0, (c // n0) % n1, c // (n0 * n1)])
        for a in range(3):
            nb = cc.copy()
            nb[a] += 1
            if nb[a] >= V.n[a]:
                continue
            d = nb[0] + n0 * (nb[1] + n1 * nb[2])
            a1, a2 = [b for b in range(3) if b != a]
            for s_, t_ in itertools.product(t, t):
                xi = np.zeros(3)
                xi[a], xi[a1], xi[a2] = 1.0, s_, t_
                xj = xi.copy()
                xj[a] = 0.0
                r = np.zeros(offs[-1])
                r[offs[c]:offs[c + 1]] = hp._tensor_values(int(V.deg[c]), xi[None])[0]
                r[offs[d]:offs[d + 1]] -= hp._tensor_values(int(V.deg[d]), xj[None])[0]
                rows.append(r)
    return np.array(rows), offs


@pytest.mark.parametrize("n,deg", [([2, 1, 1], [2, 3]), ([2, 2, 1], [2, 3, 4, 2]), ([2, 2, 2], [2, 3, 4, 2, 3, 3, 2, 4])])
def test_dimension_and_range_equal_the_continuous_broken_functions(n, deg):
    V = hp.HpSpace(n, deg)
    Jm, offs = _jumps(V)
    dim_cont = offs[-1] - np.linalg.matrix_rank(Jm, tol=1e-9)
    assert V.N == dim_cont
    C = sp.vstack([V.cell_rows(c) for c in range(V.deg.size)]).toarray()
    assert np.linalg.matrix_rank(C, tol=1e-9) == V.N  # injective
    assert np.abs(Jm @ C).max() < 1e-12  # every image is continuous


def test_continuity_at_random_face_and_edge_points():
    n = [3, 2, 2]
    deg = [2, 5, 3, 4, 2, 6, 3, 3, 4, 2, 5, 2]
    V = hp.HpSpace(n, deg)
    x = inputs.uniform_vector(V.N, 3)
    rng = np.random.default_rng(0)
    n0, n1, _ = n
    # every interior vertex/edge/face point seen from all its cells
    for _ in range(200):
        p = rng.uniform(0, 1, 3) * np.array(n)
        k = rng.integers(1, 4)  # snap k coordinates onto grid planes
        axes = rng.choice(3, size=k, replace=False)
        for a in axes:
            p[a] = rng.integers(1, n[a]) if n[a] > 1 else 0.0
        vals = []
        for cell in itertools.product(*[[c for c in (int(np.floor(p[b])) - 1, int(np.floor(p[b])))
                                         if 0 <= c < n[b] and c <= p[b] <= c + 1] for b in range(3)]):
            c = cell[0] + n0 * (cell[1] + n1 * cell[2])
            vals.append(V.evaluate(x, c, (p - np.array(cell))[None])[0])
        assert np.ptp(vals) < 1e-13


def test_reproduces_polynomials_of_the_lowest_degree():
    n = [2, 2, 2]
    deg = [2, 3, 4, 2, 3, 3, 2, 4]
    V = hp.HpSpace(n, deg)
    P = V.reference_points()
    x = _poly(P)
    rng = np.random.default_rng(1)
    for c in range(8):
        cc = np.array([c % 2, (c // 2) % 2, c // 4])
        xi = rng.uniform(0, 1, (20, 3))
        np.testing.assert_allclose(V.evaluate(x, c, xi), _poly(cc + xi), atol=1e-12)


@pytest.mark.parametrize("k", [2, 3])
def test_uniform_degree_equals_structured_oracle(k):
    n = [3, 2, 2]
    X = inputs.structured_vertices(3, n, noise=0.2, seed=4)
    H = hp.HpStokes(n, X, np.full(12, k), 0.7)
    S = fem.Space(3, n, X, k)
    K, _ = fem.stokes_operator(S, 0.7)
    Pu = hp.structured_permutation(H.V, S)
    Pp = hp.structured_permutation(H.Pspace, fem.Space(3, n, X, k - 1, 0))  # the pressure node grid
    Pf = sp.block_diag([Pu] * 3 + [Pp], format="csr")
    Kp = (Pf @ K @ Pf.T).tocsr()
    assert abs(Kp - H.K).max() < 1e-13 * abs(K).max()


def test_symmetry_kernel_and_patch():
    n = [2, 2, 2]
    X = inputs.structured_vertices(3, n, noise=0.2, seed=6)
    deg = [2, 3, 4, 2, 3, 3, 2, 4]
    H = hp.HpStokes(n, X, deg, 1.3)
    assert abs(H.K - H.K.T).max() < 1e-13 * abs(H.K).max()
    # constant pressure: B 1 = 0 on the free velocity rows
    Bp = H.B @ np.ones(H.Np)
    assert np.abs(Bp[~H.mask[:H.nvel]]).max() < 1e-12
    # patch test: A annihilates a linear field on interior rows (trilinear cells, k >= 2)
    V = H.V
    # physical coordinates of the unknowns: Q1 map of the reference points
    R = V.reference_points()
    cid = np.minimum(np.floor(R).astype(int), np.array(n) - 1)
    xi = R - cid
    Xv = X.reshape(n[2] + 1, n[1] + 1, n[0] + 1, 3)
    phys = np.zeros_like(R)
    for corner in itertools.product((0, 1), repeat=3):
        w = np.prod([xi[:, b] if corner[b] else 1 - xi[:, b] for b in range(3)], axis=0)
        phys += w[:, None] * Xv[cid[:, 2] + corner[2], cid[:, 1] + corner[1], cid[:, 0] + corner[0]]
    u = 0.4 + phys @ np.array([1.0, -2.0, 0.5])
    assert np.abs((H.A @ u)[~V.dirichlet]).max() < 1e-11


def test_transfer_reproduces_coarse_functions():
    n = [2, 2, 2]
    deg = np.array([2, 3, 4, 2, 3, 3, 2, 4])
    Vf = hp.HpSpace(n, deg)
    Vc = hp.HpSpace(n, np.maximum(deg - 1, 2))
    P = hp.hp_transfer(Vf, Vc, constrained=False)
    xc = _poly(Vc.reference_points())
    np.testing.assert_allclose(P @ xc, _poly(Vf.reference_points()), atol=1e-12)


def test_hierarchy_vcycle_contracts_and_solver_matches_direct():
    n = [4, 4, 4]
    X = inputs.structured_vertices(3, n, noise=0.1, seed=2)
    deg = inputs.block_degrees(n, seed=5, block=2, lo=2, hi=4)
    sol = hp.HpStokesSolver(n, X, deg, 1.0)
    H = sol.mg
    for l in range(len(H.hp)):
        H.lam[l] = 1.2 * H.exact_lambda_max(l)
    for l in range(len(H.mg.spaces) - 1):
        H.mg.lam[l] = 1.2 * H.mg.exact_lambda_max(l)
    A = H.A[0]
    rng = np.random.default_rng(3)
    xt = rng.standard_normal(A.shape[0])
    xt[H.fixed[0]] = 0
    b = A @ xt
    x = np.zeros_like(b)
    e0 = np.linalg.norm(xt)
    for _ in range(5):
        x = x + H.vcycle(b - A @ x)
    assert np.linalg.norm(x - xt) < 0.3 ** 5 * e0
    s = sol.sys
    xs = rng.standard_normal(s.K.shape[0])
    xs[s.mask] = 0.0
    bs = s.K @ xs
    x, its, rel = sol.solve(bs, rtol=1e-12, maxit=100)
    assert rel <= 1e-12 and its <= 60
    p = xs[s.nvel:]
    one = np.ones(s.Np)
    xs[s.nvel:] = p - (one @ (s.M @ p)) / (one @ (s.M @ one))
    # the hp system here has condition number ~6e6 (smallest nonzero singular
    # value 2.3e-7), so a 1e-12 residual bounds the pressure error by ~1e-5
    np.testing.assert_allclose(x[:s.nvel], xs[:s.nvel], atol=1e-8 * np.abs(xs).max())
    np.testing.assert_allclose(x[s.nvel:], xs[s.nvel:], atol=1e-4 * np.abs(xs).max())


def test_block_degrees_recipe():
    d = inputs.block_degrees([8, 8, 8], seed=0)
    assert d.min() >= 2 and d.max() <= 6
    D = d.reshape(8, 8, 8)
    assert np.all(D[:4, :4, :4] == D[0, 0, 0]) and len(np.unique(d)) > 1


def test_gll_closed_forms_used_by_the_entities():
    assert np.allclose(basis.gll_points(2), [0, 0.5, 1])


def test_sampled_rows_equal_the_assembled_matrix():
    """The cell-by-cell rows used for full-size checks equal the rows of the
    assembled constrained hp Stokes matrix (every kind of row: vertex, edge,
    face and interior unknowns, Dirichlet rows, pressure rows)."""
    n = [3, 2, 3]
    deg = np.array([2, 3, 4, 2, 5, 3, 2, 2, 4, 3, 3, 2, 4, 2, 3, 5, 2, 3])
    X = inputs.structured_vertices(3, n, noise=0.15, seed=4)
    H = hp.HpStokes(n, X, deg, 0.9)
    N = H.K.shape[0]
    x = inputs.uniform_vector(N, 5)
    rows = np.unique(np.concatenate([np.random.default_rng(2).choice(N, 150, replace=False),
                                     [0, H.Nu, 3 * H.Nu - 1, 3 * H.Nu, N - 1]]))
    got = hp.sampled_stokes_rows(n, X, deg, 0.9, x, rows)
    ref = H.K @ x
    assert np.abs(got - ref[rows]).max() <= 1e-12 * np.abs(ref).max()

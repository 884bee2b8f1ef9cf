"""Pins of the oracle's Stokes operator against facts that do not come from
the oracle itself: closed-form nodes and 1D matrices, exact symbolic
integrals, symmetry, null spaces, patch tests on trilinear cells, and optimal
convergence of the discrete solution (Sec. 1 eq. (stokes), Sec. 3
eq. (stokes_block))."""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import sympy

import inputs
from oracle import basis, fem, solve


# ---------------------------------------------------------------- C1 basis
def test_gll_closed_forms():
    assert np.allclose(basis.gll_points(1), [0, 1], atol=1e-15)
    assert np.allclose(basis.gll_points(2), [0, 0.5, 1], atol=1e-15)
    r5 = 1 / math.sqrt(5)
    assert np.allclose(basis.gll_points(3), [0, (1 - r5) / 2, (1 + r5) / 2, 1], atol=1e-15)
    r37 = math.sqrt(3 / 7)
    assert np.allclose(basis.gll_points(4), [0, (1 - r37) / 2, 0.5, (1 + r37) / 2, 1], atol=1e-15)


def test_gauss_rule_exactness():
    for q in range(1, 8):
        x, w = basis.gauss_rule(q)
        for p in range(2 * q):
            assert abs(w @ x ** p - 1.0 / (p + 1)) < 1e-14
        assert abs(w @ x ** (2 * q) - 1.0 / (2 * q + 1)) > 1e-12


def test_lagrange_cardinal_and_derivative():
    for k in range(1, 7):
        nodes = basis.gll_points(k)
        assert np.allclose(basis.lagrange_values(nodes, nodes), np.eye(k + 1), atol=1e-13)
        # derivative of interpolant of x^m is m x^(m-1)
        x = np.linspace(0, 1, 11)
        for m in range(k + 1):
            D = basis.lagrange_derivatives(nodes, x)
            assert np.allclose(D @ nodes ** m, m * x ** max(m - 1, 0) * (m > 0), atol=1e-10)
            H = basis.lagrange_second_derivatives(nodes, x)
            assert np.allclose(H @ nodes ** m, m * (m - 1) * x ** max(m - 2, 0) * (m > 1), atol=1e-8)


def _one_cell(dim, X):
    return fem.Space(dim, [1] * dim, np.asarray(X, float), 2)


def test_textbook_1d_matrices_tensorized_3d():
    """Cartesian 3D Q1 and Q2 Laplacian / mass: K(x)M(x)M + ... from the 1D
    textbook matrices (x fastest => x is the rightmost Kronecker factor)."""
    h = np.array([0.5, 0.25, 2.0])
    K1 = lambda hh: np.array([[1, -1], [-1, 1]]) / hh
    M1 = lambda hh: hh / 6 * np.array([[2, 1], [1, 2]])
    K2 = lambda hh: np.array([[7, -8, 1], [-8, 16, -8], [1, -8, 7]]) / (3 * hh)
    M2 = lambda hh: hh / 30 * np.array([[4, 2, -1], [2, 16, 2], [-1, 2, 4]])
    X = inputs.structured_vertices(3, [1, 1, 1]) * h[None, :]
    for k, Kf, Mf in ((1, K1, M1), (2, K2, M2)):
        S = fem.Space(3, [1, 1, 1], X, k, 0 if k == 1 else 1)
        A = fem.stokes_element_matrices(S, 1.0)["A"][0]
        Kx, Ky, Kz = Kf(h[0]), Kf(h[1]), Kf(h[2])
        Mx, My, Mz = Mf(h[0]), Mf(h[1]), Mf(h[2])
        ref = np.kron(Mz, np.kron(My, Kx)) + np.kron(Mz, np.kron(Ky, Mx)) + np.kron(Kz, np.kron(My, Mx))
        assert np.allclose(A, ref, atol=1e-13 * abs(ref).max())


def test_q1_unit_square_pins():
    S = fem.Space(2, [1, 1], inputs.structured_vertices(2, [1, 1]), 1, 0)
    A = fem.stokes_element_matrices(S, 1.0)["A"][0]
    ref = np.array([[4, -1, -1, -2], [-1, 4, -2, -1], [-1, -2, 4, -1], [-2, -1, -1, 4]]) / 6
    assert np.allclose(A, ref, atol=1e-15)
    # Q1 mass through the Q2/Q1 pressure block
    S2 = fem.Space(2, [1, 1], inputs.structured_vertices(2, [1, 1]), 2, 1)
    M = fem.stokes_element_matrices(S2, 1.0)["M"][0]
    refm = np.array([[4, 2, 2, 1], [2, 4, 1, 2], [2, 1, 4, 2], [1, 2, 2, 4]]) / 36
    assert np.allclose(M, refm, atol=1e-15)


def _sym_lagrange(nodes, t):
    out = []
    for j, xj in enumerate(nodes):
        e = sympy.Integer(1)
        for m, xm in enumerate(nodes):
            if m != j:
                e *= (t - xm) / (xj - xm)
        out.append(sympy.expand(e))
    return out


@pytest.mark.parametrize("k", [2, 3])
def test_exact_symbolic_integrals_affine_2d(k):
    """On an affine (sheared, stretched) cell the (k+1)-point Gauss rule
    integrates every Stokes integrand exactly: compare with sympy."""
    s, t = sympy.symbols("s t")
    Am = sympy.Matrix([[sympy.Rational(3, 2), sympy.Rational(1, 3)], [sympy.Rational(-1, 5), sympy.Rational(7, 8)]])
    b = sympy.Matrix([sympy.Rational(1, 7), sympy.Rational(-2, 9)])
    gll = {2: [0, sympy.Rational(1, 2), 1], 3: [0, (1 - 1 / sympy.sqrt(5)) / 2, (1 + 1 / sympy.sqrt(5)) / 2, 1]}
    nodes_v = gll[k]
    nodes_p = gll[k - 1] if k - 1 in gll else [0, 1]
    Ls, Lt = _sym_lagrange(nodes_v, s), _sym_lagrange(nodes_v, t)
    Ps, Pt = _sym_lagrange(nodes_p, s), _sym_lagrange(nodes_p, t)
    phi = [Ls[i] * Lt[j] for j in range(k + 1) for i in range(k + 1)]
    psi = [Ps[i] * Pt[j] for j in range(k) for i in range(k)]
    invA = Am.inv()
    det = Am.det()

    def grad(f):
        g = sympy.Matrix([sympy.diff(f, s), sympy.diff(f, t)])
        return invA.T * g

    gphi = [grad(f) for f in phi]

    gx, gw = np.polynomial.legendre.leggauss(12)
    gx, gw = 0.5 * (gx + 1), 0.5 * gw
    SS, TT = np.meshgrid(gx, gx, indexing="ij")
    WW = np.outer(gw, gw)

    def integrate(expr):
        if k == 2:  # exact: sum of monomial integrals over the unit square
            poly = sympy.Poly(sympy.expand(expr), s, t)
            return sum(cf / ((a + 1) * (b_ + 1)) for (a, b_), cf in poly.terms())
        # k = 3 (irrational nodes): a 12-point rule is exact for these degrees
        fn = sympy.lambdify((s, t), expr, "numpy")
        return float((WW * fn(SS, TT)).sum())

    nv, npr = len(phi), len(psi)
    A_ex = np.zeros((nv, nv))
    for i in range(nv):
        for j in range(i, nv):
            v = integrate((gphi[i].T * gphi[j])[0] * det)
            A_ex[i, j] = A_ex[j, i] = float(v)
    B_ex = np.zeros((2 * nv, npr))
    for c in range(2):
        for i in range(nv):
            for j in range(npr):
                B_ex[c * nv + i, j] = -float(integrate(psi[j] * gphi[i][c] * det))
    # the cell: vertices = affine image of the unit square
    ref = np.array([[0, 0], [1, 0], [0, 1], [1, 1]], float)
    A_np = np.array(Am.evalf(), dtype=float)
    X = ref @ A_np.T + np.array(b.evalf(), dtype=float).ravel()[None, :]
    S = fem.Space(2, [1, 1], X, k)
    em = fem.stokes_element_matrices(S, 1.0)
    assert np.allclose(em["A"][0], A_ex, atol=1e-13)
    assert np.allclose(em["B"][0], B_ex, atol=1e-13)


# ---------------------------------------------------------------- C4/C5
@pytest.mark.parametrize("dim,n,k", [(2, [3, 4], 2), (2, [2, 2], 3), (3, [2, 3, 2], 2), (3, [2, 2, 2], 3)])
def test_element_loop_equals_csr_and_symmetry(dim, n, k):
    X = inputs.structured_vertices(dim, n, noise=0.2, seed=3)
    S = fem.Space(dim, n, X, k)
    K, mats = fem.stokes_operator(S, 0.7)
    x = inputs.uniform_vector(S.n_dofs, 1)
    y1 = K @ x
    y2 = fem.element_loop_stokes_vmult(S, 0.7, x)
    assert np.abs(y1 - y2).max() <= 1e-14 * np.abs(y1).max()
    assert abs(K - K.T).max() <= 1e-14 * abs(K).max()
    assert abs(mats["K"] - mats["K"].T).max() <= 1e-14 * abs(mats["K"]).max()


@pytest.mark.parametrize("dim,n,k", [(2, [3, 3], 2), (3, [2, 2, 3], 2), (3, [2, 2, 2], 4)])
def test_null_spaces(dim, n, k):
    X = inputs.structured_vertices(dim, n, noise=0.2, seed=5)
    S = fem.Space(dim, n, X, k)
    K, mats = fem.stokes_operator(S, 1.3)
    # rigid translations are in the kernel of the unconstrained Laplacian
    one = np.ones(S.Nv)
    assert np.abs(mats["A"] @ one).max() < 1e-12
    # the constrained operator annihilates (0, 1_p)
    z = np.zeros(S.n_dofs)
    z[dim * S.Nv:] = 1.0
    assert np.abs(K @ z).max() < 1e-12


# ---------------------------------------------------------------- C6 patch tests
@pytest.mark.parametrize("dim,n,k", [(2, [3, 3], 2), (3, [3, 3, 3], 2), (3, [2, 2, 2], 3)])
def test_patch_tests_trilinear(dim, n, k):
    X = inputs.structured_vertices(dim, n, noise=0.2, seed=11)
    S = fem.Space(dim, n, X, k)
    mats = fem.assemble_stokes(S, 1.0)
    xs = S.support_points()
    rng = np.random.default_rng(0)
    G = rng.standard_normal((dim, dim))
    c0 = rng.standard_normal(dim)
    ulin = xs @ G.T + c0  # u_c(x) = sum_b G[c,b] x_b + c0
    uvec = ulin.T.ravel()
    interior = ~S.dirichlet
    # (i) A I(u_lin) = 0 on interior rows
    for c in range(dim):
        r = mats["A"] @ ulin[:, c]
        assert np.abs(r[interior]).max() < 1e-12
    # (ii) B^T I(u_lin) = -tr(G) M_p 1
    BtU = mats["B"].T @ uvec
    assert np.allclose(BtU, -np.trace(G) * (mats["M"] @ np.ones(S.Np)), atol=1e-12)
    # (iii) B I(p_lin) = dp/dx_c * int(phi_i) on interior rows
    xp = S.support_points(S.kp)
    g = rng.standard_normal(dim)
    plin = xp @ g + 0.3
    Bp = mats["B"] @ plin
    # int(phi_i): the velocity mass times one via the A-block quadrature
    _, _, _, _, JxW = S.geometry()
    N = basis.tensor_basis(dim, k, basis.gauss_rule(k + 1)[0])[0]
    intphi = np.zeros(S.Nv)
    np.add.at(intphi, S.vdofs.ravel(), (JxW @ N).ravel())
    for c in range(dim):
        rows = Bp[c * S.Nv:(c + 1) * S.Nv]
        assert np.abs(rows[interior] - g[c] * intphi[interior]).max() < 1e-12


# ---------------------------------------------------------------- C13 rates
def _solve_ms(dim, n, k, X, nu=1.0):
    S = fem.Space(dim, [n] * dim, X, k)
    xq = S.geometry()[0]
    ms = inputs.manufactured_2d if dim == 2 else inputs.manufactured_3d
    _, _, f = ms(xq, nu)
    uD = ms(S.support_points(), nu)[0]
    mats = fem.assemble_stokes(S, nu)
    b = solve.stokes_rhs(S, nu, f, uD, mats)
    x = solve.direct_solve(S, nu, b, mats)
    x = solve.pressure_mean_free(S, x, mats["M"])
    xe, JxW, u, gu, p = solve.evaluate(S, x, k + 3)
    ue, pe, _ = ms(xe, nu)
    # exact gradient by central differences of the closed form
    eps = 1e-6
    gue = np.zeros(gu.shape)
    for a in range(dim):
        d = np.zeros(dim)
        d[a] = eps
        gue[..., a] = (ms(xe + d, nu)[0] - ms(xe - d, nu)[0]) / (2 * eps)
    pm = (JxW * p).sum() / JxW.sum()
    eu = math.sqrt((JxW[..., None] * (u - ue) ** 2).sum())
    eg = math.sqrt((JxW[..., None, None] * (gu - gue) ** 2).sum())
    ep = math.sqrt((JxW * (p - pm - pe) ** 2).sum())
    return eu, eg, ep


@pytest.mark.parametrize("k,mapped", [(2, False), (2, True), (3, False)])
def test_optimal_rates_2d(k, mapped):
    errs = []
    for n in (4, 8, 16):
        X = inputs.smooth_mapped_vertices(2, [n, n]) if mapped else inputs.structured_vertices(2, [n, n])
        errs.append(_solve_ms(2, n, k, X))
    errs = np.array(errs)
    rates = np.log2(errs[:-1] / errs[1:])[-1]
    assert rates[0] > k + 1 - 0.25, rates
    assert rates[1] > k - 0.25, rates
    assert rates[2] > k - 0.25, rates


def test_rates_3d_q2q1():
    errs = np.array([_solve_ms(3, n, 2, inputs.structured_vertices(3, [n] * 3)) for n in (2, 4, 8)])
    rates = np.log2(errs[:-1] / errs[1:])[-1]
    assert rates[0] > 2.6 and rates[1] > 1.7 and rates[2] > 1.7, rates


def test_manufactured_fields_closed_form():
    """The manufactured forcing is -nu Lap u + grad p and u is divergence
    free (sympy)."""
    x, y, z = sympy.symbols("x y z")
    nu = sympy.Rational(3, 7)
    psi = sympy.sin(sympy.pi * x) ** 2 * sympy.sin(sympy.pi * y) ** 2 * sympy.sin(sympy.pi * z) ** 2
    u = [sympy.diff(psi, y) - sympy.diff(psi, z), sympy.diff(psi, z) - sympy.diff(psi, x), sympy.diff(psi, x) - sympy.diff(psi, y)]
    p = sympy.cos(sympy.pi * x) * sympy.cos(sympy.pi * y) * sympy.cos(sympy.pi * z)
    f = [-nu * sum(sympy.diff(u[c], v, 2) for v in (x, y, z)) + sympy.diff(p, v) for c, v in enumerate((x, y, z))]
    pts = np.random.default_rng(1).uniform(0, 1, (5, 3))
    uu, pp, ff = inputs.manufactured_3d(pts, float(nu))
    for i, (a, b_, c) in enumerate(pts):
        sub = {x: a, y: b_, z: c}
        assert abs(float(sum(sympy.diff(u[cc], v) for cc, v in enumerate((x, y, z))).subs(sub))) < 1e-12
        for cc in range(3):
            assert abs(float(u[cc].subs(sub)) - uu[i, cc]) < 1e-12
            assert abs(float(f[cc].subs(sub)) - ff[i, cc]) < 1e-10
        assert abs(float(p.subs(sub)) - pp[i]) < 1e-12
    # 2D
    psi2 = sympy.sin(sympy.pi * x) ** 2 * sympy.sin(sympy.pi * y) ** 2
    u2 = [sympy.diff(psi2, y), -sympy.diff(psi2, x)]
    p2 = sympy.cos(sympy.pi * x) * sympy.cos(sympy.pi * y)
    f2 = [-nu * sum(sympy.diff(u2[c], v, 2) for v in (x, y)) + sympy.diff(p2, v) for c, v in enumerate((x, y))]
    uu, pp, ff = inputs.manufactured_2d(pts[:, :2], float(nu))
    for i, (a, b_, _) in enumerate(pts):
        sub = {x: a, y: b_}
        for cc in range(2):
            assert abs(float(u2[cc].subs(sub)) - uu[i, cc]) < 1e-12
            assert abs(float(f2[cc].subs(sub)) - ff[i, cc]) < 1e-10

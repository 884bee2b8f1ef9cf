"""Pins of oracle parts that the other oracle tests only check against
each other:

* the fixed-step Jacobi-PCG of the Schur approximation (Sec. 3
  eq. (stokes_block)) against a direct solve, the finite termination of CG
  and the Galerkin characterisation of its iterates;
* the stabilised Navier-Stokes residual and its Newton and Oseen Jacobians
  (Sec. 5, F_NS + F_SUPG + F_PSPG of eq. (ns) with BDF2) against element
  vectors of the weak form integrated exactly by sympy on one affine cell,
  with the Jacobian taken as the symbolic Gateaux derivative;
* the skew-symmetry of the convection form for a divergence-free advecting
  field;
* the physical Laplacian of Q2 basis functions on affine cells;
* the SUPG/PSPG parameter delta_1 at hand-computed points.
"""
import numpy as np
import pytest
import scipy.linalg as la
import sympy

import inputs
from oracle import fem, krylov, ns


# ------------------------------------------------------------ Schur PCG
def _spd(n, seed, eigs=None):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = rng.uniform(1.0, 50.0, n) if eigs is None else np.asarray(eigs, float)
    return (Q * lam) @ Q.T


def test_pcg_fixed_n_steps_is_a_direct_solve():
    n = 12
    M = _spd(n, 0)
    dinv = 1.0 / np.random.default_rng(1).uniform(0.5, 2.0, n)
    r = np.random.default_rng(2).standard_normal(n)
    z = krylov.pcg_fixed(M, dinv, r, n + 2)
    assert np.linalg.norm(z - la.solve(M, r)) <= 1e-9 * np.linalg.norm(la.solve(M, r))


@pytest.mark.parametrize("m", [1, 2, 3, 5])
def test_pcg_fixed_terminates_after_distinct_eigenvalues(m):
    """If the preconditioned operator C^(1/2) M C^(1/2) (C = diag(dinv)) has m
    distinct eigenvalues, CG is exact after m steps."""
    n = 16
    rng = np.random.default_rng(10 + m)
    levels = np.linspace(1.0, 9.0, m) if m > 1 else np.array([4.0])
    B = _spd(n, 20 + m, eigs=levels[rng.integers(0, m, n)])
    c = rng.uniform(0.5, 3.0, n)  # C = diag(c)
    M = B / np.sqrt(c)[:, None] / np.sqrt(c)[None, :]  # C^(1/2) M C^(1/2) = B
    r = rng.standard_normal(n)
    z = krylov.pcg_fixed(M, c, r, m)
    zex = la.solve(M, r)
    assert np.linalg.norm(z - zex) <= 1e-9 * np.linalg.norm(zex)
    if m > 1:  # and not exact one step earlier
        z1 = krylov.pcg_fixed(M, c, r, m - 1)
        assert np.linalg.norm(z1 - zex) > 1e-6 * np.linalg.norm(zex)


@pytest.mark.parametrize("steps", [1, 2, 3, 4])
def test_pcg_fixed_iterates_are_galerkin_projections(steps):
    """After j steps from z = 0, preconditioned CG returns the M-orthogonal
    projection of M^-1 r onto the Krylov space span{(C M)^i C r, i < j}."""
    n = 20
    M = _spd(n, 5)
    rng = np.random.default_rng(6)
    c = rng.uniform(0.5, 2.0, n)
    r = rng.standard_normal(n)
    K = [c * r]
    for _ in range(steps - 1):
        K.append(c * (M @ K[-1]))
    Q, _ = np.linalg.qr(np.array(K).T)
    zg = Q @ la.solve(Q.T @ M @ Q, Q.T @ r)
    z = krylov.pcg_fixed(M, c, r, steps)
    assert np.linalg.norm(z - zg) <= 1e-10 * np.linalg.norm(zg)


# ------------------------------------------- stabilised Navier-Stokes, exact
def _sym_lagrange(nodes, s):
    out = []
    for j, xj in enumerate(nodes):
        e = sympy.Integer(1)
        for m, xm in enumerate(nodes):
            if m != j:
                e *= (s - xm) / (xj - xm)
        out.append(sympy.expand(e))
    return out


def _affine(dim):
    R = sympy.Rational
    if dim == 2:
        A = sympy.Matrix([[R(3, 2), R(1, 3)], [R(-1, 5), R(7, 8)]])
        b = sympy.Matrix([R(1, 7), R(-2, 9)])
    else:
        A = sympy.Matrix([[R(6, 5), R(1, 4), R(-1, 6)], [R(1, 7), R(9, 10), R(1, 5)], [R(-1, 8), R(1, 9), R(11, 10)]])
        b = sympy.Matrix([R(1, 3), R(-1, 4), R(2, 5)])
    assert A.det() > 0
    return A, b


def _poly(X, deg, rng):
    """Random polynomial of total degree `deg` in the physical coordinates."""
    import itertools

    e = sympy.Integer(0)
    for pw in itertools.product(range(deg + 1), repeat=len(X)):
        if sum(pw) <= deg:
            term = sympy.Rational(int(rng.integers(-9, 10)), int(rng.integers(1, 8)))
            for xa, pa in zip(X, pw):
                term *= xa ** pa
            e += term
    return e


class _Cell:
    """One affine cell x = b + A xi of [0,1]^dim with the Q2 Lagrange basis on
    the GLL nodes (0, 1/2, 1), built symbolically and independently of the
    oracle.  Integration by a tensor Gauss rule of `gauss` points per
    direction: 8 is exact to degree 15 per variable; 3 is the rule the
    method uses for Q2 (k + 1 points), for integrands it does not integrate
    exactly."""

    def __init__(self, dim, gauss=8):
        self.dim = dim
        self.A, self.b = _affine(dim)
        self.xi = sympy.symbols("s t r")[:dim]
        self.X = sympy.symbols("x y z")[:dim]
        nodes = [0, sympy.Rational(1, 2), 1]
        Ls = [_sym_lagrange(nodes, v) for v in self.xi]
        import itertools

        self.phi = []
        for idx in itertools.product(range(3), repeat=dim):
            idx = idx[::-1]  # x fastest
            f = sympy.Integer(1)
            for a in range(dim):
                f *= Ls[a][idx[a]]
            self.phi.append(f)
        g, w = np.polynomial.legendre.leggauss(gauss)
        g, w = 0.5 * (g + 1), 0.5 * w
        grids = np.meshgrid(*([g] * dim), indexing="ij")
        self.pts = [G.ravel() for G in grids]
        W = w
        for _ in range(dim - 1):
            W = np.multiply.outer(W, w)
        self.W = W.ravel() * float(self.A.det())
        Ainv_T = np.array(self.A.inv().T.evalf(), dtype=float)
        self.val = np.array([self._ev(f) for f in self.phi])  # [i, q]
        gref = np.array([[self._ev(sympy.diff(f, v)) for v in self.xi] for f in self.phi])  # [i, b, q]
        self.grad = np.einsum("ab,ibq->iaq", Ainv_T, gref)  # physical gradients [i, a, q]
        nodes_f = np.array([0.0, 0.5, 1.0])
        mi = np.stack(np.meshgrid(*([np.arange(3)] * dim), indexing="ij"), 0).reshape(dim, -1, order="F").T
        ref_nodes = nodes_f[mi]  # [node, dim] lexicographic, x fastest
        self.support = ref_nodes @ np.array(self.A.evalf(), dtype=float).T + np.array(self.b.evalf(), dtype=float).ravel()
        ref_v = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0], [0, 0, 1], [1, 0, 1], [0, 1, 1], [1, 1, 1]], float)
        ref_v = ref_v[: 2 ** dim, :dim]
        self.vertices = ref_v @ np.array(self.A.evalf(), dtype=float).T + np.array(self.b.evalf(), dtype=float).ravel()
        self.to_ref = {self.X[a]: (self.b[a] + sum(self.A[a, c] * self.xi[c] for c in range(dim))) for a in range(dim)}

    def _ev(self, expr):
        fn = sympy.lambdify(self.xi, expr, "numpy")
        v = fn(*self.pts)
        return np.broadcast_to(np.asarray(v, dtype=float), self.pts[0].shape)

    def nodal(self, f):
        fn = sympy.lambdify(self.X, f, "numpy")
        return np.broadcast_to(np.asarray(fn(*self.support.T), dtype=float), (len(self.support),)).copy()

    def element_vector(self, integrand, V, GV, Q, GQ):
        """Test the integrand (linear in the placeholders V_c, GV_ca, Q, GQ_a)
        with every basis function; returns the blocked [v_0 | .. | q] vector."""
        d = self.dim
        nb = len(self.phi)
        out = np.zeros((d + 1) * nb)
        e = sympy.expand(integrand)

        def coef(sym):
            return self._ev(sympy.diff(e, sym).subs(self.to_ref))

        for c in range(d):
            cv = coef(V[c])
            out[c * nb:(c + 1) * nb] += self.val @ (self.W * cv)
            for a in range(d):
                out[c * nb:(c + 1) * nb] += self.grad[:, a, :] @ (self.W * coef(GV[c][a]))
        out[d * nb:] += self.val @ (self.W * coef(Q))
        for a in range(d):
            out[d * nb:] += self.grad[:, a, :] @ (self.W * coef(GQ[a]))
        return out


def _weak_form(X, u, p, u_n, u_nm1, adv, dl, nu, dt):
    """Integrand of F_NS + F_SUPG + F_PSPG (Sec. 5) at one point, tested with
    placeholder values of v, grad v, q, grad q.  Time derivative: BDF2,
    (3 u - 4 u^n + u^{n-1}) / (2 dt).  `adv` is the advecting velocity of
    the convective and streamline terms (u itself for Navier-Stokes)."""
    d = len(X)
    V = sympy.symbols(f"V0:{d}")
    GV = [list(sympy.symbols(f"G{c}_0:{d}")) for c in range(d)]
    Q = sympy.Symbol("Q")
    GQ = sympy.symbols(f"GQ0:{d}")
    grad = lambda f: [sympy.diff(f, xa) for xa in X]  # noqa: E731
    gu = [grad(u[c]) for c in range(d)]  # gu[c][a] = d u_c / d x_a
    lap = [sum(sympy.diff(u[c], xa, 2) for xa in X) for c in range(d)]
    gp = grad(p)
    dudt = [(3 * u[c] - 4 * u_n[c] + u_nm1[c]) / (2 * dt) for c in range(d)]
    conv = [sum(adv[a] * gu[c][a] for a in range(d)) for c in range(d)]
    Rs = [dudt[c] + conv[c] + gp[c] - nu * lap[c] for c in range(d)]
    div_u = sum(gu[a][a] for a in range(d))
    div_v = sum(GV[a][a] for a in range(d))
    I = sum((dudt[c] + conv[c]) * V[c] for c in range(d))
    I += nu * sum(gu[c][a] * GV[c][a] for c in range(d) for a in range(d))
    I += -p * div_v + div_u * Q
    I += dl * sum(Rs[c] * sum(adv[a] * GV[c][a] for a in range(d)) for c in range(d))  # SUPG
    I += dl * sum(Rs[a] * GQ[a] for a in range(d))  # PSPG
    return I, (V, GV, Q, GQ)


_CELLS = {}


def _cell(dim, gauss=8):
    if (dim, gauss) not in _CELLS:
        _CELLS[dim, gauss] = _Cell(dim, gauss)
    return _CELLS[dim, gauss]


def _oracle_space(cell):
    return fem.Space(cell.dim, [1] * cell.dim, cell.vertices, 2, kp=2)


@pytest.mark.parametrize("dim", [2, 3])
def test_ns_residual_equals_exact_weak_form(dim):
    """u in P1, p in P2, BDF2 history u^n = u^{n-1} in P2, delta_1 constant:
    the (k+1)-point Gauss rule is exact for every term, so the oracle's
    element vector equals the exact integral of the weak form."""
    C = _cell(dim)
    rng = np.random.default_rng(100 + dim)
    nu, dt, dl = 0.37, 0.2, 0.083
    u = [_poly(C.X, 1, rng) for _ in range(dim)]
    p = _poly(C.X, 2, rng)
    uh = [_poly(C.X, 2, rng) for _ in range(dim)]
    I, ph = _weak_form(C.X, u, p, uh, uh, u, sympy.Rational(83, 1000), sympy.Rational(37, 100), sympy.Rational(1, 5))
    ref = C.element_vector(I, *ph)
    S = _oracle_space(C)
    uh_nodal = np.concatenate([C.nodal(f) for f in uh])
    x = np.concatenate([C.nodal(f) for f in u] + [C.nodal(p)])
    data = ns.linearization_data(S, uh_nodal, nu, dt)
    data["delta"] = np.full_like(data["delta"], dl)
    got = ns.residual(S, x, uh_nodal, nu, dt, data)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max(), np.abs(got - ref).max()


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("newton", [True, False])
def test_ns_jacobian_equals_gateaux_derivative(dim, newton):
    """Linearisation point u0 in P1, p0 = 0, history u0; direction (w, P) with
    w in P2 (so the trial Laplacian is a nonzero constant) and P in P2;
    delta_1 constant.  Newton: the symbolic derivative of the weak form.
    Oseen: the derivative with the advecting velocity frozen at u0 (drops
    w . grad u0 and (R(u0), w . grad v))."""
    C = _cell(dim)
    rng = np.random.default_rng(200 + dim)
    nu, dt, dl = 0.29, 0.125, 0.061
    eps = sympy.Symbol("eps")
    u0 = [_poly(C.X, 1, rng) for _ in range(dim)]
    w = [_poly(C.X, 2, rng) for _ in range(dim)]
    P = _poly(C.X, 2, rng)
    u = [u0[c] + eps * w[c] for c in range(dim)]
    adv = u if newton else u0
    I, ph = _weak_form(C.X, u, eps * P, u0, u0, adv, sympy.Rational(61, 1000), sympy.Rational(29, 100),
                       sympy.Rational(1, 8))
    dI = sympy.diff(I, eps).subs(eps, 0)
    ref = C.element_vector(dI, *ph)
    S = _oracle_space(C)
    u0_nodal = np.concatenate([C.nodal(f) for f in u0])
    dx = np.concatenate([C.nodal(f) for f in w] + [C.nodal(P)])
    data = ns.linearization_data(S, u0_nodal, nu, dt)
    data["delta"] = np.full_like(data["delta"], dl)
    got = ns.jacobian_apply(S, dx, data, nu, dt, newton)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max(), np.abs(got - ref).max()


@pytest.mark.parametrize("dim", [2, 3])
def test_ns_residual_and_jacobian_at_gauss_points_quadratic_fields(dim):
    """Quadratic u, u0 and history (nonzero Laplacians in R(u) and R(u0)):
    the convective and streamline terms are then beyond the rule's exactness,
    so the symbolic weak form is integrated with the same 3-point Gauss rule
    the method prescribes for Q2 (a reading: (k+1)-point Gauss)."""
    C = _cell(dim, gauss=3)
    rng = np.random.default_rng(400 + dim)
    nu, dt, dl = 0.53, 0.3, 0.071
    R_ = sympy.Rational
    S = _oracle_space(C)
    u = [_poly(C.X, 2, rng) for _ in range(dim)]
    p = _poly(C.X, 2, rng)
    uh = [_poly(C.X, 2, rng) for _ in range(dim)]
    I, ph = _weak_form(C.X, u, p, uh, uh, u, R_(71, 1000), R_(53, 100), R_(3, 10))
    ref = C.element_vector(I, *ph)
    uh_nodal = np.concatenate([C.nodal(f) for f in uh])
    data = ns.linearization_data(S, uh_nodal, nu, dt)
    data["delta"] = np.full_like(data["delta"], dl)
    x = np.concatenate([C.nodal(f) for f in u] + [C.nodal(p)])
    got = ns.residual(S, x, uh_nodal, nu, dt, data)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max(), np.abs(got - ref).max()
    # Newton Jacobian about a quadratic u0 (R(u0) carries -nu Lap u0)
    eps = sympy.Symbol("eps")
    u0 = uh
    w = [_poly(C.X, 2, rng) for _ in range(dim)]
    P = _poly(C.X, 2, rng)
    uu = [u0[c] + eps * w[c] for c in range(dim)]
    I, ph = _weak_form(C.X, uu, eps * P, u0, u0, uu, R_(71, 1000), R_(53, 100), R_(3, 10))
    ref = C.element_vector(sympy.diff(I, eps).subs(eps, 0), *ph)
    dx = np.concatenate([C.nodal(f) for f in w] + [C.nodal(P)])
    got = ns.jacobian_apply(S, dx, data, nu, dt, True)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max(), np.abs(got - ref).max()


def test_ns_jacobian_pressure_rows_against_velocity_trial():
    """The K_pu block alone: pressure rows of J applied to a velocity-only
    direction, compared with the exact (div w, q) + delta (R_lin(w), grad q)
    on a 3D affine cell."""
    C = _cell(3)
    rng = np.random.default_rng(300)
    nu, dt, dl = 0.41, 0.25, 0.05
    eps = sympy.Symbol("eps")
    u0 = [_poly(C.X, 1, rng) for _ in range(3)]
    w = [_poly(C.X, 2, rng) for _ in range(3)]
    u = [u0[c] + eps * w[c] for c in range(3)]
    I, ph = _weak_form(C.X, u, sympy.Integer(0), u0, u0, u, sympy.Rational(1, 20), sympy.Rational(41, 100),
                       sympy.Rational(1, 4))
    ref = C.element_vector(sympy.diff(I, eps).subs(eps, 0), *ph)
    S = _oracle_space(C)
    data = ns.linearization_data(S, np.concatenate([C.nodal(f) for f in u0]), nu, dt)
    data["delta"] = np.full_like(data["delta"], dl)
    dx = np.concatenate([C.nodal(f) for f in w] + [np.zeros(27)])
    got = ns.jacobian_apply(S, dx, data, nu, dt, True)
    assert np.abs(got[81:] - ref[81:]).max() <= 1e-12 * np.abs(ref[81:]).max()
    assert np.abs(ref[81:]).max() > 1e-3


@pytest.mark.parametrize("dim", [2, 3])
def test_convection_is_skew_symmetric_for_divergence_free_advection(dim):
    """(u0 . grad w2, w1) = -(u0 . grad w1, w2) when div u0 = 0 and w1, w2
    vanish on the boundary.  u0 linear with a traceless gradient; affine
    (uniformly sheared) cells so that the Gauss rule is exact."""
    n = [3] * dim
    A = np.array([[1.0, 0.3, 0.1], [-0.2, 0.9, 0.25], [0.15, -0.1, 1.1]])[:dim, :dim]
    X = inputs.structured_vertices(dim, n) @ A.T
    S = fem.Space(dim, n, X, 2, kp=2)
    xs = S.support_points()
    Gm = np.array([[0.7, -1.2, 0.4], [0.9, 0.5, -0.8], [0.3, 1.1, -1.2]])[:dim, :dim]
    Gm[-1, -1] = -np.trace(Gm[:-1, :-1])  # traceless: div u0 = 0
    u0 = np.concatenate([(xs @ Gm.T + 0.3)[:, c] for c in range(dim)])
    data = ns.linearization_data(S, u0, 0.0, np.inf)
    data["delta"] = np.zeros_like(data["delta"])
    rng = np.random.default_rng(4)
    nv = dim * S.Nv
    mask = ns.ns_dirichlet_mask(S)
    w1, w2 = (np.where(mask, 0.0, rng.uniform(-1, 1, nv + S.Nv)) for _ in range(2))
    w1[nv:] = 0.0
    w2[nv:] = 0.0
    c12 = w1[:nv] @ ns.jacobian_apply(S, w2, data, 0.0, np.inf, newton=False)[:nv]
    c21 = w2[:nv] @ ns.jacobian_apply(S, w1, data, 0.0, np.inf, newton=False)[:nv]
    assert abs(c12) > 1e-3
    assert abs(c12 + c21) <= 1e-12 * abs(c12)


def test_q2_laplacian_of_interpolated_quadratic_on_affine_cells():
    """Sum_i u_i Lap(phi_i) equals the constant Laplacian of a quadratic u at
    every Gauss point of sheared, stretched (affine) cells."""
    dim, n = 3, [2, 2, 2]
    A = np.array([[1.3, 0.4, -0.2], [0.1, 0.8, 0.3], [-0.25, 0.2, 1.5]])
    X = inputs.structured_vertices(dim, n) @ A.T
    S = fem.Space(dim, n, X, 2, kp=2)
    x, y, z = S.support_points().T
    u = 2.0 * x * x - 3.0 * y * y + 0.5 * z * z + 1.5 * x * y - 0.7 * y * z + x - 2.0
    lap = 2 * 2.0 - 3 * 2.0 + 2 * 0.5
    N, G, L, JxW, vol = ns._qp_data(S)
    vals = np.einsum("eqi,ei->eq", L, u[S.vdofs])
    assert np.abs(vals - lap).max() < 1e-11
    # and the gradient of the same interpolant is exact
    gx = np.einsum("eqi,ei->eq", G[..., 0], u[S.vdofs])
    xq = S.geometry()[0]
    assert np.abs(gx - (4.0 * xq[..., 0] + 1.5 * xq[..., 1] + 1.0)).max() < 1e-11


@pytest.mark.parametrize("h,k,dt,nu,expected", [
    # (2/0.5)^2 + (2*5/1)^2 + 9*(4*0.25/1)^2 = 16 + 100 + 9 = 125
    (1.0, 1, 0.5, 0.25, 125.0 ** -0.5),
    # h_K = 0.5/2 = 0.25: 20^2 + 40^2 + 9*(0.04/0.0625)^2 = 400 + 1600 + 3.6864
    (0.5, 2, 0.1, 0.01, 2003.6864 ** -0.5),
])
def test_delta1_hand_computed(h, k, dt, nu, expected):
    """delta_1 for a constant velocity (3, 4, 0) (|u0| = 5) on one cube of
    side h (|K|^(1/3) = h)."""
    X = inputs.structured_vertices(3, [1, 1, 1]) * h
    S = fem.Space(3, [1, 1, 1], X, k, kp=k)
    u0 = np.concatenate([np.full(S.Nv, 3.0), np.full(S.Nv, 4.0), np.zeros(S.Nv)])
    data = ns.linearization_data(S, u0, nu, dt)
    assert np.abs(data["delta"] - expected).max() <= 1e-14 * expected

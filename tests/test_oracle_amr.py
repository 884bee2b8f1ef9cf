"""Pins of the locally refined (hanging-node) oracle.

* The generated meshes cover the cube once and are 2:1 balanced over faces
  and edges (the closure the constraints rely on).
* A mesh refined everywhere is the structured mesh of twice the resolution:
  same unknowns in the same order, no hanging nodes, and the same
  Navier-Stokes Jacobian as the structured oracle.
* The constraints reproduce every Q_k polynomial exactly (the coarse
  interpolant of a Q_k polynomial is the polynomial itself).
* Nested spaces: the conforming space on the refined mesh is a subspace of
  the Q_k space on the uniform mesh of the finest level, so its mass and
  stiffness matrices equal E^T M E and E^T K E, with E the point evaluation of
  the refined space at the fine nodes (exact quadrature on Cartesian cells).
  A wrong constraint weight breaks this identity (checked by planting one).
* The constrained Jacobian: element loop = assembled matrix, the constant
  pressure is in its kernel.
* Multigrid: global coarsening reaches the uniform base mesh one level at a
  time; on a mesh refined everywhere the hierarchy and its V-cycle are the
  structured ones; the transfers interpolate Q_k polynomials exactly and
  vanish on Dirichlet rows; FGMRES with the V-cycle converges.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import inputs
from oracle import amr, fem, ns

MESH = dict(n=3, seed=0, levels=2, centre=[0.4, 0.5, 0.55], radius=0.3)


def _level_map(m):
    L, n = m["levels"], m["n"]
    F = n << L
    lev = np.full((F, F, F), -1, dtype=np.int64)
    count = np.zeros((F, F, F), dtype=np.int64)
    for l, (i, j, k) in zip(m["level"], m["idx"]):
        s = 1 << (L - l)
        lev[k * s:(k + 1) * s, j * s:(j + 1) * s, i * s:(i + 1) * s] = l
        count[k * s:(k + 1) * s, j * s:(j + 1) * s, i * s:(i + 1) * s] += 1
    return lev, count


@pytest.mark.parametrize("levels,radius", [(1, 0.3), (2, 0.3), (2, 0.22)])
def test_refined_mesh_covers_cube_and_is_balanced(levels, radius):
    m = inputs.refined_mesh(4, 0, levels=levels, centre=[0.45, 0.5, 0.6], radius=radius)
    lev, count = _level_map(m)
    assert (count == 1).all()
    vol = (1.0 / (m["n"] * 2.0 ** m["level"])) ** 3
    assert abs(vol.sum() - 1.0) < 1e-13
    F = lev.shape[0]
    for dz, dy, dx in [(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)
                       if 1 <= abs(a) + abs(b) + abs(c) <= 2]:
        A = lev[max(0, -dz):F - max(0, dz), max(0, -dy):F - max(0, dy), max(0, -dx):F - max(0, dx)]
        B = lev[max(0, dz):F - max(0, -dz), max(0, dy):F - max(0, -dy), max(0, dx):F - max(0, -dx)]
        assert np.abs(A - B).max() <= 1
    assert m["level"].max() == levels


@pytest.mark.parametrize("k", [1, 2])
def test_refinement_everywhere_is_the_structured_mesh(k):
    m = inputs.refined_mesh(2, 0, levels=1, centre=[0.5] * 3, radius=10.0)
    S = amr.AmrSpace(m, k)
    St = fem.Space(3, [4, 4, 4], inputs.structured_vertices(3, [4, 4, 4]), k, k)
    assert S.N == St.Nv and not S.hanging.any()
    assert np.abs(S.true_points() - St.support_points(k)).max() < 1e-15
    F = inputs.fourier_field(3)
    u0 = F(S.true_points()).T.ravel()
    nu, dt = 0.01, 0.02
    J = amr.jacobian_matrix(S, u0, nu, dt, True)
    Jt = ns.jacobian_matrix(St, ns.linearization_data(St, u0, nu, dt), nu, dt, True)
    assert abs(J - Jt).max() <= 1e-12 * abs(Jt).max()


@pytest.mark.parametrize("k", [1, 2])
def test_constraints_reproduce_polynomials(k):
    S = amr.AmrSpace(inputs.refined_mesh(**MESH), k)
    assert S.hanging.sum() > 50
    f = lambda p: (1 + p[:, 0] + p[:, 0] ** k * p[:, 1] ** k) * (2 - p[:, 2] ** k) + p[:, 1] ** k * p[:, 2]  # noqa
    assert np.abs(S.C @ f(S.true_points()) - f(S.raw_pos / S.R)).max() < 1e-13


def _nested_defect(S, k):
    nf = S.n[0] << S.L
    Sf = fem.Space(3, [nf] * 3, inputs.structured_vertices(3, [nf] * 3), k, k)
    Mf, Kf = amr.scalar_matrices(Sf)
    Mr, Kr = amr.scalar_matrices(S)
    E = S.evaluation_matrix(Sf.support_points(k))
    Ma, Ka = S.C.T @ Mr @ S.C, S.C.T @ Kr @ S.C
    return max(abs(E.T @ Mf @ E - Ma).max() / abs(Ma).max(), abs(E.T @ Kf @ E - Ka).max() / abs(Ka).max())


@pytest.mark.parametrize("k", [1, 2])
def test_nested_space_identity(k):
    S = amr.AmrSpace(inputs.refined_mesh(**MESH), k)
    assert _nested_defect(S, k) < 1e-13
    # a wrong weight on one hanging node is seen
    r = int(np.nonzero(S.hanging)[0][7])
    C = S.C.tolil()
    g = C.rows[r][0]
    C[r, g] = C[r, g] + 0.05
    S.C = C.tocsr()
    assert _nested_defect(S, k) > 1e-4


@pytest.mark.parametrize("k,newton", [(1, True), (2, True), (2, False)])
def test_constrained_jacobian(k, newton):
    S = amr.AmrSpace(inputs.refined_mesh(**MESH), k)
    F = inputs.fourier_field(5)
    u0 = F(S.true_points()).T.ravel()
    nu, dt = 0.01, 1e-2
    J = amr.jacobian_matrix(S, u0, nu, dt, newton)
    dx = np.random.default_rng(0).standard_normal(4 * S.N)
    y = amr.jacobian_apply(S, dx, u0, nu, dt, newton)
    assert np.abs(J @ dx - y).max() <= 1e-13 * np.abs(y).max()
    e = np.zeros(4 * S.N)
    e[3 * S.N:] = 1.0
    assert np.abs(J @ e).max() <= 1e-13 * abs(J).max()
    mask = S.ns_dirichlet_true()
    assert np.all(J[mask][:, ~mask].nnz == 0)


# ------------------------------------------------------------------ multigrid
from oracle import amr_mg, ns_mg  # noqa: E402


def test_global_coarsening_sequence():
    m = inputs.refined_mesh(**MESH)
    seq = [m]
    while seq[-1]["level"].max() > 0:
        seq.append(amr_mg.coarsen(seq[-1]))
    assert [s["level"].max() for s in seq] == list(range(m["level"].max(), -1, -1))
    for s in seq:
        _, count = _level_map(dict(s, levels=m["levels"]))
        assert (count == 1).all()
    assert len(seq[-1]["level"]) == m["n"] ** 3


@pytest.mark.parametrize("k", [1, 2])
def test_multigrid_of_refinement_everywhere_is_structured(k):
    m = inputs.refined_mesh(2, 0, levels=1, centre=[0.5] * 3, radius=10.0)
    S = amr.AmrSpace(m, k)
    u0 = inputs.fourier_field(4)(S.true_points()).T.ravel()
    H = amr_mg.AmrNSHierarchy(m, k, 0.01, 1e-2, u0)
    Hs = ns_mg.NSHierarchy(3, [4, 4, 4], inputs.structured_vertices(3, [4, 4, 4]), k, 0.01, 1e-2, u0)
    b = inputs.uniform_vector(4 * S.N, 5)
    ref = Hs.vcycle(b)
    assert np.abs(H.vcycle(b) - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("k", [1, 2])
def test_refined_multigrid_transfers_and_solve(k):
    m = inputs.refined_mesh(**MESH)
    S = amr.AmrSpace(m, k)
    u0 = inputs.fourier_field(4)(S.true_points()).T.ravel()
    H = amr_mg.AmrNSHierarchy(m, k, 0.01, 1e-2, u0)
    assert H.nga == 2
    q = lambda p: 1 + p[:, 0] ** k + p[:, 1] * p[:, 2] ** k  # noqa: E731
    for j in range(H.nga):  # the pressure block interpolates Q_k polynomials exactly
        Sf, Sc = H.spaces[j], H.spaces[j + 1]
        Pp = H.P[j][3 * Sf.N:, 3 * Sc.N:]
        assert np.abs(Pp @ q(Sc.true_points()) - q(Sf.true_points())).max() < 1e-13
        assert abs(H.P[j][:3 * Sf.N][H.fixed[j][:3 * Sf.N]]).max() == 0  # Dirichlet rows
    xt = inputs.uniform_vector(4 * S.N, 3)
    xt[H.fixed[0]] = 0.0
    b = H.J[0] @ xt
    x, its, rel = H.solve(b, rtol=1e-8)
    assert rel <= 1e-8 and its <= 12
    assert np.linalg.norm(b - H.J[0] @ x) <= 1.01e-8 * np.linalg.norm(b)

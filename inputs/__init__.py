"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds no finite-element arithmetic.  It produces only grid
coordinates, seeded random numbers and closed-form manufactured fields
evaluated at points that the caller supplies.  Both the CPU oracle and the HIP
path take their inputs from here; nothing here imports either of them.

Conventions
-----------
* Structured meshes of the unit square / cube with ``n[a]`` cells along axis
  ``a``.  Vertices are numbered lexicographically with x fastest:
  vertex (i, j, l) -> i + (n0+1) * (j + (n1+1) * l).
* Vertex noise: every interior vertex coordinate a is moved by a draw from
  U[-noise*h_a, noise*h_a], h_a = 1/n_a; vertices on the boundary stay fixed so
  the domain stays the unit square / cube.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "structured_vertices",
    "coarsen_vertices",
    "uniform_vector",
    "manufactured_2d",
    "manufactured_3d",
    "fourier_field",
    "refined_mesh",
    "request_stream",
    "Request",
]


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def structured_vertices(dim: int, n, noise: float = 0.0, seed: int = 0) -> np.ndarray:
    """Vertex coordinates ``[(n0+1)*(n1+1)*(n2+1), dim]`` float64 of a
    structured grid of the unit square/cube, optionally perturbed.

    ``noise`` is the perturbation bound as a fraction of the cell size.  The
    draw is one ``uniform(-noise*h, noise*h)`` array of shape [n_vertices, dim]
    in vertex order, so a mesh is fully determined by (dim, n, noise, seed).
    """
    n = [int(v) for v in (n if hasattr(n, "__len__") else [n] * dim)]
    assert len(n) == dim and dim in (2, 3)
    axes = [np.linspace(0.0, 1.0, na + 1) for na in n]
    grids = np.meshgrid(*axes, indexing="ij")  # grids[a][i, j, (l)]
    # lexicographic with x fastest: flatten in Fortran order of (i, j, l)
    X = np.stack([g.ravel(order="F") for g in grids], axis=1)
    if noise > 0.0:
        h = np.array([1.0 / na for na in n])
        delta = _rng(seed).uniform(-1.0, 1.0, size=X.shape) * (noise * h)[None, :]
        idx = np.stack(np.meshgrid(*[np.arange(na + 1) for na in n], indexing="ij"), 0)
        idx = idx.reshape(dim, -1, order="F")
        on_bnd = np.zeros(X.shape[0], dtype=bool)
        for a in range(dim):
            on_bnd |= (idx[a] == 0) | (idx[a] == n[a])
        delta[on_bnd] = 0.0
        X = X + delta
    return np.ascontiguousarray(X)


def coarsen_vertices(dim: int, n, X: np.ndarray, levels: int = 1) -> np.ndarray:
    """Vertices of the mesh with n/2^levels cells per direction obtained by
    keeping the fine vertices whose indices are all divisible by 2^levels."""
    n = [int(v) for v in (n if hasattr(n, "__len__") else [n] * dim)]
    s = 2 ** levels
    shape = [na + 1 for na in n]
    V = X.reshape(shape[::-1] + [dim])  # [l][j][i][:] since x fastest
    if dim == 2:
        V = V[::s, ::s]
    else:
        V = V[::s, ::s, ::s]
    return np.ascontiguousarray(V.reshape(-1, dim))


def uniform_vector(n: int, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """float64 vector of U[lo, hi] draws."""
    return _rng(seed).uniform(lo, hi, size=int(n))


# ---------------------------------------------------------------------------
# Manufactured solutions (closed forms; no discretisation involved)
# ---------------------------------------------------------------------------
_pi = math.pi


def _s(t):  # sin^2(pi t)
    return np.sin(_pi * t) ** 2


def _s1(t):  # d/dt sin^2(pi t) = pi sin(2 pi t)
    return _pi * np.sin(2 * _pi * t)


def _s2(t):
    return 2 * _pi ** 2 * np.cos(2 * _pi * t)


def _s3(t):
    return -4 * _pi ** 3 * np.sin(2 * _pi * t)


def manufactured_2d(x: np.ndarray, nu: float = 1.0):
    """u = curl(sin^2(pi x) sin^2(pi y)), p = cos(pi x) cos(pi y) and the
    forcing f = -nu Lap(u) + grad(p).  ``x``: [..., 2].  Returns (u, p, f)."""
    X, Y = x[..., 0], x[..., 1]
    # psi = s(x) s(y); u = (psi_y, -psi_x)
    u0 = _s(X) * _s1(Y)
    u1 = -_s1(X) * _s(Y)
    lap_u0 = _s2(X) * _s1(Y) + _s(X) * _s3(Y)
    lap_u1 = -(_s3(X) * _s(Y) + _s1(X) * _s2(Y))
    p = np.cos(_pi * X) * np.cos(_pi * Y)
    px = -_pi * np.sin(_pi * X) * np.cos(_pi * Y)
    py = -_pi * np.cos(_pi * X) * np.sin(_pi * Y)
    u = np.stack([u0, u1], -1)
    f = np.stack([-nu * lap_u0 + px, -nu * lap_u1 + py], -1)
    return u, p, f


def manufactured_3d(x: np.ndarray, nu: float = 1.0):
    """u = curl(psi, psi, psi) with psi = sin^2(pi x) sin^2(pi y) sin^2(pi z),
    p = cos(pi x) cos(pi y) cos(pi z), f = -nu Lap(u) + grad(p).
    ``x``: [..., 3].  Returns (u, p, f)."""
    X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
    sx, sy, sz = _s(X), _s(Y), _s(Z)
    s1x, s1y, s1z = _s1(X), _s1(Y), _s1(Z)
    s2x, s2y, s2z = _s2(X), _s2(Y), _s2(Z)
    s3x, s3y, s3z = _s3(X), _s3(Y), _s3(Z)
    psi_x = s1x * sy * sz
    psi_y = sx * s1y * sz
    psi_z = sx * sy * s1z
    lap_psi_x = s3x * sy * sz + s1x * s2y * sz + s1x * sy * s2z
    lap_psi_y = s2x * s1y * sz + sx * s3y * sz + sx * s1y * s2z
    lap_psi_z = s2x * sy * s1z + sx * s2y * s1z + sx * sy * s3z
    u = np.stack([psi_y - psi_z, psi_z - psi_x, psi_x - psi_y], -1)
    lap = np.stack([lap_psi_y - lap_psi_z, lap_psi_z - lap_psi_x, lap_psi_x - lap_psi_y], -1)
    cx, cy, cz = np.cos(_pi * X), np.cos(_pi * Y), np.cos(_pi * Z)
    snx, sny, snz = np.sin(_pi * X), np.sin(_pi * Y), np.sin(_pi * Z)
    p = cx * cy * cz
    gp = np.stack([-_pi * snx * cy * cz, -_pi * cx * sny * cz, -_pi * cx * cy * snz], -1)
    f = -nu * lap + gp
    return u, p, f


def manufactured_forcing_3d_torch(x, nu: float):
    """Forcing f = -nu Lap(u) + grad(p) of ``manufactured_3d`` for a torch
    tensor x [..., 3] (evaluated where x lives, e.g. on the device)."""
    import torch

    pi = math.pi
    X, Y, Z = x[..., 0], x[..., 1], x[..., 2]

    def s(t):
        return torch.sin(pi * t) ** 2

    def s1(t):
        return pi * torch.sin(2 * pi * t)

    def s2(t):
        return 2 * pi ** 2 * torch.cos(2 * pi * t)

    def s3(t):
        return -4 * pi ** 3 * torch.sin(2 * pi * t)

    sx, sy, sz = s(X), s(Y), s(Z)
    s1x, s1y, s1z = s1(X), s1(Y), s1(Z)
    s2x, s2y, s2z = s2(X), s2(Y), s2(Z)
    s3x, s3y, s3z = s3(X), s3(Y), s3(Z)
    lap_psi_x = s3x * sy * sz + s1x * s2y * sz + s1x * sy * s2z
    lap_psi_y = s2x * s1y * sz + sx * s3y * sz + sx * s1y * s2z
    lap_psi_z = s2x * sy * s1z + sx * s2y * s1z + sx * sy * s3z
    cx, cy, cz = torch.cos(pi * X), torch.cos(pi * Y), torch.cos(pi * Z)
    snx, sny, snz = torch.sin(pi * X), torch.sin(pi * Y), torch.sin(pi * Z)
    f = torch.stack([-nu * (lap_psi_y - lap_psi_z) - pi * snx * cy * cz,
                     -nu * (lap_psi_z - lap_psi_x) - pi * cx * sny * cz,
                     -nu * (lap_psi_x - lap_psi_y) - pi * cx * cy * snz], -1)
    return f


def manufactured_inhomogeneous_3d(x: np.ndarray, nu: float = 1.0):
    """u = (sin pi y, sin pi z, sin pi x), p = 0: divergence free, nonzero on
    the boundary, Lap u = -pi^2 u.  Returns (u, p, f)."""
    X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
    u = np.stack([np.sin(_pi * Y), np.sin(_pi * Z), np.sin(_pi * X)], -1)
    p = np.zeros_like(X)
    f = nu * _pi ** 2 * u
    return u, p, f


# ---------------------------------------------------------------------------
# Random divergence-free Fourier field (linearisation point of the NS Jacobian)
# ---------------------------------------------------------------------------
def _fourier_modes():
    modes = []
    for a in range(-2, 3):
        for b in range(-2, 3):
            for c in range(-2, 3):
                k = (a, b, c)
                if k == (0, 0, 0):
                    continue
                first = next(v for v in k if v != 0)
                if first > 0:
                    modes.append(k)
    return np.array(modes, dtype=np.int64)  # 62 representatives of {-2..2}^3\0 mod +-


@dataclass
class FourierField:
    kappa: np.ndarray  # [m, 3] int
    a: np.ndarray  # [m, 3]
    b: np.ndarray  # [m, 3]

    def __call__(self, x: np.ndarray) -> np.ndarray:
        """Evaluate the field at points x [..., 3] -> [..., 3]."""
        ph = 2 * _pi * np.tensordot(x, self.kappa.T.astype(np.float64), axes=1)  # [..., m]
        return np.tensordot(np.cos(ph), self.a, axes=1) + np.tensordot(np.sin(ph), self.b, axes=1)


def fourier_field(seed: int, n_modes: int = 8) -> FourierField:
    """Divergence-free field sum_m a_m cos(2 pi k_m.x) + b_m sin(2 pi k_m.x),
    k_m drawn without replacement from the 62 representatives of
    {-2..2}^3 minus 0 modulo sign, a_m, b_m ~ N(0, I) projected orthogonal to
    k_m, scaled so that 1/2 sum(|a_m|^2 + |b_m|^2) = 1 (unit RMS on the unit
    cube)."""
    rng = _rng(seed)
    modes = _fourier_modes()
    sel = rng.choice(len(modes), size=n_modes, replace=False)
    kap = modes[sel]
    a = rng.standard_normal((n_modes, 3))
    b = rng.standard_normal((n_modes, 3))
    kn = kap / np.linalg.norm(kap, axis=1, keepdims=True)
    a -= (a * kn).sum(1, keepdims=True) * kn
    b -= (b * kn).sum(1, keepdims=True) * kn
    scale = math.sqrt(0.5 * ((a ** 2).sum() + (b ** 2).sum()))
    return FourierField(kap, a / scale, b / scale)


# ---------------------------------------------------------------------------
# Locally refined meshes
# ---------------------------------------------------------------------------
_FACE_EDGE = [(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)
              if 1 <= abs(a) + abs(b) + abs(c) <= 2]


def _dilate(m: np.ndarray) -> np.ndarray:
    """Cells of a boolean [z, y, x] grid that are set or share a face or an
    edge with a set cell."""
    out = m.copy()
    Z, Y, X = m.shape
    for dz, dy, dx in _FACE_EDGE:
        src = m[max(0, -dz):Z - max(0, dz), max(0, -dy):Y - max(0, dy), max(0, -dx):X - max(0, dx)]
        out[max(0, dz):Z - max(0, -dz), max(0, dy):Y - max(0, -dy), max(0, dx):X - max(0, -dx)] |= src
    return out


def refined_mesh(n: int, seed: int = 0, levels: int = 2, centre=None, radius=None) -> dict:
    """Leaves of a locally refined mesh of the unit cube: n^3 base cells;
    cells whose centre lies in a sphere are split into 8 children, ``levels``
    times; then a 2:1 closure over face and edge neighbours (a cell whose
    face or edge neighbour is refined is refined too, finest level first).
    Sphere: centre ~ U[0.3, 0.7]^3, radius ~ U[0.1, 0.2] (PCG64), unless given.

    Returns {"n", "levels", "centre", "radius", "level" [nc] int32,
    "idx" [nc, 3] int32}: cell (l, i, j, k) spans
    [i, i + 1] x [j, j + 1] x [k, k + 1] / (n 2^l).  Leaves are listed by
    level, then lexicographically (x fastest) within a level."""
    rng = _rng(seed)
    c0 = rng.uniform(0.3, 0.7, 3)
    r0 = rng.uniform(0.1, 0.2)
    centre = c0 if centre is None else np.asarray(centre, dtype=np.float64)
    radius = r0 if radius is None else float(radius)
    ref = []  # ref[l]: [z, y, x] booleans, level-l cell is split
    for l in range(levels):
        m = n << l
        ax = (np.arange(m) + 0.5) / m
        zz, yy, xx = np.meshgrid(ax, ax, ax, indexing="ij")
        inside = (xx - centre[0]) ** 2 + (yy - centre[1]) ** 2 + (zz - centre[2]) ** 2 < radius ** 2
        if l > 0:  # only children of split cells exist
            inside &= ref[l - 1].repeat(2, 0).repeat(2, 1).repeat(2, 2)
        ref.append(inside)
    for l in range(levels - 1, 0, -1):  # 2:1 closure
        need = _dilate(ref[l])
        m = n << (l - 1)
        ref[l - 1] |= need.reshape(m, 2, m, 2, m, 2).any(axis=(1, 3, 5))
    lev, idx = [], []
    for l in range(levels + 1):
        m = n << l
        exists = np.ones((m, m, m), dtype=bool) if l == 0 else ref[l - 1].repeat(2, 0).repeat(2, 1).repeat(2, 2)
        leaf = exists & ~ref[l] if l < levels else exists
        z, y, x = np.nonzero(leaf)
        lev.append(np.full(len(x), l, dtype=np.int32))
        idx.append(np.stack([x, y, z], 1).astype(np.int32))
    return {"n": int(n), "levels": int(levels), "centre": centre, "radius": radius,
            "level": np.concatenate(lev), "idx": np.concatenate(idx)}


# ---------------------------------------------------------------------------
# Served request stream
# ---------------------------------------------------------------------------
@dataclass
class Request:
    rid: int
    arrival: float  # seconds after stream start
    n: int  # cells per direction
    k: int  # velocity degree
    nu: float
    noise: float
    mesh_seed: int


def request_stream(n_requests: int, rate: float, seed: int = 0, sizes=(8, 16, 32, 64),
                   degrees=(2, 3, 4), nu_range=(1e-2, 1.0), noise: float = 0.1):
    """Poisson arrivals at ``rate`` per second; n uniform over ``sizes``, k
    uniform over ``degrees``, nu log-uniform in ``nu_range``."""
    rng = _rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n_requests)
    t = np.cumsum(gaps)
    ns = rng.choice(np.array(sizes), size=n_requests)
    ks = rng.choice(np.array(degrees), size=n_requests)
    lo, hi = math.log10(nu_range[0]), math.log10(nu_range[1])
    nus = 10.0 ** rng.uniform(lo, hi, size=n_requests)
    out = []
    for i in range(n_requests):
        out.append(Request(i, float(t[i]), int(ns[i]), int(ks[i]), float(nus[i]), noise, seed * 100003 + i))
    return out


def smooth_mapped_vertices(dim: int, n, amp: float = 0.1) -> np.ndarray:
    """Vertices of the structured grid moved by the smooth map
    x_a -> x_a + amp * prod_b sin(pi x_b), which fixes the boundary."""
    X = structured_vertices(dim, n)
    bump = np.prod(np.sin(_pi * X), axis=1)
    return np.ascontiguousarray(X + amp * bump[:, None])


def ns_velocity(dim: int, node_counts, seed: int = 0, n_modes: int = 8) -> np.ndarray:
    """Smooth linearisation point for the Navier-Stokes Jacobian: the Fourier
    field of ``fourier_field(seed)`` sampled on a uniform grid of the unit cube
    with ``node_counts`` points per direction (node index / (count - 1), so
    no basis or mesh information is used), blocked [u_0 | u_1 | (u_2)] with x
    fastest.  Unit RMS; nonzero on the boundary."""
    F = fourier_field(seed, n_modes)
    c = [int(v) for v in node_counts][:dim]
    axes = [np.linspace(0.0, 1.0, v) if v > 1 else np.zeros(1) for v in c]
    while len(axes) < 3:
        axes.append(np.full(1, 0.3))
    out = np.empty((dim, int(np.prod(c))))
    zz, yy = np.meshgrid(axes[2], axes[1], indexing="ij")
    for iz in range(len(axes[2])):  # slab by slab (bounded memory on large grids)
        pts = np.stack(np.broadcast_arrays(axes[0][None, :], yy[iz][:, None], zz[iz][:, None]), -1)
        v = F(pts.reshape(-1, 3))[:, :dim]
        m = v.shape[0]
        out[:, iz * m:(iz + 1) * m] = v.T
    return out.ravel()


def block_degrees(n, seed: int, block: int = 4, lo: int = 2, hi: int = 6) -> np.ndarray:
    """Per-cell polynomial degrees of a 3D structured mesh with n cells per
    direction: one degree per block^3 cell block, uniform on {lo..hi}
    (PCG64), returned per cell in lexicographic order (x fastest)."""
    n = [int(v) for v in (n if hasattr(n, "__len__") else [n] * 3)]
    nb = [(v + block - 1) // block for v in n]
    d = _rng(seed).integers(lo, hi + 1, size=nb[::-1])  # [bz, by, bx]
    z, y, x = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    return d[z // block, y // block, x // block].ravel().astype(np.int32)

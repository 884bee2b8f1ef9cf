"""GPU parity of the hp variant (Sec. 3, minimum rule) against the CPU oracle,
through the C ABI: hp Stokes operator and blocks, the velocity block and its
Jacobi diagonal on every hp level, the p-transfers (including the last one
into the structured degree-2 level), the V-cycle, the block preconditioner
and the FGMRES solve.

Tolerances as for the structured path: FP64 operators, diagonals and
transfers within 1e-12 relative (2-norm and max-norm), FP32 operators within
1e-5, V-cycle and preconditioner within 1e-10 (λ passed from the oracle),
solves to the FGMRES tolerance with the error bound set by the system's
condition number (velocity 1e-6, pressure 1e-3 relative, see the oracle
pins).
"""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

import inputs
import paper_2603_29621_amd as mfs
from oracle import hp

pytestmark = pytest.mark.gpu


def cuda(x, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda", dtype)


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def relerr(y, ref):
    d = y - ref
    n2 = np.linalg.norm(ref)
    ninf = np.abs(ref).max()
    return max(np.linalg.norm(d) / (n2 if n2 > 0 else 1), np.abs(d).max() / (ninf if ninf > 0 else 1))


CASES = [
    ([2, 2, 2], [2, 3, 4, 2, 3, 3, 2, 4], 0.2),
    ([3, 2, 2], [2, 5, 3, 4, 2, 6, 3, 3, 4, 2, 5, 2], 0.2),
    ([4, 4, 4], "blocks", 0.1),
]


def _case(n, deg, noise, seed=2):
    if deg == "blocks":
        deg = inputs.block_degrees(n, seed=5, block=2, lo=2, hi=6)
    X = inputs.structured_vertices(3, n, noise=noise, seed=seed)
    return X, np.asarray(deg, dtype=np.int32)


@pytest.mark.parametrize("n,deg,noise", CASES)
def test_hp_operators(n, deg, noise):
    X, deg = _case(n, deg, noise)
    nu = 0.7
    H = hp.HpStokes(n, X, deg, nu)
    h = mfs.mfs_setup_hp(n, X, deg, nu, mfs.mfs_default_options(mg_levels=0))
    try:
        assert mfs.mfs_n_dofs(h, 0) == (H.Nu, H.Np)
        N = H.K.shape[0]
        x = inputs.uniform_vector(N, 11)
        y = torch.empty(N, dtype=torch.float64, device="cuda")
        mfs.mfs_vmult(h, mfs.MFS_OP_STOKES, mfs.MFS_FP64, 0, y, cuda(x))
        assert relerr(host(y), H.K @ x) <= 1e-12
        y32 = torch.empty(N, dtype=torch.float32, device="cuda")
        mfs.mfs_vmult(h, mfs.MFS_OP_STOKES, mfs.MFS_FP32, 0, y32, cuda(x, torch.float32))
        assert relerr(host(y32), H.K @ x) <= 1e-5
        nv = H.nvel
        mask = H.mask[:nv]
        z = (~mask).astype(float)
        A = (sp.diags(z) @ H.Avec @ sp.diags(z) + sp.diags(mask.astype(float))).tocsr()
        du = torch.empty(nv, dtype=torch.float64, device="cuda")
        dp = torch.empty(H.Np, dtype=torch.float64, device="cuda")
        mfs.mfs_vmult(h, mfs.MFS_OP_A, mfs.MFS_FP64, 0, du, cuda(x[:nv]))
        assert relerr(host(du), A @ x[:nv]) <= 1e-12
        mfs.mfs_vmult(h, mfs.MFS_OP_B, mfs.MFS_FP64, 0, du, cuda(x[nv:]))
        assert relerr(host(du), z * (H.B @ x[nv:])) <= 1e-12
        mfs.mfs_vmult(h, mfs.MFS_OP_BT, mfs.MFS_FP64, 0, dp, cuda(x[:nv]))
        assert relerr(host(dp), H.B.T @ (z * x[:nv])) <= 1e-12
        mfs.mfs_vmult(h, mfs.MFS_OP_MASS_P, mfs.MFS_FP64, 0, dp, cuda(x[nv:]))
        assert relerr(host(dp), H.M @ x[nv:]) <= 1e-12
    finally:
        mfs.mfs_destroy(h)


def test_hp_full_size_properties():
    """The 32^3 hp workload (degrees 2..6 per 4^3 block, seed 0, noise 0.1h),
    too large to assemble: sampled rows against the oracle computed cell by
    cell (1e-12), the constant pressure in the kernel, symmetry on the free
    rows, and FP32 against FP64."""
    n = [32, 32, 32]
    deg = inputs.block_degrees(n, seed=0, block=4, lo=2, hi=6)
    X = inputs.structured_vertices(3, n, noise=0.1, seed=0)
    h = mfs.mfs_setup_hp(n, X, deg, 1.0, mfs.mfs_default_options(mg_levels=0))
    try:
        Nu, Np = mfs.mfs_n_dofs(h, 0)
        nv = 3 * Nu
        N = nv + Np

        def K(x, op=mfs.MFS_OP_STOKES, prec=mfs.MFS_FP64, n_out=N):
            dt = torch.float64 if prec == mfs.MFS_FP64 else torch.float32
            y = torch.empty(n_out, dtype=dt, device="cuda")
            mfs.mfs_vmult(h, op, prec, 0, y, cuda(x, dt))
            return host(y)

        # Dirichlet velocity rows: A x = x there, for two random x
        x1, x2 = inputs.uniform_vector(nv, 3), inputs.uniform_vector(nv, 4)
        dirichlet = (K(x1, mfs.MFS_OP_A, n_out=nv) == x1) & (K(x2, mfs.MFS_OP_A, n_out=nv) == x2)
        assert 0 < dirichlet.sum() < nv // 4
        x = inputs.uniform_vector(N, 1)
        y = K(x)
        scale = np.abs(y[:nv][~dirichlet]).max()
        # constant pressure: B 1 = 0 on free rows, Dirichlet rows take the zero source
        e = np.zeros(N)
        e[nv:] = 1.0
        assert np.abs(K(e)).max() <= 1e-11 * scale
        # symmetry on the free rows
        m = np.concatenate([dirichlet, np.zeros(Np, dtype=bool)])
        xf, zf = np.where(m, 0.0, x), np.where(m, 0.0, inputs.uniform_vector(N, 2))
        a, b = K(xf) @ zf, xf @ K(zf)
        assert abs(a - b) <= 1e-11 * (np.abs(K(xf)) @ np.abs(zf))
        # FP32 against FP64
        x32 = x.astype(np.float32).astype(np.float64)
        assert relerr(K(x32, prec=mfs.MFS_FP32), K(x32)) <= 1e-5
        # sampled rows against the oracle, cell by cell (every kind of row)
        rows = np.unique(np.concatenate([
            np.random.default_rng(7).choice(N, 300, replace=False),
            [0, Nu - 1, Nu, 3 * Nu - 1, nv, N - 1]]))
        ref = hp.sampled_stokes_rows(n, X, deg, 1.0, x, rows)
        assert np.abs(y[rows] - ref).max() <= 1e-12 * np.abs(ref).max()
    finally:
        mfs.mfs_destroy(h)


def _hier(n, deg, noise, nu=1.0):
    X, deg = _case(n, deg, noise)
    sol = hp.HpStokesSolver(n, X, deg, nu)
    Hm = sol.mg
    h = mfs.mfs_setup_hp(n, X, deg, nu, mfs.mfs_default_options())
    nhp = len(Hm.hp)
    for l in range(nhp):
        Hm.lam[l] = 1.2 * Hm.exact_lambda_max(l)
        mfs.mfs_set_lambda(h, l, Hm.lam[l])
    for l in range(len(Hm.mg.spaces) - 1):
        Hm.mg.lam[l] = 1.2 * Hm.mg.exact_lambda_max(l)
        mfs.mfs_set_lambda(h, nhp + l, Hm.mg.lam[l])
    return h, sol


@pytest.mark.parametrize("n,deg,noise", CASES)
def test_hp_levels_diagonals_transfers(n, deg, noise):
    h, sol = _hier(n, deg, noise)
    Hm = sol.mg
    try:
        nhp = len(Hm.hp)
        assert mfs.mfs_n_levels(h) == nhp + len(Hm.mg.spaces)
        for l in range(nhp):
            V = Hm.hp[l][0]
            assert mfs.mfs_n_dofs(h, l)[0] == V.N
            x = inputs.uniform_vector(3 * V.N, 20 + l)
            y = torch.empty(3 * V.N, dtype=torch.float64, device="cuda")
            mfs.mfs_vmult(h, mfs.MFS_OP_A, mfs.MFS_FP64, l, y, cuda(x))
            assert relerr(host(y), Hm.A[l] @ x) <= 1e-12, l
            d = torch.empty(V.N, dtype=torch.float64, device="cuda")
            mfs.mfs_diagonal(h, l, d)
            assert relerr(host(d), 1.0 / Hm.Dinv[l][:V.N]) <= 1e-12, l
            P = Hm.P[l]
            xc = inputs.uniform_vector(P.shape[1], 30 + l)
            yf = cuda(x)
            mfs.mfs_prolongate_add(h, mfs.MFS_FP64, l, yf, cuda(xc))
            assert relerr(host(yf), x + P @ xc) <= 1e-12, l
            bc = torch.empty(P.shape[1], dtype=torch.float64, device="cuda")
            mfs.mfs_restrict(h, mfs.MFS_FP64, l, bc, cuda(x))
            assert relerr(host(bc), P.T @ x) <= 1e-12, l
    finally:
        mfs.mfs_destroy(h)


@pytest.mark.parametrize("n,deg,noise", CASES[:2])
def test_hp_vcycle_and_preconditioner(n, deg, noise):
    h, sol = _hier(n, deg, noise)
    try:
        nv = sol.sys.nvel
        b = inputs.uniform_vector(nv, 61)
        ref = sol.mg.vcycle(b)
        x = torch.empty(nv, dtype=torch.float64, device="cuda")
        mfs.mfs_vcycle(h, mfs.MFS_FP64, x, cuda(b))
        assert relerr(host(x), ref) <= 1e-10
        x32 = torch.empty(nv, dtype=torch.float32, device="cuda")
        mfs.mfs_vcycle(h, mfs.MFS_FP32, x32, cuda(b, torch.float32))
        assert relerr(host(x32), ref) <= 1e-4
        N = sol.sys.K.shape[0]
        r = inputs.uniform_vector(N, 62)
        refp = sol.precondition(r)
        y = torch.empty(N, dtype=torch.float64, device="cuda")
        mfs.mfs_precondition(h, mfs.MFS_FP64, y, cuda(r))
        assert relerr(host(y), refp) <= 1e-10
    finally:
        mfs.mfs_destroy(h)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_hp_solve(prec):
    n = [4, 4, 4]
    h, sol = _hier(n, "blocks", 0.1)
    try:
        s = sol.sys
        rng = np.random.default_rng(3)
        xs = rng.standard_normal(s.K.shape[0])
        xs[s.mask] = 0.0
        b = s.K @ xs
        x_ref, its_ref, _ = sol.solve(b, rtol=1e-10, maxit=100)
        x = torch.zeros(s.K.shape[0], dtype=torch.float64, device="cuda")
        p = mfs.MFS_FP64 if prec == "f64" else mfs.MFS_FP32
        info = mfs.mfs_solve(h, cuda(b), x, mfs.mfs_default_options(rtol=1e-10, maxit=100, precond_precision=p))
        assert info.status == 0 and info.rel_residual <= 1e-10
        xg = host(x)
        assert relerr(xg[:s.nvel], x_ref[:s.nvel]) <= 1e-6
        assert relerr(xg[s.nvel:], x_ref[s.nvel:]) <= 1e-3
        if prec == "f64":
            assert abs(info.iterations - its_ref) <= 1
        else:
            assert info.iterations <= its_ref + 3
    finally:
        mfs.mfs_destroy(h)

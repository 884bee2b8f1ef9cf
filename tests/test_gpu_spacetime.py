"""GPU parity of the space-time Kronecker operator (Sec. 4
eq. (proceedings-kronecker)) and of the temporal stage transfers against the
CPU oracle, through the C ABI; and of the velocity mass it is built from.

Tolerances: FP64 within 1e-12 relative (2-norm and max-norm), FP32 within
1e-5, as for the Stokes operator; stage transfers (a dense Q x Q mix per
entry) within 1e-14."""
import numpy as np
import pytest
import torch

import inputs
import paper_2603_29621_amd as mfs
from oracle import fem, spacetime

pytestmark = pytest.mark.gpu


def cuda(x, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda", dtype)


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def relerr(y, ref):
    d = y - ref
    return max(np.linalg.norm(d) / np.linalg.norm(ref), np.abs(d).max() / np.abs(ref).max())


CASES = [(2, [6, 5], 2, 0.2), (3, [4, 3, 5], 2, 0.2), (3, [3, 4, 3], 3, 0.2), (3, [3, 2, 3], 4, 0.1)]


@pytest.mark.parametrize("dim,n,k,noise", CASES)
def test_velocity_mass(dim, n, k, noise):
    nu = 0.8
    X = inputs.structured_vertices(dim, n, noise=noise, seed=3)
    h = mfs.mfs_setup(dim, n, X, k, nu, mfs.mfs_default_options(mg_levels=0))
    try:
        S = fem.Space(dim, n, X, k)
        Mu = spacetime.velocity_mass(S)
        mask = S.dirichlet
        x = inputs.uniform_vector(dim * S.Nv, 6)
        ref = np.concatenate([Mu @ np.where(mask, 0.0, x[c * S.Nv:(c + 1) * S.Nv]) for c in range(dim)])
        full_mask = np.tile(mask, dim)
        ref[full_mask] = x[full_mask]
        for prec, tol in ((mfs.MFS_FP64, 1e-12), (mfs.MFS_FP32, 1e-5)):
            dt = torch.float64 if prec == mfs.MFS_FP64 else torch.float32
            y = torch.empty(dim * S.Nv, dtype=dt, device="cuda")
            mfs.mfs_vmult(h, mfs.MFS_OP_MASS_U, prec, 0, y, cuda(x, dt))
            assert relerr(host(y), ref) <= tol
    finally:
        mfs.mfs_destroy(h)


@pytest.mark.parametrize("dim,n,k,noise", CASES)
@pytest.mark.parametrize("q", [1, 2, 3])
def test_space_time_operator(dim, n, k, noise, q):
    nu, tau = 0.6, 0.03
    X = inputs.structured_vertices(dim, n, noise=noise, seed=4)
    h = mfs.mfs_setup(dim, n, X, k, nu, mfs.mfs_default_options(mg_levels=0))
    try:
        S = fem.Space(dim, n, X, k)
        G = spacetime.G_matrix(q - 1)
        x = inputs.uniform_vector(q * S.n_dofs, 7)
        ref = spacetime.kron_apply(S, nu, tau, G, x)
        for prec, tol in ((mfs.MFS_FP64, 1e-12), (mfs.MFS_FP32, 1e-5)):
            dt = torch.float64 if prec == mfs.MFS_FP64 else torch.float32
            y = torch.empty(q * S.n_dofs, dtype=dt, device="cuda")
            work = torch.empty(q * dim * S.Nv, dtype=dt, device="cuda")
            mfs.mfs_st_vmult(h, G, tau, prec, y, cuda(x, dt), work)
            assert relerr(host(y), ref) <= tol, (prec, relerr(host(y), ref))
    finally:
        mfs.mfs_destroy(h)


@pytest.mark.parametrize("kf,kc", [(1, 0), (2, 1), (3, 1)])
def test_stage_transfers(kf, kc):
    dim, n, k = 3, [3, 2, 3], 2
    X = inputs.structured_vertices(dim, n, noise=0.1, seed=5)
    h = mfs.mfs_setup(dim, n, X, k, 1.0, mfs.mfs_default_options(mg_levels=0))
    try:
        S = fem.Space(dim, n, X, k)
        P = spacetime.time_prolongation(kf, kc)
        qf, qc = kf + 1, kc + 1
        xc = inputs.uniform_vector(qc * S.n_dofs, 8).reshape(qc, -1)
        xf = inputs.uniform_vector(qf * S.n_dofs, 9).reshape(qf, -1)
        y = torch.empty(qf * S.n_dofs, dtype=torch.float64, device="cuda")
        mfs.mfs_st_stage_transfer(h, P, mfs.MFS_FP64, y, cuda(xc.ravel()))
        assert relerr(host(y), (P @ xc).ravel()) <= 1e-14
        z = torch.empty(qc * S.n_dofs, dtype=torch.float64, device="cuda")
        mfs.mfs_st_stage_transfer(h, P.T.copy(), mfs.MFS_FP64, z, cuda(xf.ravel()))
        assert relerr(host(z), (P.T @ xf).ravel()) <= 1e-14
    finally:
        mfs.mfs_destroy(h)

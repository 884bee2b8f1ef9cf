"""GPU parity of the additive Schwarz relaxation of the monolithic
Navier-Stokes multigrid (Sec. 2; Sec. 5, Exp. 4: two relaxation steps around
ASM) against the CPU oracle, through the C ABI: the V-cycle with vertex-patch
ASM on every relaxation level, and FGMRES solves preconditioned by it.

Tolerances: as for the Jacobi V-cycle, FP64 within 1e-9 (about 30 operator
applications, explicit dense inverses of the patches and of the coarse level
on the GPU against LU-based inverses in the oracle) and FP32 within 1e-4;
solves to a true relative residual of 1e-10 within 1e-6 of the oracle's
FGMRES solution, FP64 iteration counts within one of the oracle's."""
import numpy as np
import pytest
import torch

import inputs
import paper_2603_29621_amd as mfs
from oracle import ns_mg

pytestmark = pytest.mark.gpu

ASM = dict(relax_type=mfs.MFS_RELAX_ASM, relax_steps=2, relax_omega=1.0)


def asm_opts(k):
    """Two sweeps; omega = 1 for the overlapping degree-2 patches, 0.5 for the
    degree-1 patches, which do not overlap (point-block Jacobi, which diverges
    undamped)."""
    return dict(ASM, relax_omega=1.0 if k == 2 else 0.5)


def cuda(x, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda", dtype)


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def relerr(y, ref):
    d = y - ref
    return max(np.linalg.norm(d) / np.linalg.norm(ref), np.abs(d).max() / np.abs(ref).max())


def _hierarchy(dim, n, k, nu, dt, noise=0.1, newton=True):
    X = inputs.structured_vertices(dim, n, noise=noise, seed=3)
    opts = mfs.mfs_default_options(pressure_offset=0, mg_levels=1, **asm_opts(k))
    h = mfs.mfs_setup(dim, n, X, k, nu, opts)
    u0 = inputs.ns_velocity(dim, [k * v + 1 for v in n], 5)
    H = ns_mg.NSHierarchy(dim, n, X, k, nu, dt, u0, newton=newton, smoother="asm", relax_steps=2,
                          omega=asm_opts(k)["relax_omega"])
    mfs.mfs_set_linearization(h, cuda(u0), dt, int(newton))
    return h, H


# every patch size (2D and 3D, degrees 1 and 2), ragged colour counts (odd
# vertex counts per direction)
CASES = [(2, [8, 8], 2), (2, [6, 10], 1), (2, [6, 4], 2), (3, [4, 4, 4], 2), (3, [6, 4, 4], 1), (3, [4, 2, 6], 2)]


@pytest.mark.parametrize("dim,n,k", CASES)
@pytest.mark.parametrize("dt", [0.05, 1.0])
def test_asm_vcycle(dim, n, k, dt):
    print(f"[asm vcycle] dim={dim} n={n} k={k} dt={dt}", flush=True)
    h, H = _hierarchy(dim, n, k, 0.01, dt)
    try:
        N = (dim + 1) * H.spaces[0].Nv
        b = inputs.uniform_vector(N, 60)
        ref = H.vcycle(b)
        x = torch.empty(N, dtype=torch.float64, device="cuda")
        mfs.mfs_vcycle(h, mfs.MFS_FP64, x, cuda(b))
        assert relerr(host(x), ref) <= 1e-9
        x32 = torch.empty(N, dtype=torch.float32, device="cuda")
        mfs.mfs_vcycle(h, mfs.MFS_FP32, x32, cuda(b, torch.float32))
        assert relerr(host(x32), ref) <= 1e-4
        # the patch colours add in a fixed order; in 3D so do the Jacobian's
        # cell colours, and the preconditioner entry point gives the same
        # bits (the 2D Jacobian adds with atomics: equal up to summation order)
        xp = torch.empty(N, dtype=torch.float64, device="cuda")
        mfs.mfs_precondition(h, mfs.MFS_FP64, xp, cuda(b))
        if dim == 3:
            assert torch.equal(xp, x)
        else:
            assert relerr(host(xp), host(x)) <= 1e-13
    finally:
        mfs.mfs_destroy(h)


@pytest.mark.parametrize("dim,n,k", [(2, [8, 8], 2), (3, [4, 4, 4], 2), (3, [8, 8, 8], 1)])
def test_asm_solve(dim, n, k):
    print(f"[asm solve] dim={dim} n={n} k={k}", flush=True)
    h, H = _hierarchy(dim, n, k, 0.01, 1.0)
    try:
        S = H.spaces[0]
        N = (dim + 1) * S.Nv
        xt = inputs.uniform_vector(N, 70)
        xt[H.fixed[0]] = 0.0
        b = H.J[0] @ xt
        x_ref, its_ref, rel_ref = ns_mg.solve(H, b, rtol=1e-10)
        assert rel_ref <= 1e-10
        for prec in (mfs.MFS_FP64, mfs.MFS_FP32):
            x = torch.zeros(N, dtype=torch.float64, device="cuda")
            info = mfs.mfs_solve(h, cuda(b), x, mfs.mfs_default_options(
                pressure_offset=0, rtol=1e-10, precond_precision=prec))
            assert info.status == 0 and info.rel_residual <= 1e-10
            xs = host(x)
            assert relerr(xs, x_ref) <= 1e-6
            if prec == mfs.MFS_FP64:
                assert abs(info.iterations - its_ref) <= 1
            else:
                assert info.iterations <= its_ref + 3
    finally:
        mfs.mfs_destroy(h)


def test_asm_footprint_and_refined_rejected():
    n = [8, 8, 8]
    X = inputs.structured_vertices(3, n)
    base = mfs.mfs_footprint(3, n, X, 2, mfs.mfs_default_options(pressure_offset=0))
    more = mfs.mfs_footprint(3, n, X, 2, mfs.mfs_default_options(pressure_offset=0, **ASM))
    # FP64 + FP32 inverses of 108 x 108 on the two relaxation levels (9^3 and 5^3 patches)
    assert more - base >= (9 ** 3 + 5 ** 3) * 108 * 108 * 12
    mesh = inputs.refined_mesh(4, seed=0, levels=1, radius=0.3)
    with pytest.raises(mfs.MfsError):
        mfs.mfs_setup_refined(mesh, 1, 0.01, mfs.mfs_default_options(pressure_offset=0, **ASM))

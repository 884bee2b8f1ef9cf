"""The allocation-free Q2/Q1 Stokes vmult (scratch in a static device array)
against the problem-based mfs_vmult through the C ABI: the same kernels, so
the results must be identical, on two calls in a row with the second on a
smaller mesh (the scratch keeps the first call's contents); the FP64 result
is also compared with the oracle; meshes beyond the static scratch are
rejected on the host before anything is enqueued."""
import numpy as np
import pytest
import torch

import inputs
import paper_2603_29621_amd as mfs
from oracle import fem

pytestmark = pytest.mark.gpu

NU = 0.7


def _reference(n, X, x, prec):
    """dst of mfs_vmult(STOKES) on a problem with the same mesh."""
    h = mfs.mfs_setup(3, n, X, 2, NU, mfs.mfs_default_options(mg_levels=0))
    try:
        dt = torch.float64 if prec == mfs.MFS_FP64 else torch.float32
        src = torch.from_numpy(x).to("cuda", dt)
        dst = torch.full_like(src, float("nan"))
        mfs.mfs_vmult(h, mfs.MFS_OP_STOKES, prec, 0, dst, src)
        torch.cuda.synchronize()
        return dst
    finally:
        mfs.mfs_destroy(h)


@pytest.mark.parametrize("prec", [mfs.MFS_FP64, mfs.MFS_FP32])
def test_noalloc_vmult_equals_problem_vmult(prec):
    dt = torch.float64 if prec == mfs.MFS_FP64 else torch.float32
    # several bricks with ragged tails in every direction, then a smaller mesh
    for n, seed in (([19, 11, 5], 1), ([5, 3, 3], 2)):
        print(f"noalloc vmult prec={prec} n={n}", flush=True)
        X = inputs.structured_vertices(3, n, noise=0.2, seed=seed)
        ndof = 3 * int(np.prod([2 * v + 1 for v in n])) + int(np.prod([v + 1 for v in n]))
        x = inputs.uniform_vector(ndof, seed + 10)
        ref = _reference(n, X, x, prec)
        Xd = torch.from_numpy(np.ascontiguousarray(X)).to("cuda", dt)
        src = torch.from_numpy(x).to("cuda", dt)
        dst = torch.full_like(src, float("nan"))
        mfs.mfs_stokes_vmult_noalloc(n, Xd, NU, prec, dst, src)
        torch.cuda.synchronize()
        assert torch.isfinite(dst).all()
        assert torch.equal(dst, ref)
        if prec == mfs.MFS_FP64:
            S = fem.Space(3, n, X, 2)
            K, _ = fem.stokes_operator(S, NU)
            y = K @ x
            assert np.abs(dst.cpu().numpy() - y).max() <= 1e-12 * np.abs(y).max()


def test_noalloc_vmult_rejects_meshes_beyond_the_scratch():
    n = [64, 64, 64]  # 4,096 bricks, more than the static scratch holds
    nv = int(np.prod([2 * v + 1 for v in n]))
    npr = int(np.prod([v + 1 for v in n]))
    Xd = torch.zeros(3 * npr, dtype=torch.float64, device="cuda")
    v = torch.zeros(3 * nv + npr, dtype=torch.float64, device="cuda")
    w = torch.zeros_like(v)
    with pytest.raises(mfs.MfsError) as e:
        mfs.mfs_stokes_vmult_noalloc(n, Xd, NU, mfs.MFS_FP64, w, v)
    assert e.value.code == mfs.MFS_EINVAL
    assert "scratch" in str(e.value)

"""The C-ABI library loads and exports every entry point of the header, and
its host-side validation works without a GPU (no compute calls here)."""
import ctypes
import os
import re

import numpy as np
import pytest

import inputs
import paper_2603_29621_amd as mfs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    txt = open(os.path.join(ROOT, "include", "mfstokes.h")).read()
    return sorted(set(re.findall(r"\b(mfs_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_header_symbols():
    L = mfs.lib()
    names = _header_functions()
    assert len(names) >= 20
    for name in names:
        assert hasattr(L, name), name
    assert sorted(names) == sorted(mfs.EXPORTED)


def test_default_options():
    o = mfs.mfs_default_options()
    assert o.pressure_offset == 1 and o.cheb_degree == 5 and o.restart == 30
    assert o.precond_precision == mfs.MFS_FP32 and abs(o.rtol - 1e-8) < 1e-20
    assert o.graphs == 1


def test_footprint_and_validation_host_only():
    X = inputs.structured_vertices(3, [4, 4, 4])
    b = mfs.mfs_footprint(3, [4, 4, 4], X, 2)
    assert b > 0
    b2 = mfs.mfs_footprint(3, [8, 8, 8], inputs.structured_vertices(3, [8, 8, 8]), 2)
    assert b2 > 4 * b
    with pytest.raises(mfs.MfsError) as e:
        mfs.mfs_footprint(4, [4, 4, 4], X, 2)
    assert e.value.code == mfs.MFS_EINVAL
    with pytest.raises(mfs.MfsError):
        mfs.mfs_footprint(3, [4, 4, 4], X, 1)  # Taylor-Hood needs k >= 2
    with pytest.raises(mfs.MfsError):
        mfs.mfs_footprint(3, [4, 4, 4], X, 9)
    o = mfs.mfs_default_options(restart=40)
    with pytest.raises(mfs.MfsError):
        mfs.mfs_footprint(3, [4, 4, 4], X, 2, o)


def test_navier_stokes_options_validated_on_host():
    X = inputs.structured_vertices(3, [4, 4, 4])
    o = mfs.mfs_default_options()
    assert o.relax_steps == 5 and o.relax_omega == 0.5
    # equal order: k <= 3 for the operator, k <= 2 with the multigrid hierarchy
    with pytest.raises(mfs.MfsError) as e:
        mfs.mfs_footprint(3, [4, 4, 4], X, 3, mfs.mfs_default_options(pressure_offset=0))
    assert e.value.code == mfs.MFS_EUNSUPPORTED
    assert mfs.mfs_footprint(3, [4, 4, 4], X, 3, mfs.mfs_default_options(pressure_offset=0, mg_levels=0)) > 0
    with pytest.raises(mfs.MfsError) as e:
        mfs.mfs_footprint(3, [4, 4, 4], X, 4, mfs.mfs_default_options(pressure_offset=0, mg_levels=0))
    assert e.value.code == mfs.MFS_EUNSUPPORTED
    with pytest.raises(mfs.MfsError):
        mfs.mfs_footprint(3, [4, 4, 4], X, 2, mfs.mfs_default_options(pressure_offset=0, relax_omega=2.0))
    # the footprint holds the per-point linearisation data of every level (FP64 + FP32)
    fp1 = mfs.mfs_footprint(3, [8, 8, 8], inputs.structured_vertices(3, [8, 8, 8]), 1,
                            mfs.mfs_default_options(pressure_offset=0, mg_levels=0))
    assert fp1 >= 8 ** 3 * 8 * 16 * 12


def test_hp_setup_validates_degrees_on_host():
    X = inputs.structured_vertices(3, [2, 2, 2])
    with pytest.raises(mfs.MfsError) as e:
        mfs.mfs_setup_hp([2, 2, 2], X, [2, 3, 7, 2, 2, 2, 2, 2], 1.0, stream=0)
    assert e.value.code == mfs.MFS_EINVAL
    with pytest.raises(mfs.MfsError) as e:
        mfs.mfs_setup_hp([2, 2, 2], X, [2] * 8, 1.0, mfs.mfs_default_options(pressure_offset=0), stream=0)
    assert e.value.code == mfs.MFS_EINVAL


def test_refined_mesh_validation_host_only():
    """mfs_setup_refined rejects bad leaves and unsupported options before it
    touches the device (null stream, no GPU needed)."""
    m = inputs.refined_mesh(3, 0, levels=2, centre=[0.4, 0.5, 0.55], radius=0.3)
    overlap = dict(m, idx=m["idx"].copy())
    overlap["idx"][5] = overlap["idx"][6]
    gap = dict(m, level=m["level"][1:], idx=m["idx"][1:])
    deep = dict(m, level=m["level"].copy())
    deep["level"][0] = 3
    cases = [(overlap, 2, None, mfs.MFS_EINVAL), (gap, 2, None, mfs.MFS_EINVAL), (deep, 2, None, mfs.MFS_EINVAL),
             (m, 3, None, mfs.MFS_EUNSUPPORTED),
             (m, 2, mfs.mfs_default_options(pressure_offset=1, mg_levels=0), mfs.MFS_EUNSUPPORTED)]
    for mesh, k, opts, code in cases:
        with pytest.raises(mfs.MfsError) as e:
            mfs.mfs_setup_refined(mesh, k, 0.01, opts, stream=0)
        assert e.value.code == code


@pytest.mark.parametrize("k", [1, 2])
def test_refined_space_counts_host_only(k):
    """The host construction of the refined-mesh space (no device): unknown and
    hanging-node counts equal the oracle's on seeded and degenerate meshes."""
    from oracle import amr

    for kw in [dict(n=3, seed=0, levels=2, centre=[0.4, 0.5, 0.55], radius=0.3), dict(n=4, seed=1, levels=2),
               dict(n=1, seed=0, levels=2, centre=[0.3, 0.4, 0.6], radius=0.45),
               dict(n=2, seed=0, levels=1, centre=[0.5, 0.5, 0.5], radius=10.0)]:
        m = inputs.refined_mesh(**kw)
        S = amr.AmrSpace(m, k)
        assert mfs.mfs_refined_count(m, k) == (S.N, int(S.hanging.sum()))

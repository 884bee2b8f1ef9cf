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
    return sorted(set(re.findall(r"\b(mfs_[a-z_]+)\s*\(", txt)))


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

"""vfpi_vnode_pattern (host code of the C library, no GPU): the block pattern
of the eq. vnode system against the nonzero blocks of the oracle's matrix,
and its argument checks."""
import ctypes

import numpy as np
import pytest

import scenes
from oracle.vnode import augmented_matrix
from paper_2201_09212_amd import _abi


def _i32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _pattern(vs, cap=None):
    rp, ci, jp, jc = _i32(vs.row_ptr), _i32(vs.col_idx), _i32(vs.jv_ptr), _i32(vs.jv_col)
    g_ptr = np.zeros(vs.n_o + vs.n_v + 1, dtype=np.int32)
    nnz = _abi.vfpi_vnode_pattern(vs.n_o, rp.ctypes.data, ci.ctypes.data, vs.n_v, jp.ctypes.data, jc.ctypes.data,
                                  g_ptr.ctypes.data, None, 0)
    g_col = np.zeros(max(nnz, 1), dtype=np.int32)
    _abi.vfpi_vnode_pattern(vs.n_o, rp.ctypes.data, ci.ctypes.data, vs.n_v, jp.ctypes.data, jc.ctypes.data,
                            g_ptr.ctypes.data, g_col.ctypes.data, nnz if cap is None else cap)
    return g_ptr, g_col[:nnz]


@pytest.mark.parametrize("make", [lambda: scenes.rigid_box_on_floor(), lambda: scenes.particles_on_cloth(0),
                                  lambda: scenes.particles_on_cloth(3)])
def test_pattern_covers_exactly_the_nonzero_blocks(make):
    vs = make()
    g_ptr, g_col = _pattern(vs)
    n = vs.n_o + vs.n_v
    A = augmented_matrix(vs, 7.0).toarray().reshape(n, 3, n, 3)
    nz = np.abs(A).max(axis=(1, 3)) != 0
    mine = np.zeros((n, n), dtype=bool)
    for r in range(n):
        cols = g_col[g_ptr[r]:g_ptr[r + 1]]
        assert np.all(np.diff(cols[cols < vs.n_o]) > 0) and np.all(np.diff(cols[cols >= vs.n_o]) > 0)
        if r < vs.n_o:  # virtual columns last
            assert np.all(np.diff((cols >= vs.n_o).astype(int)) >= 0)
        mine[r, cols] = True
    assert np.array_equal(mine, nz)


def test_pattern_argument_errors():
    vs = scenes.particles_on_cloth(0)
    lib = _abi.load()
    rp, ci, jp, jc = _i32(vs.row_ptr), _i32(vs.col_idx), _i32(vs.jv_ptr), _i32(vs.jv_col)
    g_ptr = np.zeros(vs.n_o + vs.n_v + 1, dtype=np.int32)
    nnz = ctypes.c_int64()
    assert lib.vfpi_vnode_pattern(vs.n_o, rp.ctypes.data, ci.ctypes.data, vs.n_v, jp.ctypes.data, jc.ctypes.data,
                                  None, None, 0, ctypes.byref(nnz)) == _abi.VFPI_E_NULL
    g_col = np.zeros(10, dtype=np.int32)
    assert lib.vfpi_vnode_pattern(vs.n_o, rp.ctypes.data, ci.ctypes.data, vs.n_v, jp.ctypes.data, jc.ctypes.data,
                                  g_ptr.ctypes.data, g_col.ctypes.data, 10, ctypes.byref(nnz)) == _abi.VFPI_E_CAPACITY
    bad = jc.copy()
    bad[1] = bad[0]  # repeated column in one J_v row
    assert lib.vfpi_vnode_pattern(vs.n_o, rp.ctypes.data, ci.ctypes.data, vs.n_v, jp.ctypes.data, bad.ctypes.data,
                                  g_ptr.ctypes.data, None, 0, ctypes.byref(nnz)) == _abi.VFPI_E_SHAPE
    bad = jc.copy()
    bad[0] = vs.n_o
    assert lib.vfpi_vnode_pattern(vs.n_o, rp.ctypes.data, ci.ctypes.data, vs.n_v, jp.ctypes.data, bad.ctypes.data,
                                  g_ptr.ctypes.data, None, 0, ctypes.byref(nnz)) == _abi.VFPI_E_SHAPE
    unsorted = ci.copy()
    unsorted[[0, 1]] = unsorted[[1, 0]]
    assert lib.vfpi_vnode_pattern(vs.n_o, rp.ctypes.data, unsorted.ctypes.data, vs.n_v, jp.ctypes.data,
                                  jc.ctypes.data, g_ptr.ctypes.data, None, 0, ctypes.byref(nnz)) == _abi.VFPI_E_SHAPE

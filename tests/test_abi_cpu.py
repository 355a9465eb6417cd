"""The C ABI without a GPU: the library loads, exports every declared entry
point, and rejects bad arguments before touching HIP."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2608_07327_amd import mbpcg as M

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "mbpcg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mbpcg_[a-z_]+)\s*\(", src)))


def test_header_declares_the_documented_entry_points():
    assert set(_declared()) == set(M.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = M.load()
    for name in _declared():
        assert hasattr(L, name), name


def test_default_params():
    p = M.default_params()
    assert p.s == 4 and p.tol == 1e-8 and p.max_iter == 100000
    assert p.precond == M.PRECOND_JACOBI and p.tau == 1e-12 and p.precision == M.FP64
    assert p.block_size == 8


def test_status_strings():
    for st in (0, 1, -1, -2, -3, -4, -5, -6, -7):
        assert M.status_str(st)


def _create_csr(n, nnz, rowptr, colind, vals):
    L = M.load()
    h = C.c_void_p()
    rc = L.mbpcg_create_csr(C.byref(h), n, nnz, rowptr.ctypes.data if rowptr is not None else None,
                            colind.ctypes.data, vals.ctypes.data, M.MEM_HOST, None)
    return rc, h


def test_create_csr_rejects_bad_structure_before_hip():
    rp = np.array([0, 1, 2], np.int32)
    ci = np.array([0, 1], np.int32)
    v = np.array([1.0, 2.0])
    assert _create_csr(0, 2, rp, ci, v)[0] == M.ERR_INVALID_ARG
    assert _create_csr(2, 2, None, ci, v)[0] == M.ERR_INVALID_ARG
    assert _create_csr(2, 3, rp, ci, v)[0] == M.ERR_INVALID_ARG          # rowptr[n] != nnz
    assert _create_csr(2, 2, np.array([1, 1, 2], np.int32), ci, v)[0] == M.ERR_INVALID_ARG
    assert _create_csr(2, 2, np.array([0, 2, 1], np.int32), ci, v)[0] == M.ERR_INVALID_ARG
    assert _create_csr(2, 2, rp, np.array([0, 2], np.int32), v)[0] == M.ERR_INVALID_ARG
    assert _create_csr(2, 2, rp, ci, np.array([1.0, np.nan]))[0] == M.ERR_INVALID_ARG
    assert M.load().mbpcg_last_error(None)


def test_create_dense_rejects_bad_sizes():
    L = M.load()
    a = np.eye(3)
    h = C.c_void_p()
    assert L.mbpcg_create_dense(C.byref(h), 3, a.ctypes.data, 2, M.MEM_HOST, None) == M.ERR_INVALID_ARG
    assert L.mbpcg_create_dense(C.byref(h), 0, a.ctypes.data, 3, M.MEM_HOST, None) == M.ERR_INVALID_ARG
    assert L.mbpcg_create_dense(C.byref(h), 3, None, 3, M.MEM_HOST, None) == M.ERR_INVALID_ARG


def test_solve_rejects_null_context_and_bad_params():
    L = M.load()
    b = np.ones(4)
    x = np.zeros(4)
    p = M.default_params()
    assert L.mbpcg_solve(None, b.ctypes.data, x.ctypes.data, M.MEM_HOST, C.byref(p), None) == \
        M.ERR_INVALID_ARG
    assert L.mbpcg_cg_solve(None, b.ctypes.data, x.ctypes.data, M.MEM_HOST, C.byref(p), None) == \
        M.ERR_INVALID_ARG


def test_batch_validation():
    L = M.load()
    rp = np.array([0, 1], np.int32)
    ci = np.array([0], np.int32)
    v = np.array([2.0])
    b = np.ones(1)
    x = np.zeros(1)
    p = M.default_params()
    sysv = (M.System * 1)(M.System(1, 1, rp.ctypes.data, ci.ctypes.data, v.ctypes.data,
                                   b.ctypes.data, x.ctypes.data, 9))
    assert L.mbpcg_solve_batch(1, sysv, C.byref(p), None, M.MEM_HOST, None) == M.ERR_UNSUPPORTED
    sysv[0].s = 0
    assert L.mbpcg_solve_batch(1, sysv, C.byref(p), None, M.MEM_HOST, None) == M.ERR_INVALID_ARG
    assert L.mbpcg_solve_batch(0, sysv, C.byref(p), None, M.MEM_HOST, None) == M.ERR_INVALID_ARG
    # the batched kernel has no block-Jacobi path (checked before any HIP call)
    sysv[0].s = 1
    p.precond = M.PRECOND_BLOCK_JACOBI
    assert L.mbpcg_solve_batch(1, sysv, C.byref(p), None, M.MEM_HOST, None) == M.ERR_UNSUPPORTED
    # an unknown preconditioner is an invalid argument, not a silent "none"
    p.precond = 7
    assert L.mbpcg_solve_batch(1, sysv, C.byref(p), None, M.MEM_HOST, None) == M.ERR_INVALID_ARG
    # unequal tolerances and low-precision refinement are single-system features
    p = M.default_params()
    p.tol_initial = 1e-6
    assert L.mbpcg_solve_batch(1, sysv, C.byref(p), None, M.MEM_HOST, None) == M.ERR_UNSUPPORTED
    p = M.default_params()
    p.precision = M.FP32_IR
    assert L.mbpcg_solve_batch(1, sysv, C.byref(p), None, M.MEM_HOST, None) == M.ERR_UNSUPPORTED
    p = M.default_params()
    p.max_iter = 2 ** 31
    assert L.mbpcg_solve_batch(1, sysv, C.byref(p), None, M.MEM_HOST, None) == M.ERR_INVALID_ARG
    p = M.default_params()
    p.tau = float("nan")
    assert L.mbpcg_solve_batch(1, sysv, C.byref(p), None, M.MEM_HOST, None) == M.ERR_INVALID_ARG


def test_batch_context_validation():
    L = M.load()
    rp = np.array([0, 1], np.int32)
    ci = np.array([0], np.int32)
    v = np.array([2.0])
    b = np.ones(1)
    x = np.zeros(1)
    h = C.c_void_p()
    sysv = (M.System * 1)(M.System(1, 1, rp.ctypes.data, ci.ctypes.data, v.ctypes.data,
                                   b.ctypes.data, x.ctypes.data, 9))
    assert L.mbpcg_batch_create(C.byref(h), 1, sysv, M.MEM_HOST, None) == M.ERR_UNSUPPORTED
    sysv[0].s = 1
    sysv[0].rowptr = None
    assert L.mbpcg_batch_create(C.byref(h), 1, sysv, M.MEM_HOST, None) == M.ERR_INVALID_ARG
    assert L.mbpcg_batch_create(None, 1, sysv, M.MEM_HOST, None) == M.ERR_INVALID_ARG
    p = M.default_params()
    assert L.mbpcg_batch_solve(None, C.byref(p), None, None) == M.ERR_INVALID_ARG
    t = M.BatchTuning()
    assert L.mbpcg_batch_autotune(None, C.byref(p), C.byref(t)) == M.ERR_INVALID_ARG
    L.mbpcg_batch_destroy(None)


def test_stream_copy_rejects_null():
    assert M.load().mbpcg_stream_copy(None, None, 8, None) == M.ERR_INVALID_ARG


def test_no_cpu_fallback_when_library_missing(monkeypatch, tmp_path):
    monkeypatch.setattr(M, "_lib", None)
    monkeypatch.setattr(M, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        M.load()


def test_tile_shapes_listing():
    for s in (1, 2, 4, 8, 16, 32):
        shapes = M.tile_shapes(s)
        assert len(shapes) >= 3
        for sh in shapes:
            V, L = sh["cols_per_lane"], sh["lanes_per_row"]
            assert V in (1, 2, 4) and s % V == 0
            slots = L * V // s
            assert slots in (1, 2) and slots * s == L * V
            assert sh["tile_rows"] in (32, 64, 128, 256)
            assert sh["loads_in_flight"] in (4, 8)
            assert sh["waves_per_simd"] in (0, 5, 6, 8)
    L = M.load()
    cnt = C.c_int32()
    assert L.mbpcg_tile_shapes(3, None, 0, C.byref(cnt)) == M.ERR_UNSUPPORTED
    assert L.mbpcg_tile_shapes(0, None, 0, C.byref(cnt)) == M.ERR_INVALID_ARG
    assert L.mbpcg_set_tile_shape(None, 4, None) == M.ERR_INVALID_ARG

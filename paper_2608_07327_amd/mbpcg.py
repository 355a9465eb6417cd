"""Python binding of the mbpcg C ABI (include/mbpcg.h).

Argument marshalling only: every step of a solve runs in the HIP library.
PyTorch supplies device memory (CUDA/HIP tensors) and the stream; numpy
arrays are passed as host memory.  The library must be built in-tree
(``python -m paper_2608_07327_amd.build``); there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmbpcg.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "mbpcg.h")

OK, NOT_CONVERGED = 0, 1
ERR_INVALID_ARG, ERR_NOT_SPD, ERR_BREAKDOWN, ERR_NONFINITE = -1, -2, -3, -4
ERR_HIP, ERR_OOM, ERR_UNSUPPORTED = -5, -6, -7
PRECOND_NONE, PRECOND_JACOBI, PRECOND_BLOCK_JACOBI = 0, 1, 2
FP64, FP32_IR, BF16_IR = 0, 1, 2
MEM_HOST, MEM_DEVICE = 0, 1

EXPORTS = ("mbpcg_autotune", "mbpcg_default_params", "mbpcg_create_csr", "mbpcg_create_dense", "mbpcg_solve",
           "mbpcg_cg_solve", "mbpcg_block_product", "mbpcg_block_product_noalloc",
           "mbpcg_time_block_product",
           "mbpcg_solve_batch", "mbpcg_batch_create", "mbpcg_batch_solve", "mbpcg_batch_autotune",
           "mbpcg_batch_destroy", "mbpcg_stream_copy", "mbpcg_destroy", "mbpcg_status_str",
           "mbpcg_last_error", "mbpcg_tile_shapes", "mbpcg_set_tile_shape")


class Params(C.Structure):
    _fields_ = [("s", C.c_int32), ("tol", C.c_double), ("tol_initial", C.c_double),
                ("max_iter", C.c_int64), ("precond", C.c_int), ("seed", C.c_uint64),
                ("U", C.c_void_p), ("tau", C.c_double), ("precision", C.c_int),
                ("ir_tol", C.c_double), ("inner_tol", C.c_double), ("max_outer", C.c_int32),
                ("history", C.c_void_p), ("poll_every", C.c_int32), ("profile", C.c_int32),
                ("block_size", C.c_int32), ("X_out", C.c_void_p)]


class Info(C.Structure):
    _fields_ = [("iterations", C.c_int64), ("outer_iterations", C.c_int64),
                ("best_column", C.c_int32), ("final_width", C.c_int32),
                ("deflations", C.c_int32), ("used_fallback", C.c_int32),
                ("rel_res_best_basis", C.c_double), ("rel_res_ls", C.c_double),
                ("rel_res_true", C.c_double), ("ms_total", C.c_double),
                ("ms_per_iter", C.c_double), ("ms_spmm", C.c_double),
                ("spmm_launches", C.c_int64), ("ms_phase", C.c_double * 8),
                ("status", C.c_int32), ("reserved", C.c_int32)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_ if f != "ms_phase"}
        d["ms_phase"] = list(self.ms_phase)
        return d


class System(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("rowptr", C.c_void_p),
                ("colind", C.c_void_p), ("vals", C.c_void_p), ("b", C.c_void_p),
                ("x", C.c_void_p), ("s", C.c_int32)]


class TileShape(C.Structure):
    _fields_ = [("tile_rows", C.c_int32), ("lanes_per_row", C.c_int32),
                ("cols_per_lane", C.c_int32), ("loads_in_flight", C.c_int32),
                ("workgroups", C.c_int32), ("waves_per_simd", C.c_int32), ("ms", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class BatchTuning(C.Structure):
    _fields_ = [("workgroups", C.c_int32), ("classes", C.c_int32),
                ("two_slot_classes", C.c_int32), ("trials", C.c_int32), ("ms", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class MbpcgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"mbpcg status {status}: {msg}")
        self.status = status


_lib = None


def load():
    """Load the in-tree library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2608_07327_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, i64, i32 = C.c_void_p, C.c_int64, C.c_int32
    L.mbpcg_default_params.argtypes = [C.POINTER(Params)]
    L.mbpcg_default_params.restype = None
    L.mbpcg_create_csr.argtypes = [C.POINTER(vp), i64, i64, vp, vp, vp, C.c_int, vp]
    L.mbpcg_create_dense.argtypes = [C.POINTER(vp), i64, vp, i64, C.c_int, vp]
    L.mbpcg_solve.argtypes = [vp, vp, vp, C.c_int, C.POINTER(Params), C.POINTER(Info)]
    L.mbpcg_cg_solve.argtypes = [vp, vp, vp, C.c_int, C.POINTER(Params), C.POINTER(Info)]
    L.mbpcg_block_product.argtypes = [vp, i32, C.c_int, vp, vp, vp]
    L.mbpcg_block_product_noalloc.argtypes = [vp, i32, C.c_int, vp, vp, vp]
    L.mbpcg_time_block_product.argtypes = [vp, i32, i32, vp, vp, C.POINTER(C.c_double)]
    L.mbpcg_solve_batch.argtypes = [i32, C.POINTER(System), C.POINTER(Params), C.POINTER(Info),
                                    C.c_int, vp]
    L.mbpcg_stream_copy.argtypes = [vp, vp, i64, vp]
    L.mbpcg_batch_create.argtypes = [C.POINTER(vp), i32, C.POINTER(System), C.c_int, vp]
    L.mbpcg_batch_solve.argtypes = [vp, C.POINTER(Params), C.POINTER(Info), vp]
    L.mbpcg_batch_autotune.argtypes = [vp, C.POINTER(Params), C.POINTER(BatchTuning)]
    L.mbpcg_batch_destroy.argtypes = [vp]
    L.mbpcg_batch_destroy.restype = None
    L.mbpcg_autotune.argtypes = [vp, i32, C.POINTER(TileShape)]
    L.mbpcg_tile_shapes.argtypes = [i32, C.POINTER(TileShape), i32, C.POINTER(i32)]
    L.mbpcg_set_tile_shape.argtypes = [vp, i32, C.POINTER(TileShape)]
    L.mbpcg_destroy.argtypes = [vp]
    L.mbpcg_destroy.restype = None
    L.mbpcg_status_str.argtypes = [C.c_int]
    L.mbpcg_status_str.restype = C.c_char_p
    L.mbpcg_last_error.argtypes = [vp]
    L.mbpcg_last_error.restype = C.c_char_p
    for f in ("mbpcg_create_csr", "mbpcg_create_dense", "mbpcg_solve", "mbpcg_cg_solve",
              "mbpcg_block_product", "mbpcg_block_product_noalloc", "mbpcg_time_block_product",
              "mbpcg_solve_batch", "mbpcg_batch_create", "mbpcg_batch_solve", "mbpcg_batch_autotune",
              "mbpcg_stream_copy", "mbpcg_autotune", "mbpcg_tile_shapes", "mbpcg_set_tile_shape"):
        getattr(L, f).restype = C.c_int
    _lib = L
    return L


def status_str(st: int) -> str:
    return load().mbpcg_status_str(st).decode()


def default_params(**kw) -> Params:
    p = Params()
    load().mbpcg_default_params(C.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise TypeError(f"unknown parameter {k}")
        setattr(p, k, v)
    return p


def _is_torch(a):
    return type(a).__module__.startswith("torch")


def _ptr_mem(a):
    """(pointer, mem kind) of a torch tensor or numpy array (kept alive by the caller)."""
    if a is None:
        return None, MEM_HOST
    if _is_torch(a):
        if a.is_cuda:
            return a.data_ptr(), MEM_DEVICE
        return a.data_ptr(), MEM_HOST
    return a.ctypes.data, MEM_HOST


def _stream_ptr(stream):
    if stream is not None:
        return int(stream)
    try:
        import torch
        if torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
    except Exception:
        pass
    return 0


def _check(st, ctx=None, allow=(OK, NOT_CONVERGED)):
    if st in allow:
        return st
    msg = load().mbpcg_last_error(ctx).decode() if ctx is not None or st != 0 else ""
    raise MbpcgError(st, f"{status_str(st)}: {msg}")


class Solver:
    """A context holding a device copy of A (CSR or dense, FP64)."""

    def __init__(self, handle, n, dense):
        self._h = handle
        self.n = n
        self.dense = dense

    # ---------------------------------------------------------------- create
    @classmethod
    def from_csr(cls, n, rowptr, colind, vals, stream=None):
        L = load()
        keep = []
        if not _is_torch(rowptr):
            rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
            colind = np.ascontiguousarray(colind, dtype=np.int32)
            vals = np.ascontiguousarray(vals, dtype=np.float64)
        keep += [rowptr, colind, vals]
        pr, mem = _ptr_mem(rowptr)
        pc, _ = _ptr_mem(colind)
        pv, _ = _ptr_mem(vals)
        nnz = int(vals.numel() if _is_torch(vals) else vals.size)
        h = C.c_void_p()
        st = L.mbpcg_create_csr(C.byref(h), int(n), nnz, pr, pc, pv, mem, _stream_ptr(stream))
        _check(st, None, allow=(OK,))
        return cls(h, int(n), False)

    @classmethod
    def from_matrix(cls, A, stream=None):
        """A: a workloads.CSR, a scipy CSR matrix, or a dense square array (column-major
        storage is taken from a numpy array's memory order; symmetric inputs are the same
        either way)."""
        if hasattr(A, "rowptr"):
            return cls.from_csr(A.n, A.rowptr, A.colind, A.vals, stream)
        if hasattr(A, "indptr"):
            return cls.from_csr(A.shape[0], A.indptr, A.indices, A.data, stream)
        return cls.from_dense(A, stream)

    @classmethod
    def from_dense(cls, A, stream=None):
        L = load()
        if _is_torch(A):
            n = int(A.shape[0])
            # column-major element (r, c) at c*lda + r: a row-major torch tensor of A^T
            At = A.t().contiguous() if not A.t().is_contiguous() else A.t()
            p, mem = At.data_ptr(), (MEM_DEVICE if At.is_cuda else MEM_HOST)
            keep = At
        else:
            a = np.asfortranarray(A, dtype=np.float64)
            n = a.shape[0]
            p, mem = a.ctypes.data, MEM_HOST
            keep = a
        h = C.c_void_p()
        st = L.mbpcg_create_dense(C.byref(h), n, p, n, mem, _stream_ptr(stream))
        del keep
        _check(st, None, allow=(OK,))
        return cls(h, n, True)

    def close(self):
        if self._h:
            load().mbpcg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # ----------------------------------------------------------------- solve
    def _solve(self, fn, b, x, params, history):
        L = load()
        pb, mem = _ptr_mem(b)
        if x is None:
            if _is_torch(b):
                import torch
                x = torch.empty_like(b)
            else:
                x = np.zeros(self.n)
        px, memx = _ptr_mem(x)
        if memx != mem:
            raise ValueError("b and x must both be host or both be device memory")
        hist = None
        if history:
            hist = np.full(int(params.max_iter), np.nan)
            params.history = hist.ctypes.data
        info = Info()
        st = getattr(L, fn)(self._h, pb, px, mem, C.byref(params), C.byref(info))
        info.status = st
        _check(st, self._h, allow=(OK, NOT_CONVERGED, ERR_NOT_SPD, ERR_BREAKDOWN, ERR_NONFINITE))
        d = info.as_dict()
        d["status"] = st
        if history:
            d["history"] = hist[: int(d["iterations"])].copy()
        return x, d

    def solve(self, b, x=None, history=False, **kw):
        """MBPCG (Algorithm 1).  kw: fields of Params (s, tol, seed, precond, U, ...);
        X_out: an optional n x s array (same memory kind as b) that receives the
        block iterate X~ + X0 at exit (scaled space)."""
        U = kw.pop("U", None)
        X_out = kw.pop("X_out", None)
        p = default_params(**kw)
        if U is not None:
            p.U, _ = _ptr_mem(U)
        if X_out is not None:
            p.X_out, _ = _ptr_mem(X_out)
        return self._solve("mbpcg_solve", b, x, p, history)

    def cg_solve(self, b, x=None, history=False, **kw):
        """Chronopoulos-Gear CG from x0 = 0 on the same scaled system."""
        p = default_params(**kw)
        return self._solve("mbpcg_cg_solve", b, x, p, history)

    def block_product(self, P, Q, Cmat, s, precond=PRECOND_JACOBI):
        """Q = A~ P and lower triangle of C = P^T Q (device tensors)."""
        st = load().mbpcg_block_product(self._h, int(s), int(precond), P.data_ptr(), Q.data_ptr(),
                                        Cmat.data_ptr())
        _check(st, self._h, allow=(OK,))

    def block_product_noalloc(self, P, Q, Cmat, s, precond=PRECOND_JACOBI):
        """block_product without any allocation (fixed per-GPU scratch array;
        CSR contexts only; overlapping calls on one GPU race)."""
        st = load().mbpcg_block_product_noalloc(self._h, int(s), int(precond), P.data_ptr(),
                                                Q.data_ptr(), Cmat.data_ptr())
        _check(st, self._h, allow=(OK,))

    def autotune(self, s):
        """Time the block-product shapes for width s; later solves use the best.
        Returns the chosen shape as a dict (tile_rows, lanes_per_row,
        cols_per_lane, loads_in_flight, workgroups, ms)."""
        t = TileShape()
        st = load().mbpcg_autotune(self._h, int(s), C.byref(t))
        _check(st, self._h, allow=(OK,))
        return t.as_dict()

    def set_tile_shape(self, s, shape):
        """Fix the block-product shape for width s (a dict as returned by
        tile_shapes() or autotune(); workgroups <= 0 means the default grid)."""
        t = TileShape(**{k: int(v) for k, v in shape.items() if k != "ms"})
        st = load().mbpcg_set_tile_shape(self._h, int(s), C.byref(t))
        _check(st, self._h, allow=(OK,))

    def time_block_product(self, P, Q, s, reps=20):
        ms = C.c_double()
        st = load().mbpcg_time_block_product(self._h, int(s), int(reps), P.data_ptr(),
                                             Q.data_ptr(), C.byref(ms))
        _check(st, self._h, allow=(OK,))
        return ms.value


def _systems(systems):
    arr = (System * len(systems))()
    mem = None
    for i, y in enumerate(systems):
        pr, m = _ptr_mem(y["rowptr"])
        mem = m if mem is None else mem
        if m != mem:
            raise ValueError("all systems must be in the same memory kind")
        vals = y["vals"]
        nnz = int(vals.numel() if _is_torch(vals) else vals.size)
        arr[i] = System(int(y["n"]), nnz, pr, _ptr_mem(y["colind"])[0], _ptr_mem(vals)[0],
                        _ptr_mem(y["b"])[0], _ptr_mem(y["x"])[0], int(y["s"]))
    return arr, mem


class Batch:
    """A batch context: the systems (dicts as for solve_batch) uploaded once,
    the persistent kernel's graph replayed by every solve; x is written
    through the systems' "x" arrays.  The arrays must outlive the context."""

    def __init__(self, systems, stream=None):
        L = load()
        self._keep = systems
        arr, mem = _systems(systems)
        h = C.c_void_p()
        st = L.mbpcg_batch_create(C.byref(h), len(systems), arr, mem, _stream_ptr(stream))
        _check(st, None, allow=(OK,))
        self._h = h
        self.n = len(systems)

    def solve(self, stream=None, **kw):
        """Returns (status, infos)."""
        p = default_params(**kw)
        infos = (Info * self.n)()
        st = load().mbpcg_batch_solve(self._h, C.byref(p), infos, _stream_ptr(stream))
        _check(st, None, allow=(OK, NOT_CONVERGED, ERR_NOT_SPD, ERR_BREAKDOWN, ERR_NONFINITE))
        return st, [infos[i].as_dict() for i in range(self.n)]

    def autotune(self, **kw):
        """Timed trials of the batched kernel's lane groups per row and grid;
        returns the choice as a dict (overwrites x)."""
        p = default_params(**kw)
        t = BatchTuning()
        st = load().mbpcg_batch_autotune(self._h, C.byref(p), C.byref(t))
        _check(st, None, allow=(OK,))
        return t.as_dict()

    def close(self):
        if getattr(self, "_h", None):
            load().mbpcg_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def solve_batch(systems, **kw):
    """Solve independent sparse systems together (one persistent kernel).

    systems: list of dicts with keys n, rowptr, colind, vals, b, x, s -- all
    torch device tensors, or all numpy arrays.  Returns (status, infos)."""
    L = load()
    arr = (System * len(systems))()
    mem = None
    for i, y in enumerate(systems):
        pr, m = _ptr_mem(y["rowptr"])
        mem = m if mem is None else mem
        if m != mem:
            raise ValueError("all systems must be in the same memory kind")
        vals = y["vals"]
        nnz = int(vals.numel() if _is_torch(vals) else vals.size)
        arr[i] = System(int(y["n"]), nnz, pr, _ptr_mem(y["colind"])[0], _ptr_mem(vals)[0],
                        _ptr_mem(y["b"])[0], _ptr_mem(y["x"])[0], int(y["s"]))
    p = default_params(**kw)
    infos = (Info * len(systems))()
    st = L.mbpcg_solve_batch(len(systems), arr, C.byref(p), infos, mem, _stream_ptr(None))
    _check(st, None, allow=(OK, NOT_CONVERGED, ERR_NOT_SPD, ERR_BREAKDOWN, ERR_NONFINITE))
    return st, [infos[i].as_dict() for i in range(len(systems))]


def tile_shapes(s):
    """Compiled block-product tile shapes for width s (list of dicts)."""
    cnt = C.c_int32()
    buf = (TileShape * 64)()
    st = load().mbpcg_tile_shapes(int(s), buf, 64, C.byref(cnt))
    _check(st, allow=(OK,))
    return [buf[i].as_dict() for i in range(min(cnt.value, 64))]


def stream_copy(dst, src, nbytes, stream=None):
    st = load().mbpcg_stream_copy(dst.data_ptr(), src.data_ptr(), int(nbytes), _stream_ptr(stream))
    _check(st, None, allow=(OK,))

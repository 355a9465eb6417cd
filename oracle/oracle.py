"""ctypes shim over the C oracle (``mbpcg_oracle.c``).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline of the benchmark load this module.  It never touches the GPU
library and the GPU library never touches it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mbpcg_oracle.c")
LIB = os.path.join(HERE, "libmbpcg_oracle.so")
# The same source compiled with multiply-adds contracted to fused
# multiply-adds: a third rounding of the same arithmetic, used only to
# measure the method's rounding noise (see set_variant).
LIB_FMA = os.path.join(HERE, "libmbpcg_oracle_fma.so")

_FLAGS = {LIB: ["-ffp-contract=off"], LIB_FMA: ["-ffp-contract=fast", "-mfma"]}


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no fast-math; no FMA contraction in
    the reference build, contraction in the noise-measurement build)."""
    hdr = os.path.join(HERE, "mbpcg_oracle.h")
    for lib_path, flags in _FLAGS.items():
        if force or not os.path.exists(lib_path) or os.path.getmtime(lib_path) < max(
                os.path.getmtime(SRC), os.path.getmtime(hdr)):
            tmp = lib_path + ".tmp"
            subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", *flags,
                                   "-Wall", "-o", tmp, SRC, "-lm"])
            os.replace(tmp, lib_path)
    return LIB


class OrMatrix(C.Structure):
    _fields_ = [("n", C.c_int64), ("dense", C.c_int), ("rowptr", C.c_void_p),
                ("colind", C.c_void_p), ("vals", C.c_void_p), ("a", C.c_void_p),
                ("lda", C.c_int64), ("lo", C.c_int)]


class OrParams(C.Structure):
    _fields_ = [("s", C.c_int), ("tol", C.c_double), ("tol_initial", C.c_double),
                ("max_iter", C.c_int64), ("jacobi", C.c_int), ("seed", C.c_uint64),
                ("U", C.c_void_p), ("tau", C.c_double), ("ls_scaled", C.c_int),
                ("history", C.c_void_p), ("X_out", C.c_void_p), ("R_out", C.c_void_p),
                ("prop1_gap", C.c_void_p), ("check_true", C.c_int), ("bj_block", C.c_int)]


class OrInfo(C.Structure):
    _fields_ = [("status", C.c_int), ("iterations", C.c_int64), ("best_column", C.c_int),
                ("final_width", C.c_int), ("deflations", C.c_int), ("used_fallback", C.c_int),
                ("rel_res_best", C.c_double), ("rel_res_ls", C.c_double),
                ("rel_res_true", C.c_double), ("seconds", C.c_double),
                ("seconds_setup", C.c_double), ("ls_kept", C.c_int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_libs = {}
_variant = "seq"


def _load(path):
    L = C.CDLL(path)
    vp, i64, dbl = C.c_void_p, C.c_int64, C.c_double
    L.or_set_summation.argtypes = [C.c_int]
    L.or_splitmix64.argtypes = [C.c_uint64, C.c_uint64]
    L.or_splitmix64.restype = C.c_uint64
    L.or_uniform_block.argtypes = [C.c_uint64, i64, C.c_int, vp]
    L.or_matmul_block.argtypes = [vp, C.c_int, vp, vp]
    L.or_round_bf16.argtypes = [dbl]
    L.or_round_bf16.restype = dbl
    L.or_gram.argtypes = [i64, C.c_int, vp, C.c_int, vp, vp]
    L.or_cholesky.argtypes = [C.c_int, vp, vp]
    L.or_spd_inverse.argtypes = [C.c_int, vp, vp]
    L.or_cholqr_deflate.argtypes = [i64, C.c_int, vp, dbl, vp, vp, vp]
    L.or_cholqr_deflate_prec.argtypes = [i64, C.c_int, vp, vp, dbl, vp, vp, vp, vp]
    L.or_block_jacobi_apply.argtypes = [vp, C.c_int, C.c_int, C.c_int, vp, vp, vp]
    L.or_lstsq.argtypes = [i64, C.c_int, vp, vp, vp]
    L.or_mbpcg_solve.argtypes = [vp, vp, vp, vp, vp]
    L.or_hs_cg.argtypes = [vp, vp, vp, dbl, i64, C.c_int, C.c_int, vp, vp, vp]
    L.or_cg_cg.argtypes = [vp, vp, vp, dbl, i64, C.c_int, C.c_int, vp, vp, vp]
    return L


def lib():
    """The oracle library of the current variant (the reference build unless
    set_variant chose the fused multiply-add build)."""
    if not _libs:
        build()
        _libs["ref"] = _load(LIB)
        _libs["fma"] = _load(LIB_FMA)
    return _libs["fma" if _variant == "fma" else "ref"]


VARIANTS = ("seq", "pairwise", "fma")


def set_variant(v: str):
    """Rounding variant of every following call: "seq" (the reference:
    sequential sums, every product and sum rounded separately), "pairwise"
    (the same with blocked-pairwise sums over the n rows and the dense
    product's n columns), or "fma" (sequential sums with multiply-adds
    contracted to fused multiply-adds).  The three runs of one input measure
    how much the method moves under a change of rounding alone."""
    global _variant
    if v not in VARIANTS:
        raise ValueError(v)
    _variant = v
    lib()
    for L in _libs.values():
        L.or_set_summation(1 if v == "pairwise" else 0)


def _p(a):
    return None if a is None else a.ctypes.data


LO_FP64, LO_FP32, LO_BF16 = 0, 1, 2
OR_OK, OR_NOT_CONVERGED, OR_ERR_NOT_SPD, OR_ERR_BREAKDOWN, OR_ERR_NONFINITE = 0, 1, -2, -3, -4


class Matrix:
    """Keeps the numpy arrays alive behind an OrMatrix.  lo (dense only)
    selects low-precision products: LO_FP32 or LO_BF16."""

    def __init__(self, A, lo=LO_FP64):
        if isinstance(A, np.ndarray):
            self.a = np.asfortranarray(A, dtype=np.float64)
            self.s = OrMatrix(A.shape[0], 1, None, None, None, self.a.ctypes.data, A.shape[0],
                              int(lo))
        else:
            self.rowptr = np.ascontiguousarray(A.rowptr, dtype=np.int32)
            self.colind = np.ascontiguousarray(A.colind, dtype=np.int32)
            self.vals = np.ascontiguousarray(A.vals, dtype=np.float64)
            self.s = OrMatrix(A.n, 0, self.rowptr.ctypes.data, self.colind.ctypes.data,
                              self.vals.ctypes.data, None, 0, 0)
        self.n = int(self.s.n)


def set_summation(mode: int):
    """0: the reference variant, 1: blocked-pairwise sums (set_variant)."""
    set_variant("pairwise" if int(mode) == 1 else "seq")


def splitmix64(seed: int, k: int) -> int:
    return int(lib().or_splitmix64(seed, k))


def uniform_block(seed: int, n: int, s: int) -> np.ndarray:
    U = np.empty((n, s))
    lib().or_uniform_block(seed, n, s, U.ctypes.data)
    return U


def matmul_block(A, X):
    M = A if isinstance(A, Matrix) else Matrix(A)
    X = np.ascontiguousarray(X, dtype=np.float64)
    k = 1 if X.ndim == 1 else X.shape[1]
    Y = np.empty((M.n, k))
    lib().or_matmul_block(C.byref(M.s), k, X.ctypes.data, Y.ctypes.data)
    return Y.reshape(X.shape)


def gram(X, Y):
    X = np.ascontiguousarray(X, dtype=np.float64)
    Y = np.ascontiguousarray(Y, dtype=np.float64)
    Cm = np.empty((X.shape[1], Y.shape[1]))
    lib().or_gram(X.shape[0], X.shape[1], X.ctypes.data, Y.shape[1], Y.ctypes.data, Cm.ctypes.data)
    return Cm


def cholesky(Cm):
    Cm = np.ascontiguousarray(Cm, dtype=np.float64)
    L = np.empty_like(Cm)
    rc = lib().or_cholesky(Cm.shape[0], Cm.ctypes.data, L.ctypes.data)
    return rc, L


def spd_inverse(L):
    L = np.ascontiguousarray(L, dtype=np.float64)
    Xi = np.empty_like(L)
    lib().or_spd_inverse(L.shape[0], L.ctypes.data, Xi.ctypes.data)
    return Xi


def cholqr_deflate(V, tau=1e-12):
    V = np.ascontiguousarray(V, dtype=np.float64)
    n, m = V.shape
    W = np.empty(n * m)
    Z = np.empty(m * m)
    keep = np.zeros(m, dtype=np.int32)
    k = lib().or_cholqr_deflate(n, m, V.ctypes.data, tau, W.ctypes.data, Z.ctypes.data,
                                keep.ctypes.data)
    return W[: n * k].reshape(n, k), Z[: k * m].reshape(k, m), keep.astype(bool)


def cholqr_deflate_prec(V, Y, tau=1e-12):
    """Cholesky QR in the M^-1 inner product (Y = M^-1 V): returns W, M^-1 W,
    Z and the kept-column flags."""
    V = np.ascontiguousarray(V, dtype=np.float64)
    Y = np.ascontiguousarray(Y, dtype=np.float64)
    n, m = V.shape
    W = np.empty(n * m)
    MW = np.empty(n * m)
    Z = np.empty(m * m)
    keep = np.zeros(m, dtype=np.int32)
    k = lib().or_cholqr_deflate_prec(n, m, V.ctypes.data, Y.ctypes.data, tau, W.ctypes.data,
                                     MW.ctypes.data, Z.ctypes.data, keep.ctypes.data)
    return (W[: n * k].reshape(n, k), MW[: n * k].reshape(n, k), Z[: k * m].reshape(k, m),
            keep.astype(bool))


def block_jacobi_apply(A, X, bs, jacobi=True):
    """M^-1 X for the block-Jacobi preconditioner (blocks of bs rows) of the
    matrix as a solve scales it; returns (Y, status)."""
    M = A if isinstance(A, Matrix) else Matrix(A)
    X = np.ascontiguousarray(X, dtype=np.float64)
    X2 = X.reshape(M.n, -1)
    Y = np.zeros_like(X2)
    st = C.c_int(0)
    lib().or_block_jacobi_apply(C.byref(M.s), int(bool(jacobi)), int(bs), X2.shape[1],
                                X2.ctypes.data, Y.ctypes.data, C.byref(st))
    return Y.reshape(X.shape), st.value


def lstsq(B, b):
    B = np.ascontiguousarray(B, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    c = np.zeros(B.shape[1])
    rc = lib().or_lstsq(B.shape[0], B.shape[1], B.ctypes.data, b.ctypes.data, c.ctypes.data)
    return rc, c


STATUS = {0: "OK", 1: "NOT_CONVERGED", -2: "NOT_SPD", -3: "BREAKDOWN", -4: "NONFINITE"}


def mbpcg_solve(A, b, s, tol=1e-8, tol_initial=0.0, max_iter=100000, jacobi=True, seed=0,
                U=None, tau=1e-12, ls_scaled=False, want_history=False, want_X=False,
                want_prop1=False, check_true=True, block_jacobi=0):
    """Run Algorithm 1 on the CPU.  Returns (x, info dict, extras dict).
    check_true: an accepted least-squares combination whose true residual
    is not below tol gives way to the best column if that column's true
    residual is lower (used_fallback = 1).  block_jacobi >= 2: the
    preconditioned form with the block-Jacobi preconditioner of that block
    size on the (scaled) matrix."""
    M = A if isinstance(A, Matrix) else Matrix(A)
    n = M.n
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros(n)
    hist = np.full(max_iter, np.nan) if want_history else None
    Xo = np.zeros((n, s)) if want_X else None
    Ro = np.zeros((n, s)) if want_X else None
    gap = np.full(max_iter, np.nan) if want_prop1 else None
    Uc = None if U is None else np.ascontiguousarray(U, dtype=np.float64)
    p = OrParams(s, tol, tol_initial, max_iter, int(bool(jacobi)), seed, _p(Uc), tau,
                 int(bool(ls_scaled)), _p(hist), _p(Xo), _p(Ro), _p(gap), int(bool(check_true)),
                 int(block_jacobi))
    info = OrInfo()
    lib().or_mbpcg_solve(C.byref(M.s), b.ctypes.data, C.byref(p), x.ctypes.data, C.byref(info))
    d = info.as_dict()
    it = int(d["iterations"])
    extra = {}
    if want_history:
        extra["history"] = hist[:it]
    if want_X:
        extra["X"] = Xo
        extra["R"] = Ro
    if want_prop1:
        extra["prop1_gap"] = gap[:it]
    return x, d, extra


def _cg(fn, A, b, x0, tol, max_iter, jacobi, want_history, block_jacobi=0):
    M = A if isinstance(A, Matrix) else Matrix(A)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros(M.n)
    hist = np.full(max_iter, np.nan) if want_history else None
    x0c = None if x0 is None else np.ascontiguousarray(x0, dtype=np.float64)
    info = OrInfo()
    fn(C.byref(M.s), b.ctypes.data, _p(x0c), tol, max_iter, int(bool(jacobi)), int(block_jacobi),
       x.ctypes.data, _p(hist), C.byref(info))
    d = info.as_dict()
    return x, d, (hist[: int(d["iterations"])] if want_history else None)


def hs_cg(A, b, x0=None, tol=1e-8, max_iter=100000, jacobi=True, want_history=False,
          block_jacobi=0):
    """Textbook (preconditioned, when block_jacobi >= 2) CG."""
    return _cg(lib().or_hs_cg, A, b, x0, tol, max_iter, jacobi, want_history, block_jacobi)


def cg_cg(A, b, x0=None, tol=1e-8, max_iter=100000, jacobi=True, want_history=False,
          block_jacobi=0):
    """Chronopoulos-Gear CG (preconditioned, when block_jacobi >= 2)."""
    return _cg(lib().or_cg_cg, A, b, x0, tol, max_iter, jacobi, want_history, block_jacobi)


def round_bf16(x: float) -> float:
    return float(lib().or_round_bf16(float(x)))


def ir_solve(A, b, s, lo, ir_tol=1e-10, inner_tol=5e-6, max_outer=50, seed=0, tau=1e-12):
    """Mixed-precision iterative refinement around Algorithm 1 (an extension;
    the paper runs FP64 only).  Dense A, no scaling.  x = 0, r = b; each
    outer step runs Algorithm 1 on the rounded operator (lo = LO_FP32 or
    LO_BF16: A and the blocks it multiplies rounded, products accumulated in
    FP32, the rest FP64) for A d = r, to the relative tolerance
    clamp(0.5 ir_tol / rel, inner_tol, 0.1) where rel = ||r|| / ||b||; then
    x += d and r = b - A x in FP64.  It stops when rel <= ir_tol, and takes
    the step back and stops when an outer step does not lower rel.  Inner
    solve k (from 1) uses seed + (k - 1) * 7919.  Returns (x, info)."""
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    Mlo = Matrix(A, lo=lo)
    bn = float(np.linalg.norm(b))
    x = np.zeros_like(b)
    info = {"outer_iterations": 0, "iterations": 0, "status": 0, "rel_res_true": 1.0,
            "inner_iterations": []}
    if bn == 0.0:
        info["rel_res_true"] = 0.0
        return x, info
    r = b.copy()
    rel = 1.0
    stalled = False
    for k in range(1, max_outer + 1):
        tol_k = min(0.1, max(inner_tol, 0.5 * ir_tol / rel))
        d, ii, _ = mbpcg_solve(Mlo, r, s, tol=tol_k, jacobi=False, seed=seed + (k - 1) * 7919,
                               tau=tau, check_true=False)
        info["iterations"] += ii["iterations"]
        info["inner_iterations"].append(ii["iterations"])
        info["outer_iterations"] = k
        if ii["status"] in (OR_ERR_NOT_SPD, OR_ERR_NONFINITE):
            break
        x_new = x + d
        r_new = b - A @ x_new
        rel_new = float(np.linalg.norm(r_new)) / bn
        if not rel_new < rel:
            stalled = True
            break
        x, r, rel = x_new, r_new, rel_new
        if rel <= ir_tol:
            break
    info["rel_res_true"] = rel
    info["status"] = 0 if rel <= ir_tol else 1
    info["stalled"] = stalled
    return x, info

"""Seeded synthetic inputs for the block-CG solver and for its CPU oracle.

This module builds problems only: matrices, right-hand sides and block
widths.  It holds none of the solver's arithmetic, imports neither the
native library nor the oracle, and is the one piece of code that the GPU
path and the oracle share.

Every generator draws from ``numpy.random.default_rng([260807327, tag])``
(PCG64) so that the same call gives the same bytes on any machine.

Workloads (the paper measures on SuiteSparse matrices and on dense
``M^T M`` systems, Sec. 5; neither is available offline, so these seeded
families stand in for them with the shapes and value distributions of the
headline configurations):

* ``poisson2d(64)``            2-D 5-point Dirichlet Poisson, n = 4096.
* ``diffusion3d(128)``         3-D 7-point variable-coefficient diffusion,
                                log-normal(sigma=1) cell coefficients,
                                harmonic-mean face weights, n = 2,097,152;
                                optionally with highly conducting cubic
                                inclusions (a few isolated small eigenvalues).
* ``dense_spd(8192)``          A = G G^T / n + 1e-3 I, G iid N(0,1) on a
                                2^-8 grid (the product is then exact).
* ``graph_laplacian_batch``    random-graph Laplacians (average degree 8)
                                plus 1e-2 I, n log-uniform in [1e3, 2e5].
* ``tiny_spd``                 A = Q diag(lambda) Q^T with a set condition
                                number, for finite-termination checks.
"""
from __future__ import annotations

import dataclasses
import numpy as np

SEED_BASE = 260807327

# configuration tags used as the second seed word
CFG_POISSON2D = 1
CFG_DIFFUSION3D = 2
CFG_DENSE = 3
CFG_DENSE_MIXED = 4
CFG_BATCH = 5


def _flat(tag):
    if isinstance(tag, (list, tuple)):
        out = []
        for t in tag:
            out.extend(_flat(t))
        return out
    return [int(tag)]


def rng_for(tag) -> np.random.Generator:
    """PCG64 stream for a (possibly nested) tuple of integer tags."""
    return np.random.default_rng([SEED_BASE, *_flat(tag)])


@dataclasses.dataclass
class CSR:
    n: int
    rowptr: np.ndarray  # int32, n+1
    colind: np.ndarray  # int32, nnz, ascending within each row
    vals: np.ndarray    # float64, nnz

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.vals, self.colind, self.rowptr), shape=(self.n, self.n))

    def to_dense(self) -> np.ndarray:
        a = np.zeros((self.n, self.n))
        rows = np.repeat(np.arange(self.n), np.diff(self.rowptr))
        a[rows, self.colind] = self.vals
        return a


def _stencil_csr(n: int, cols: np.ndarray, vals: np.ndarray, valid: np.ndarray) -> CSR:
    """Assemble CSR from an n x k table of candidate entries whose columns are
    already ascending along axis 1; ``valid`` masks the entries that exist."""
    counts = valid.sum(axis=1)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    colind = cols[valid].astype(np.int32)
    v = vals[valid].astype(np.float64)
    return CSR(n, rowptr.astype(np.int32), colind, v)


def poisson2d(m: int = 64) -> CSR:
    """Dirichlet 5-point Laplacian on an m x m grid, lexicographic (x fastest):
    diagonal 4, neighbours -1."""
    n = m * m
    idx = np.arange(n)
    x = idx % m
    y = idx // m
    offs = [(-m, y > 0), (-1, x > 0), (0, np.ones(n, bool)), (1, x < m - 1), (m, y < m - 1)]
    cols = np.stack([idx + o for o, _ in offs], axis=1)
    valid = np.stack([msk for _, msk in offs], axis=1)
    vals = np.full(cols.shape, -1.0)
    vals[:, 2] = 4.0
    return _stencil_csr(n, cols, vals, valid)


def diffusion3d(m: int = 128, sigma: float = 1.0, tag=CFG_DIFFUSION3D, inclusions: int = 0,
                contrast: float = 1e4, size: int = 4) -> CSR:
    """Cell-centred 7-point finite-volume diffusion on an m^3 grid with iid
    log-normal cell coefficients kappa_c = exp(sigma * g_c), g_c ~ N(0,1).

    Interior face weight: harmonic mean 2 / (1/kappa_c + 1/kappa_c').
    Dirichlet boundary face (half-cell distance): 2 kappa_c.
    A_cc = sum of the cell's face weights, A_cc' = -w(c, c').
    Lexicographic order with x fastest, so every row's columns ascend as
    (-z, -y, -x, self, +x, +y, +z).

    inclusions > 0: that many size^3 cubes of cells (corners drawn uniformly
    in [1, m - size - 1] per axis from a stream of their own, so the other
    coefficients do not change) have kappa multiplied by `contrast`.  Highly
    conducting inclusions give the scaled operator one small eigenvalue per
    inclusion, well separated from the rest of the spectrum: the case where
    CG needs many iterations and a block of s >= inclusions columns does
    not."""
    rng = rng_for(tag)
    n = m ** 3
    g = rng.standard_normal(n)
    kap = np.exp(sigma * g)
    idx = np.arange(n)
    x = idx % m
    y = (idx // m) % m
    z = idx // (m * m)
    if inclusions > 0:
        if not 1 <= size <= m - 2:
            raise ValueError("inclusion size must lie in [1, m - 2]")
        ri = rng_for((CFG_DIFFUSION3D, 77, m, inclusions, size))
        for _ in range(inclusions):
            c = ri.integers(1, m - size, 3)        # corner, in [1, m - size - 1]
            inside = ((x >= c[0]) & (x < c[0] + size) & (y >= c[1]) & (y < c[1] + size)
                      & (z >= c[2]) & (z < c[2] + size))
            kap[inside] *= contrast
    strides = [m * m, m, 1]
    coords = [z, y, x]
    cols = np.empty((n, 7), dtype=np.int64)
    vals = np.empty((n, 7))
    valid = np.ones((n, 7), dtype=bool)
    diag = np.zeros(n)
    inv = 1.0 / kap
    # lower neighbours: slots 0..2 = -z, -y, -x
    for slot, (st, cc) in enumerate(zip(strides, coords)):
        has = cc > 0
        nb = np.where(has, idx - st, idx)
        w = np.where(has, 2.0 / (inv + inv[nb]), 2.0 * kap)
        cols[:, slot] = nb
        vals[:, slot] = -w
        valid[:, slot] = has
        diag += w
    # upper neighbours: slots 4..6 = +x, +y, +z
    for slot, (st, cc) in zip((4, 5, 6), zip(strides[::-1], coords[::-1])):
        has = cc < m - 1
        nb = np.where(has, idx + st, idx)
        w = np.where(has, 2.0 / (inv + inv[nb]), 2.0 * kap)
        cols[:, slot] = nb
        vals[:, slot] = -w
        valid[:, slot] = has
        diag += w
    cols[:, 3] = idx
    vals[:, 3] = diag
    return _stencil_csr(n, cols, vals, valid)


def rhs(n: int, tag) -> np.ndarray:
    """b ~ N(0,1), iid, from its own seed stream."""
    return rng_for((tag, 7777)).standard_normal(n)


# G's entries are N(0,1) draws rounded to the grid 2^-8 (and clipped to
# [-8, 8], which no draw reaches in practice): every product of two entries is
# an integer multiple of 2^-16 below 2^6 in magnitude, so each entry of G G^T,
# a sum of at most 2^14 such products for n <= 16384, is an exact FP64 value
# whatever the order or blocking of the sum.  Any BLAS, on any host or GPU,
# then returns the same bytes for A.
DENSE_GRID = 256.0


def dense_factor(n: int, tag=CFG_DENSE) -> np.ndarray:
    """G (n x n) of the dense construction: iid N(0,1) on the 2^-8 grid."""
    if n > 16384:
        raise ValueError("dense_factor: the product is exact only for n <= 16384")
    g = rng_for(tag).standard_normal((n, n))
    np.rint(g * DENSE_GRID, out=g)
    np.clip(g, -8 * DENSE_GRID, 8 * DENSE_GRID, out=g)
    g /= DENSE_GRID
    return g


def _finish_dense(a, n: int, shift: float):
    """A = P / n + shift I from the exact product P = G G^T, lower triangle
    mirrored (A is bitwise symmetric; row- and column-major are the same
    bytes).  `a` is a numpy array or a torch tensor."""
    a /= n
    if isinstance(a, np.ndarray):
        a = np.tril(a)
        a = a + np.tril(a, -1).T
        a[np.diag_indices(n)] += shift
        return a
    a = a.tril()
    a = a + a.tril(-1).t()
    a.diagonal().add_(shift)
    return a


def dense_spd(n: int, tag=CFG_DENSE, shift: float = 1e-3) -> np.ndarray:
    """A = G G^T / n + shift I in FP64 with G iid N(0,1) on the 2^-8 grid
    (n x n); the product is exact, so the bytes do not depend on the BLAS."""
    g = dense_factor(n, tag)
    a = g @ g.T
    del g
    return np.ascontiguousarray(_finish_dense(a, n, shift))


def dense_spd_torch(n: int, tag=CFG_DENSE, shift: float = 1e-3, device="cuda:0"):
    """dense_spd with the n^3 product done by torch on `device` (input
    generation only); the same bytes as dense_spd because the product is
    exact."""
    import torch
    g = torch.as_tensor(dense_factor(n, tag), device=device)
    a = torch.mm(g, g.t().contiguous())
    del g
    return _finish_dense(a, n, shift).contiguous()


def tiny_spd(n: int, cond: float, tag) -> np.ndarray:
    """A = Q diag(lam) Q^T, Q from the QR of a Gaussian matrix, lam log-spaced
    in [1, cond]; mirrored to bitwise symmetry."""
    rng = rng_for(tag)
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.geomspace(1.0, cond, n)
    a = (q * lam) @ q.T
    a = np.tril(a)
    return a + np.tril(a, -1).T


def dense_to_csr(a: np.ndarray) -> CSR:
    n = a.shape[0]
    nz = a != 0.0
    counts = nz.sum(axis=1)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    rows, cols = np.nonzero(nz)
    return CSR(n, rowptr.astype(np.int32), cols.astype(np.int32), a[rows, cols].astype(np.float64))


def graph_laplacian(n: int, avg_degree: int, shift: float, rng: np.random.Generator) -> CSR:
    """Unit-weight Laplacian of a random simple graph with n*avg_degree/2
    distinct uniformly drawn edges (no self loops), plus shift*I."""
    m = n * avg_degree // 2
    keys = np.empty(0, dtype=np.int64)
    while keys.size < m:
        draw = int((m - keys.size) * 1.2) + 16
        u = rng.integers(0, n, draw)
        v = rng.integers(0, n, draw)
        ok = u != v
        lo = np.minimum(u[ok], v[ok]).astype(np.int64)
        hi = np.maximum(u[ok], v[ok]).astype(np.int64)
        cand = np.concatenate([keys, lo * n + hi])
        _, first = np.unique(cand, return_index=True)
        keys = cand[np.sort(first)]
    keys = keys[:m]
    lo = keys // n
    hi = keys % n
    rows = np.concatenate([lo, hi, np.arange(n)])
    cols = np.concatenate([hi, lo, np.arange(n)])
    deg = np.bincount(lo, minlength=n) + np.bincount(hi, minlength=n)
    vals = np.concatenate([-np.ones(2 * m), deg + shift])
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    counts = np.bincount(rows, minlength=n)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    return CSR(n, rowptr.astype(np.int32), cols.astype(np.int32), vals.astype(np.float64))


@dataclasses.dataclass
class BatchSystem:
    A: CSR
    b: np.ndarray
    s: int


def graph_laplacian_batch(count: int = 512, n_lo: float = 1e3, n_hi: float = 2e5,
                          avg_degree: int = 8, shift: float = 1e-2,
                          widths=(1, 4, 8), tag=CFG_BATCH) -> list:
    """The batched workload: ``count`` independent systems, n log-uniform in
    [n_lo, n_hi], random-graph Laplacian + shift*I, b ~ N(0,1), block width
    drawn uniformly from ``widths``."""
    rng = rng_for(tag)
    ns = np.rint(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi), count))).astype(np.int64)
    ss = rng.choice(np.asarray(widths), count)
    out = []
    for i in range(count):
        sub = rng_for((tag, 1000 + i))
        A = graph_laplacian(int(ns[i]), avg_degree, shift, sub)
        b = sub.standard_normal(int(ns[i]))
        out.append(BatchSystem(A, b, int(ss[i])))
    return out


def uniform_block_seed(cfg_id: int, s: int) -> int:
    """Seed of the counter-based generator for the random initial block."""
    return cfg_id * 1000 + s

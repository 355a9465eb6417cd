// Device-side building blocks of the MBPCG library for gfx950 (CDNA4).
//
// Layout conventions
//   * n x S blocks are row-major with the S columns of a row contiguous, so a
//     row of P is one 8*S-byte segment (the paper keeps column-major blocks
//     and notes that row-major would coalesce the block product, Sec. 3).
//   * S is the padded storage width (1, 2, 4, 8, 16 or 32); the caller's s <= S
//     columns are the copies, columns s..S-1 hold zeros and are inactive.
//   * Small S x S matrices live in the DevState with a fixed stride of 32.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define MB_SM 32
#define MB_BLOCK 256

// threads of the one-workgroup tail kernels: enough that each entry of an
// s = 32 Gram (528 entries) is summed by one thread in one pass
constexpr int TAIL_THREADS = 1024;

namespace mb {

enum DoneCode : int32_t {
    DONE_RUNNING = 0,
    DONE_CONVERGED = 1,
    DONE_MAXITER = 2,
    DONE_BREAKDOWN = 3,
    DONE_NOTSPD = 4,
    DONE_NONFINITE = 5,
    DONE_ZERO_RHS = 6,
    // the best column met tol_initial > tol: the host runs the least squares
    // and either finishes the solve or resumes the loop (Alg. 1's two tests)
    DONE_LS = 7,
};

// Per-solve state resident in device memory.  The host reads `done` and
// `iter` (adjacent, 8 bytes) between graph launches.
struct DevState {
    int32_t done, iter, h, width;
    int32_t deflations, max_iter, s, accepted;
    int32_t ls_ok, ls_width, n_hist, ready;  // ready: setup finished (X0, X~ valid)
    double tol, tol0, bnorm, nu_h;
    double gamma, rel_ls, rel_true, y0;
    double tau, bbar_norm, res_norm, pad2;
    // Chronopoulos-Gear scalars
    double cg_alpha, cg_beta, cg_gamma, cg_rel;
    double Xi[MB_SM * MB_SM];
    double alpha[MB_SM * MB_SM];
    double Sigma[MB_SM * MB_SM];
    double M[MB_SM * MB_SM];   // W = V M   (inverse of the kept Cholesky factor)
    double Z[MB_SM * MB_SM];   // P = W + P Z^T, Sigma <- Z Sigma
    double nu[MB_SM];
    double chat[MB_SM + 1];
    int32_t active[MB_SM];
    // 1 from the Xi tail of an iteration whose update runs until the next
    // Xi tail: tells the direction update to apply that iteration's
    // X~ += P alpha even when the QR tail has just stopped the loop
    int32_t xt_pending;
    // 1 when tol_initial > tol: the stop test on the best column hands over to
    // the least squares (DONE_LS) instead of finishing the solve
    int32_t ls_inloop;
    // 1 after a resumed Cholesky QR: the direction kernel of that iteration
    // leaves X~ alone (its update was applied when the loop stopped)
    int32_t xt_skip, pad3;
};

__host__ __device__ constexpr int tri_count(int S) { return S * (S + 1) / 2; }
__host__ __device__ constexpr int floor_pow2(int v) {
    int p = 1;
    while (p * 2 <= v) p *= 2;
    return p;
}

// e -> (i, j) with i >= j, e = i (i + 1) / 2 + j
__device__ __forceinline__ void tri_ij(int e, int& i, int& j) {
    int r = (int)((sqrt(8.0 * (double)e + 1.0) - 1.0) * 0.5);
    while ((r + 1) * (r + 2) / 2 <= e) ++r;
    while (r * (r + 1) / 2 > e) --r;
    i = r;
    j = e - r * (r + 1) / 2;
}

// Loads and stores of data that is touched once per iteration and not again
// before a whole iteration (about a gigabyte at 128^3, s = 4) has streamed
// past it -- the CSR arrays, X~ and R -- are non-temporal, so that the blocks
// the next kernel reads again (P, Q, V, W) stay in the 256 MB last-level
// cache.  Measured in a full solve: 10 % less time per iteration at s = 4.
template <class T>
__device__ __forceinline__ T stream_load(const T* p) { return __builtin_nontemporal_load(p); }
template <class T>
__device__ __forceinline__ void stream_store(T* p, T v) { __builtin_nontemporal_store(v, p); }

// ---------------------------------------------------------------------------
// A copy of N consecutive doubles into LDS, split into a load step and a
// store step so that a kernel can issue every load of a tile (several
// blocks, its own rows) before the first LDS store: the copy then costs one
// memory round trip instead of one per element a thread moves.  Elements at
// or beyond `valid` are zero; their addresses are clamped to src[0].
// ---------------------------------------------------------------------------
template <int N>
struct Stage {
    static constexpr int EPT = (N + MB_BLOCK - 1) / MB_BLOCK;
    double v[EPT];
    __device__ __forceinline__ void load(const double* __restrict__ src, int valid) {
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
            const int e = threadIdx.x + q * MB_BLOCK;
            const bool in = e < valid;
            const double x = src[in ? e : 0];
            v[q] = in ? x : 0.0;
        }
    }
    __device__ __forceinline__ void store(double* dst) const {
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
            const int e = threadIdx.x + q * MB_BLOCK;
            if (N % MB_BLOCK == 0 || e < N) dst[e] = v[q];
        }
    }
};

// ---------------------------------------------------------------------------
// Work split of n rows, in tiles of T rows, over the grid.  On MI355X
// consecutive workgroup ids land on different XCDs (8 of them, each with its
// own L2), so when the grid is a multiple of 8 each XCD is given one
// contiguous slab of tiles and its workgroups sweep that slab together: the
// stencil/graph neighbours of a tile are then rows the same L2 saw recently.
// ---------------------------------------------------------------------------
struct TileRange {
    int64_t first, end, step;
};

__device__ __forceinline__ TileRange tile_range(int64_t ntiles) {
    const int nwg = gridDim.x;
    TileRange t;
    if ((nwg & 7) == 0 && ntiles >= nwg) {
        const int x = blockIdx.x & 7, k = blockIdx.x >> 3;
        const int64_t lo = ntiles * x / 8, hi = ntiles * (x + 1) / 8;
        t.first = lo + k;
        t.end = hi;
        t.step = nwg >> 3;
    } else {
        t.first = blockIdx.x;
        t.end = ntiles;
        t.step = nwg;
    }
    return t;
}

// ---------------------------------------------------------------------------
// Deterministic per-workgroup accumulator of ETOT sums over rows of LDS tiles.
// Entries are spread over the 256 threads; when ETOT < 256 each entry's rows
// are split over TPE threads whose partial sums are added in a fixed order at
// the end.  f(k, r) returns the term of this thread's k-th entry (ent[k]) for
// tile row r.
// ---------------------------------------------------------------------------
template <int ETOT>
struct TileSums {
    static constexpr int TPE = ETOT >= MB_BLOCK ? 1 : floor_pow2(MB_BLOCK / ETOT);
    static constexpr int EPT = TPE == 1 ? (ETOT + MB_BLOCK - 1) / MB_BLOCK : 1;
    double acc[EPT];
    int ent[EPT];
    int sub;

    __device__ __forceinline__ void init() {
        const int t = threadIdx.x;
        if (TPE > 1) {
            ent[0] = t / TPE;
            sub = t % TPE;
            if (ent[0] >= ETOT) ent[0] = -1;
        } else {
            sub = 0;
#pragma unroll
            for (int k = 0; k < EPT; ++k) {
                int e = t + k * MB_BLOCK;
                ent[k] = e < ETOT ? e : -1;
            }
        }
#pragma unroll
        for (int k = 0; k < EPT; ++k) acc[k] = 0.0;
    }

    template <class F>
    __device__ __forceinline__ void add_rows(int rows, F f) {
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
            const int e = ent[k];
            if (e < 0) continue;
            double a = acc[k];
            for (int r = sub; r < rows; r += TPE) a += f(k, r);
            acc[k] = a;
        }
    }

    // Writes the workgroup's ETOT sums to out[0..ETOT).  lds must hold
    // MB_BLOCK doubles.  Ends with a barrier.  The TPE partial sums of an
    // entry are added by a pairwise tree (fixed order).
    __device__ __forceinline__ void finish(double* lds, double* out) {
        if (TPE > 1) {
            __syncthreads();
            lds[threadIdx.x] = acc[0];
            __syncthreads();
            const int q = threadIdx.x % TPE;
#pragma unroll
            for (int h = TPE / 2; h >= 1; h /= 2) {
                if (q < h) lds[threadIdx.x] += lds[threadIdx.x + h];
                __syncthreads();
            }
            const int e = threadIdx.x;
            if (e < ETOT) out[e] = lds[e * TPE];
            __syncthreads();
        } else {
#pragma unroll
            for (int k = 0; k < EPT; ++k)
                if (ent[k] >= 0) out[ent[k]] = acc[k];
        }
    }
};

// Column sums of red[q * S + j] over q < MB_BLOCK / S (one value per thread,
// thread t = q * S + j already stored), by a pairwise tree over q; the sum
// of column j ends in red[j].  Starts and ends with a barrier.
template <int S>
__device__ __forceinline__ void column_sums(double* red) {
    constexpr int RPP = MB_BLOCK / S;
    const int t = threadIdx.x, q = t / S;
    __syncthreads();
#pragma unroll
    for (int h = RPP / 2; h >= 1; h /= 2) {
        if (q < h) red[t] += red[t + h * S];
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Lower triangle of X^T Y over the rows of tiles, on the matrix cores
// (v_mfma_f64_16x16x4f64), for S >= 8.  Wavefront w takes rows 4w..4w+3 of
// every 16-row group of a tile; lane l feeds A = X^T[i = l%16][k = l/16] and
// B = Y[k = l/16][j = l%16], and holds C[i = l/16 + 4v][j = l%16] in element
// v of its accumulator.  The four wavefronts' sums are added in a fixed order
// once, at the end.
// ---------------------------------------------------------------------------
typedef double mb_d4 __attribute__((ext_vector_type(4)));

template <int S>
struct GramMfma {
    static constexpr int NB = S >= 16 ? S / 16 : 1;  // 16 x 16 blocks per dimension
    mb_d4 acc[NB][NB];

    __device__ __forceinline__ void init() {
#pragma unroll
        for (int a = 0; a < NB; ++a)
#pragma unroll
            for (int b = 0; b < NB; ++b) acc[a][b] = mb_d4{0.0, 0.0, 0.0, 0.0};
    }

    // xv(r, c) / yv(r, c): element (row r, column c) of X / Y in this tile
    template <class FX, class FY>
    __device__ __forceinline__ void add_tile(int rows, FX xv, FY yv) {
        const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
        const int li = l & 15, lk = l >> 4;
        for (int k0 = wave * 4; k0 < rows; k0 += 16) {
            const int r = k0 + lk;
            const bool ok = r < rows;
            double a[NB], b[NB];
#pragma unroll
            for (int q = 0; q < NB; ++q) {
                const int c = q * 16 + li;
                a[q] = (ok && c < S) ? xv(r, c) : 0.0;
                b[q] = (ok && c < S) ? yv(r, c) : 0.0;
            }
#pragma unroll
            for (int ib = 0; ib < NB; ++ib)
#pragma unroll
                for (int jb = 0; jb <= ib; ++jb)
                    acc[ib][jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ib], b[jb], acc[ib][jb], 0, 0, 0);
        }
    }

    // Writes the workgroup's lower triangle (e = i(i+1)/2 + j) to out.  lds
    // must hold S*S doubles; ends with a barrier.
    __device__ __forceinline__ void finish(double* lds, double* out) {
        const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
        const int li = l & 15, lk = l >> 4;
        __syncthreads();
        for (int w = 0; w < MB_BLOCK / 64; ++w) {
            if (wave == w) {
#pragma unroll
                for (int ib = 0; ib < NB; ++ib)
#pragma unroll
                    for (int jb = 0; jb <= ib; ++jb)
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int i = ib * 16 + lk + 4 * v, j = jb * 16 + li;
                            if (i < S && j < S) {
                                const double x = acc[ib][jb][v];
                                lds[i * S + j] = (w == 0) ? x : lds[i * S + j] + x;
                            }
                        }
            }
            __syncthreads();
        }
        for (int e = threadIdx.x; e < tri_count(S); e += MB_BLOCK) {
            int i, j;
            tri_ij(e, i, j);
            out[e] = lds[i * S + j];
        }
        __syncthreads();
    }
};

// Sum of part[w * stride + e] for w in [w0, w1): eight interleaved
// accumulators (partial w0 + i goes to accumulator i mod 8, the last
// (w1 - w0) mod 8 to accumulators 0, 1, ...), combined in a fixed tree;
// up to 32 loads in flight.
__device__ __forceinline__ double sum_strided(const double* __restrict__ part, int w0, int w1,
                                              int stride, int e) {
    double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int w = w0;
    // runs of 32 and then 16 partials issue all their loads before adding
    // them (same additions in the same order as the runs of 8)
    for (; w + 32 <= w1; w += 32) {
        double v[32];
#pragma unroll
        for (int u = 0; u < 32; ++u) v[u] = part[(int64_t)(w + u) * stride + e];
#pragma unroll
        for (int u = 0; u < 32; ++u) a[u % 8] += v[u];
    }
    if (w + 16 <= w1) {
        double v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) v[u] = part[(int64_t)(w + u) * stride + e];
#pragma unroll
        for (int u = 0; u < 16; ++u) a[u % 8] += v[u];
        w += 16;
    }
    for (; w + 8 <= w1; w += 8) {
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] += part[(int64_t)(w + u) * stride + e];
    }
    // the last w1 - w < 8 partials go to a[0], a[1], ... (loads first)
    const int r = w1 - w;
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = u < r ? part[(int64_t)(w + u) * stride + e] : 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u)
        if (u < r) a[u] += v[u];
    return ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
}

// Sum part[w * stride + e] over w = 0..nwg-1 in a fixed order into out[e]
// (LDS), using all threads of the block: tpe = floor_pow2(blockDim / E)
// threads per entry each add a contiguous range of partials, then a pairwise
// tree over those tpe sums.  tmp must hold max(blockDim, E) doubles.  Ends
// with a barrier.
__device__ __forceinline__ void reduce_partials(const double* __restrict__ part, int nwg, int E,
                                                int stride, double* out, double* tmp) {
    const int B = blockDim.x, t = threadIdx.x;
    if (E >= B) {
        for (int e = t; e < E; e += B) out[e] = sum_strided(part, 0, nwg, stride, e);
        __syncthreads();
        return;
    }
    int tpe = 1;
    while (tpe * 2 * E <= B) tpe *= 2;
    const int e = t % E, q = t / E;
    if (q < tpe) {
        const int chunk = (nwg + tpe - 1) / tpe;
        const int w0 = min(nwg, q * chunk), w1 = min(nwg, w0 + chunk);
        tmp[q * E + e] = sum_strided(part, w0, w1, stride, e);
    }
    __syncthreads();
    for (int h = tpe / 2; h >= 1; h /= 2) {
        if (q < h) tmp[q * E + e] += tmp[(q + h) * E + e];
        __syncthreads();
    }
    if (t < E) out[t] = tmp[t];
    __syncthreads();
}

__device__ __forceinline__ bool finite_d(double v) { return v - v == 0.0; }

}  // namespace mb

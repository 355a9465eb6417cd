// Dense block product Q = A P on the matrix cores (the A P of Alg. 1 for dense
// A; Sec. 3 keeps dense A column-major in FP64).
//
// A workgroup of four wavefronts owns 256 rows and one of KSPLIT column
// ranges; wavefront w owns rows [64w, 64w + 64) as four 16-row MFMA tiles, and
// every S/16 output column tile reuses each loaded A operand.  The FP64
// kernel reads P directly (the block is a few MB and stays in the L2) and
// issues the loads of the next k-steps ahead of the MFMAs.  The
// KSPLIT partial products are written to a scratch block and added in a fixed
// order by k_dense_reduce, which also forms the Gram P^T Q of the tail.
//
//   FP64:  v_mfma_f64_16x16x4f64 on the caller's column-major A.
//   FP32:  v_mfma_f32_16x16x4f32 on a tiled FP32 copy of A.
//   BF16:  v_mfma_f32_16x16x32_bf16 on a tiled BF16 copy of A.
// Low-precision kinds accumulate in FP32 inside a workgroup; their partials
// are stored as FP32 (the accumulators' values, half the bytes of FP64) and
// added in FP64.  Every kernel reads A with non-temporal loads (A is not read
// again before the next product and does not fit the last-level cache); the
// partials of S >= 16 columns are stored non-temporally as well (measured
// faster there, slower for narrower blocks).
#include "kernels.hpp"

#include <algorithm>

#include <hip/hip_bf16.h>

namespace mb {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int DENSE_ROWS = 256;  // rows per workgroup
constexpr int DENSE_KSPLIT = 16;

int dense_ksplit(int64_t n) {
    int k = DENSE_KSPLIT;
    while (k > 1 && n / k < 256) k /= 2;
    return k;
}
int dense_nwg_rows(int64_t n) { return (int)((n + DENSE_ROWS - 1) / DENSE_ROWS); }

// ---------------------------------------------------------------------------
template <int S>
__global__ __launch_bounds__(MB_BLOCK) void k_dense_f64(int64_t n, const double* __restrict__ A,
                                                        int64_t lda, const double* __restrict__ P,
                                                        double* __restrict__ qpart, int ksplit,
                                                        const DevState* __restrict__ st) {
    if (st && st->done) return;
    constexpr int CT = S >= 16 ? S / 16 : 1;  // output column tiles
    constexpr int QS = 4;                     // MFMA k-steps (of 4) per trip
    const int rb = blockIdx.x / ksplit, ks = blockIdx.x % ksplit;
    const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int64_t kchunk = (n + ksplit - 1) / ksplit;
    const int64_t kbeg = ks * kchunk, kend = min(n, kbeg + kchunk);
    const int64_t rbase = (int64_t)rb * DENSE_ROWS + wave * 64;
    const int li = l & 15, lk = l >> 4;
    int64_t row[4];
    bool rok[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        row[t] = rbase + 16 * t + li;
        rok[t] = row[t] < n;
    }
    d4 acc[4][CT];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int c = 0; c < CT; ++c) acc[t][c] = d4{0.0, 0.0, 0.0, 0.0};
    // operands of QS k-steps from k0: lane (li, lk) holds A[row t][k0 + 4q + lk]
    // and P[k0 + 4q + lk][16c + li] (P is a few MB and stays in the L2)
    auto load = [&](int64_t k0, double (&a)[QS][4], double (&b)[QS][CT]) {
#pragma unroll
        for (int q = 0; q < QS; ++q) {
            const int64_t k = k0 + 4 * q + lk;
            const bool kin = k < kend;
#pragma unroll
            for (int t = 0; t < 4; ++t) a[q][t] = (kin && rok[t]) ? stream_load(A + k * lda + row[t]) : 0.0;
#pragma unroll
            for (int c = 0; c < CT; ++c) {
                const int j = 16 * c + li;
                b[q][c] = (kin && j < S) ? P[k * S + j] : 0.0;
            }
        }
    };
    auto mma = [&](const double (&a)[QS][4], const double (&b)[QS][CT]) {
#pragma unroll
        for (int q = 0; q < QS; ++q)
#pragma unroll
            for (int c = 0; c < CT; ++c)
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    acc[t][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q][t], b[q][c], acc[t][c], 0,
                                                                    0, 0);
    };
    // no LDS and no barriers: the loads of the next trip are issued before
    // the MFMAs of this one, and the other wavefronts of the CU overlap theirs
    double a0[QS][4], b0[QS][CT], a1[QS][4], b1[QS][CT];
    int64_t k0 = kbeg;
    if (k0 < kend) load(k0, a0, b0);
    for (; k0 < kend; k0 += 8 * QS) {
        const int64_t k1 = k0 + 4 * QS;
        if (k1 < kend) load(k1, a1, b1);
        mma(a0, b0);
        if (k1 < kend) {
            if (k1 + 4 * QS < kend) load(k1 + 4 * QS, a0, b0);
            mma(a1, b1);
        }
    }
    // D layout of v_mfma_f64_16x16x4f64: lane l, element v -> row l/16 + 4v, column l % 16
    double* out = qpart + (int64_t)ks * n * S;
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int c = 0; c < CT; ++c)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t r = rbase + 16 * t + lk + 4 * v;
                const int j = 16 * c + li;
                if (r < n && j < S) {
                    if constexpr (S >= 16) stream_store(out + r * S + j, acc[t][c][v]);
                    else out[r * S + j] = acc[t][c][v];
                }
            }
}

// Low-precision products on the tiled copies (layouts in kernels.hpp).  A
// wavefront streams its four 16-row tiles of A with one contiguous 1 KiB load
// each per k-step and reads its P operand (one 16-byte vector per lane, the
// P block is L2-resident) directly: no LDS and no barriers, so the loads of
// the next steps overlap the matrix-core work of this one.
//   FP32: v_mfma_f32_16x16x4f32, k-step 16 = four MFMAs on k = 16kc + 4lk + u.
//   BF16: v_mfma_f32_16x16x32_bf16, k-step 32: lane (lk, li) holds
//         A[row li][8 lk .. 8 lk + 7] and P[8 lk .. 8 lk + 7][column li].
template <int S>
__global__ __launch_bounds__(MB_BLOCK) void k_dense_f32(int64_t n, const float* __restrict__ A,
                                                        const float* __restrict__ P,
                                                        float* __restrict__ qpart, int ksplit,
                                                        const DevState* __restrict__ st) {
    if (st && st->done) return;
    constexpr int CT = S >= 16 ? S / 16 : 1;
    const int rb = blockIdx.x / ksplit, ks = blockIdx.x % ksplit;
    const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int li = l & 15, lk = l >> 4;
    const int64_t NK = (n + 15) / 16, RT = (n + 15) / 16;
    const int64_t sps = (NK + ksplit - 1) / ksplit;
    const int64_t kc0 = ks * sps, kc1 = min(NK, kc0 + sps);
    const f4* A4 = reinterpret_cast<const f4*>(A);
    const f4* P4 = reinterpret_cast<const f4*>(P);
    int64_t rt[4];
    bool rok[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        rt[t] = (int64_t)rb * 16 + wave * 4 + t;
        rok[t] = rt[t] < RT;
    }
    f4 acc[4][CT];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int c = 0; c < CT; ++c) acc[t][c] = f4{0.f, 0.f, 0.f, 0.f};
    // k-step kc (kc0 <= kc < kc1) with no branches: a row tile past the
    // matrix and a column past S read an in-range tile or column instead,
    // whose products land only in rows and columns that are never stored
    int64_t rtc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) rtc[t] = rok[t] ? rt[t] : RT - 1;
    auto load = [&](int64_t kc, f4* a, f4* bv) {
#pragma unroll
        for (int t = 0; t < 4; ++t) a[t] = stream_load(A4 + (rtc[t] * NK + kc) * 64 + l);
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            const int j = 16 * c + li;
            bv[c] = P4[(4 * kc + lk) * S + (j < S ? j : S - 1)];
        }
    };
    auto mma = [&](const f4* a, const f4* bv) {
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int c = 0; c < CT; ++c)
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[t][u], bv[c][u], acc[t][c],
                                                                     0, 0, 0);
    };
    // k-steps in pairs, one register set per step, two sets in turn: the next
    // step's loads go out before this step's MFMAs, so a wavefront keeps a
    // step of A in flight while its matrix-core work runs.  The last prefetch
    // re-reads the final step (an in-range address, no branch: the waits
    // before each MFMA then count only the loads they need).  An odd count
    // ends with the last step and an all-zero step, the same MFMAs in the
    // same order as a pair whose second step is past the range.
    const f4 z4 = {0.f, 0.f, 0.f, 0.f};
    const int64_t kp = kc0 + ((kc1 - kc0) & ~(int64_t)1);
    f4 a0[4], b0[CT], a1[4], b1[CT];
    int64_t kc = kc0;
    if (kc < kp) load(kc, a0, b0);
    for (; kc < kp; kc += 2) {
        load(kc + 1, a1, b1);
        __builtin_amdgcn_sched_barrier(0);   // the loads stay ahead of the MFMAs
        mma(a0, b0);
        __builtin_amdgcn_sched_barrier(0);
        load(kc + 2 < kp ? kc + 2 : kp - 1, a0, b0);
        __builtin_amdgcn_sched_barrier(0);
        mma(a1, b1);
        __builtin_amdgcn_sched_barrier(0);
    }
    if (kc < kc1) {
        load(kc, a0, b0);
#pragma unroll
        for (int t = 0; t < 4; ++t) a1[t] = z4;
#pragma unroll
        for (int c = 0; c < CT; ++c) b1[c] = z4;
        mma(a0, b0);
        mma(a1, b1);
    }
    // D layout of the FP32-accumulating MFMAs: lane l, element v -> row
    // 4 (l/16) + v, column l % 16.  The partials are the FP32 accumulators
    // themselves, stored as FP32 (half the bytes of FP64, the same values)
    float* out = qpart + (int64_t)ks * n * S;
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int c = 0; c < CT; ++c)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t r = rt[t] * 16 + 4 * lk + v;
                const int j = 16 * c + li;
                if (r < n && j < S) {
                    if constexpr (S >= 16) stream_store(out + r * S + j, acc[t][c][v]);
                    else out[r * S + j] = acc[t][c][v];
                }
            }
}

template <int S>
__global__ __launch_bounds__(MB_BLOCK) void k_dense_bf16(int64_t n, const __bf16* __restrict__ A,
                                                         const __bf16* __restrict__ P,
                                                         float* __restrict__ qpart, int ksplit,
                                                         const DevState* __restrict__ st) {
    if (st && st->done) return;
    constexpr int CT = S >= 16 ? S / 16 : 1;
    const int rb = blockIdx.x / ksplit, ks = blockIdx.x % ksplit;
    const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int li = l & 15, lk = l >> 4;
    const int64_t NK = (n + 31) / 32, RT = (n + 15) / 16;
    const int64_t sps = (NK + ksplit - 1) / ksplit;
    const int64_t kc0 = ks * sps, kc1 = min(NK, kc0 + sps);
    const bf8* A8 = reinterpret_cast<const bf8*>(A);
    const bf8* P8 = reinterpret_cast<const bf8*>(P);
    bf8 zero8;
#pragma unroll
    for (int u = 0; u < 8; ++u) zero8[u] = (__bf16)0.0f;
    int64_t rt[4];
    bool rok[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        rt[t] = (int64_t)rb * 16 + wave * 4 + t;
        rok[t] = rt[t] < RT;
    }
    f4 acc[4][CT];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int c = 0; c < CT; ++c) acc[t][c] = f4{0.f, 0.f, 0.f, 0.f};
    // k-step kc (kc0 <= kc < kc1) with no branches, as in the FP32 kernel
    int64_t rtc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) rtc[t] = rok[t] ? rt[t] : RT - 1;
    auto load = [&](int64_t kc, bf8* a, bf8* bv) {
#pragma unroll
        for (int t = 0; t < 4; ++t) a[t] = stream_load(A8 + (rtc[t] * NK + kc) * 64 + l);
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            const int j = 16 * c + li;
            bv[c] = P8[(4 * kc + lk) * S + (j < S ? j : S - 1)];
        }
    };
    auto mma = [&](const bf8* a, const bf8* bv) {
#pragma unroll
        for (int c = 0; c < CT; ++c)
#pragma unroll
            for (int t = 0; t < 4; ++t)
                acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[t], bv[c], acc[t][c], 0, 0, 0);
    };
    // the FP32 kernel's step order and prefetch
    const int64_t kp = kc0 + ((kc1 - kc0) & ~(int64_t)1);
    bf8 a0[4], b0[CT], a1[4], b1[CT];
    int64_t kc = kc0;
    if (kc < kp) load(kc, a0, b0);
    for (; kc < kp; kc += 2) {
        load(kc + 1, a1, b1);
        __builtin_amdgcn_sched_barrier(0);   // the loads stay ahead of the MFMAs
        mma(a0, b0);
        __builtin_amdgcn_sched_barrier(0);
        load(kc + 2 < kp ? kc + 2 : kp - 1, a0, b0);
        __builtin_amdgcn_sched_barrier(0);
        mma(a1, b1);
        __builtin_amdgcn_sched_barrier(0);
    }
    if (kc < kc1) {
        load(kc, a0, b0);
#pragma unroll
        for (int t = 0; t < 4; ++t) a1[t] = zero8;
#pragma unroll
        for (int c = 0; c < CT; ++c) b1[c] = zero8;
        mma(a0, b0);
        mma(a1, b1);
    }
    // D layout of the FP32-accumulating MFMAs: lane l, element v -> row
    // 4 (l/16) + v, column l % 16.  The partials are the FP32 accumulators
    // themselves, stored as FP32 (half the bytes of FP64, the same values)
    float* out = qpart + (int64_t)ks * n * S;
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int c = 0; c < CT; ++c)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t r = rt[t] * 16 + 4 * lk + v;
                const int j = 16 * c + li;
                if (r < n && j < S) {
                    if constexpr (S >= 16) stream_store(out + r * S + j, acc[t][c][v]);
                    else out[r * S + j] = acc[t][c][v];
                }
            }
}

// Q = sum over k-ranges of the partials (fixed order) and the lower triangle
// of P^T Q per workgroup, as the sparse block product's epilogue.
template <int S, class PT>
__global__ __launch_bounds__(MB_BLOCK) void k_dense_reduce(int64_t n, int ksplit,
                                                           const PT* __restrict__ qpart,
                                                           const double* __restrict__ P,
                                                           double* __restrict__ Q,
                                                           double* __restrict__ part,
                                                           const DevState* __restrict__ st) {
    if (st && st->done) return;
    constexpr int T = dense_reduce_rows(S);
    constexpr int E = tri_count(S);
    constexpr bool MF = S >= 8;
    __shared__ double sP[T * S], sQ[T * S], red[MB_BLOCK];
    const int t = threadIdx.x;
    TileSums<E> gs;
    GramMfma<S> gm;
    int gi[TileSums<E>::EPT], gj[TileSums<E>::EPT];
    if constexpr (MF) {
        gm.init();
    } else {
        gs.init();
#pragma unroll
        for (int k = 0; k < TileSums<E>::EPT; ++k) {
            gi[k] = gj[k] = 0;
            if (gs.ent[k] >= 0) tri_ij(gs.ent[k], gi[k], gj[k]);
        }
    }
    const int64_t ntiles = (n + T - 1) / T;
    const TileRange tr = tile_range(ntiles);
    const int64_t nS = n * S;
    for (int64_t tile = tr.first; tile < tr.end; tile += tr.step) {
        const int64_t r0 = tile * T;
        const int rows = (int)min((int64_t)T, n - r0);
        // each thread's EPT entries: four running sums per entry (partial k
        // goes to sum k mod 4), combined in a fixed order; the loads of all
        // entries and of four partials are issued together
        constexpr int EPT = (T * S + MB_BLOCK - 1) / MB_BLOCK;
        double q4[EPT][4], pv[EPT];
        int64_t gq[EPT];
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
            const int e = t + q * MB_BLOCK;
            gq[q] = r0 * S + (e < rows * S ? e : 0);
            pv[q] = P[gq[q]];
#pragma unroll
            for (int u = 0; u < 4; ++u) q4[q][u] = 0.0;
        }
        int k = 0;
        for (; k + 4 <= ksplit; k += 4) {
            double v[EPT][4];
#pragma unroll
            for (int q = 0; q < EPT; ++q)
#pragma unroll
                for (int u = 0; u < 4; ++u) v[q][u] = (double)qpart[(k + u) * nS + gq[q]];
#pragma unroll
            for (int q = 0; q < EPT; ++q)
#pragma unroll
                for (int u = 0; u < 4; ++u) q4[q][u] += v[q][u];
        }
        for (int u = 0; k < ksplit; ++k, ++u)
#pragma unroll
            for (int q = 0; q < EPT; ++q) q4[q][u] += (double)qpart[k * nS + gq[q]];
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
            const int e = t + q * MB_BLOCK;
            if (e >= T * S) continue;
            const bool in = e < rows * S;
            const double qv = (q4[q][0] + q4[q][1]) + (q4[q][2] + q4[q][3]);
            if (in) Q[gq[q]] = qv;
            sQ[e] = in ? qv : 0.0;
            sP[e] = in ? pv[q] : 0.0;
        }
        __syncthreads();
        if (part) {
            if constexpr (MF)
                gm.add_tile(rows, [&](int r, int c) { return sP[r * S + c]; },
                            [&](int r, int c) { return sQ[r * S + c]; });
            else
                gs.add_rows(rows, [&](int k, int r) { return sP[r * S + gi[k]] * sQ[r * S + gj[k]]; });
        }
        __syncthreads();
    }
    if (part) {
        if constexpr (MF) gm.finish(sQ, part + (int64_t)blockIdx.x * E);
        else gs.finish(red, part + (int64_t)blockIdx.x * E);
    }
}

// r = b - sum of partials of A x (S = 1), partial ||r||^2 per workgroup
__global__ __launch_bounds__(MB_BLOCK) void k_dense_resid_reduce(int64_t n, int ksplit,
                                                                 const double* __restrict__ qpart,
                                                                 const double* __restrict__ b,
                                                                 double* __restrict__ r_out,
                                                                 double* __restrict__ part) {
    __shared__ double red[MB_BLOCK];
    double s2 = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)MB_BLOCK + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * MB_BLOCK) {
        double q = 0.0;
        for (int k = 0; k < ksplit; ++k) q += qpart[k * n + i];
        const double e = b[i] - q;
        if (r_out) r_out[i] = e;
        s2 += e * e;
    }
    red[threadIdx.x] = s2;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int k = 0; k < MB_BLOCK; ++k) s += red[k];
        part[blockIdx.x] = s;
    }
}

// FP64 column-major A -> tiled low-precision layout (round to nearest even).
// One thread writes one lane vector of one tile; the 16 lanes li of a k-group
// read 16 consecutive rows of a column (128 contiguous bytes).
template <int KIND>
__global__ void k_cast_dense(int64_t n, const double* __restrict__ A, int64_t lda,
                             void* __restrict__ out) {
    constexpr int VL = lo_vec(KIND), KS = lo_kstep(KIND);
    const int64_t NK = (n + KS - 1) / KS, RT = (n + 15) / 16;
    const int64_t total = RT * NK * 64;
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < total;
         v += (int64_t)gridDim.x * blockDim.x) {
        const int lane = (int)(v & 63);
        const int64_t tile = v >> 6;
        const int64_t rt = tile / NK, kc = tile % NK;
        const int64_t r = rt * 16 + (lane & 15);
        const int64_t k = kc * KS + (int64_t)(lane >> 4) * VL;
#pragma unroll
        for (int u = 0; u < VL; ++u) {
            const double x = (r < n && k + u < n) ? A[(k + u) * lda + r] : 0.0;
            if (KIND == DENSE_F32) static_cast<float*>(out)[v * VL + u] = (float)x;
            else static_cast<__hip_bfloat16*>(out)[v * VL + u] = __double2bfloat16(x);
        }
    }
}

size_t dense_lo_bytes(DenseKind kind, int64_t n) {
    const int KS = lo_kstep(kind);
    const size_t rows = (size_t)((n + 15) / 16) * 16, cols = (size_t)((n + KS - 1) / KS) * KS;
    return rows * cols * (kind == DENSE_F32 ? 4 : 2);
}

__global__ void k_diag_dense(int64_t n, const double* __restrict__ A, int64_t lda, int jacobi,
                             double* __restrict__ d, DevState* st) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * blockDim.x) {
        const double a = A[r * lda + r];
        double dr = 1.0;
        if (jacobi) {
            if (!(a > 0.0) || !finite_d(a)) st->done = DONE_NOTSPD;
            else dr = sqrt(a);
        }
        d[r] = dr;
    }
}

__global__ void k_scale_dense(int64_t n, const double* __restrict__ A, int64_t lda,
                              const double* __restrict__ d, double* __restrict__ As) {
    const int64_t total = n * n;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = e / n, r = e % n;
        As[e] = A[c * lda + r] / (d[r] * d[c]);
    }
}

// ---------------------------------------------------------------------------
#define MB_DENSE_S(S, CALL)         \
    switch (S) {                    \
        case 1: { constexpr int SS = 1; CALL; } \
        case 2: { constexpr int SS = 2; CALL; } \
        case 4: { constexpr int SS = 4; CALL; } \
        case 8: { constexpr int SS = 8; CALL; } \
        case 16: { constexpr int SS = 16; CALL; } \
        case 32: { constexpr int SS = 32; CALL; } \
    }                               \
    return hipErrorInvalidValue;

hipError_t launch_dense_ap(int S, DenseKind kind, int64_t n, const void* A, int64_t lda,
                           const void* Plo, const double* P, double* qpart, int ksplit,
                           const DevState* st, hipStream_t stream) {
    const int nwg = dense_nwg_rows(n) * ksplit;
    MB_DENSE_S(S, {
        if (kind == DENSE_F64)
            hipLaunchKernelGGL(k_dense_f64<SS>, dim3(nwg), dim3(MB_BLOCK), 0, stream, n,
                               (const double*)A, lda, P, qpart, ksplit, st);
        else if (kind == DENSE_F32)
            hipLaunchKernelGGL(k_dense_f32<SS>, dim3(nwg), dim3(MB_BLOCK), 0, stream, n,
                               (const float*)A, (const float*)Plo, (float*)qpart, ksplit, st);
        else
            hipLaunchKernelGGL(k_dense_bf16<SS>, dim3(nwg), dim3(MB_BLOCK), 0, stream, n,
                               (const __bf16*)A, (const __bf16*)Plo, (float*)qpart, ksplit, st);
        return hipGetLastError();
    })
}

hipError_t launch_dense_reduce(int S, DenseKind kind, int64_t n, int ksplit, const double* qpart,
                               const double* P, double* Q, double* part, int nwg,
                               const DevState* st, hipStream_t stream) {
    MB_DENSE_S(S, {
        if (kind == DENSE_F64)
            hipLaunchKernelGGL((k_dense_reduce<SS, double>), dim3(nwg), dim3(MB_BLOCK), 0, stream,
                               n, ksplit, qpart, P, Q, part, st);
        else
            hipLaunchKernelGGL((k_dense_reduce<SS, float>), dim3(nwg), dim3(MB_BLOCK), 0, stream,
                               n, ksplit, (const float*)qpart, P, Q, part, st);
        return hipGetLastError();
    })
}

hipError_t launch_cast_dense(DenseKind kind, int64_t n, const double* A, int64_t lda, void* out,
                             hipStream_t stream) {
    const int g = 8192;
    if (kind == DENSE_F32)
        hipLaunchKernelGGL(k_cast_dense<DENSE_F32>, dim3(g), dim3(MB_BLOCK), 0, stream, n, A, lda, out);
    else if (kind == DENSE_BF16)
        hipLaunchKernelGGL(k_cast_dense<DENSE_BF16>, dim3(g), dim3(MB_BLOCK), 0, stream, n, A, lda,
                           out);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_diag_dense(int64_t n, const double* A, int64_t lda, int jacobi, double* d,
                             DevState* st, hipStream_t s) {
    int nb = (int)std::min<int64_t>((n + MB_BLOCK - 1) / MB_BLOCK, 4096);
    hipLaunchKernelGGL(k_diag_dense, dim3(nb), dim3(MB_BLOCK), 0, s, n, A, lda, jacobi, d, st);
    return hipGetLastError();
}

hipError_t launch_scale_dense(int64_t n, const double* A, int64_t lda, const double* d, double* As,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_scale_dense, dim3(8192), dim3(MB_BLOCK), 0, s, n, A, lda, d, As);
    return hipGetLastError();
}

hipError_t launch_dense_resid_reduce(int64_t n, int ksplit, const double* qpart, const double* b,
                                     double* r_out, double* part, int nwg, hipStream_t stream) {
    hipLaunchKernelGGL(k_dense_resid_reduce, dim3(nwg), dim3(MB_BLOCK), 0, stream, n, ksplit, qpart,
                       b, r_out, part);
    return hipGetLastError();
}

}  // namespace mb

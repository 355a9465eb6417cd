// One tile of the CSR block product Q = A P (row-major P, Q with S columns),
// as the batched persistent kernel computes it (the single-system kernel in
// k_sparse.hip has its own tile loop and tuned shapes).
//
// The tile's row pointers and then its slice of column indices and values
// (one contiguous range of the CSR arrays) are copied into LDS with
// coalesced loads, in chunks of NZC nonzeros so rows of any length work.
// A row is then handled by (S / V) * SL lanes: lane (slot, jv) walks every
// SL-th nonzero of the row from LDS and gathers the V adjacent columns
// jv .. jv+V-1 of P[col] (16-byte loads for V = 2, 4), U gathers in flight,
// adding them in order; the SL slot sums are combined by a fixed butterfly.
// With V = S / 2 for S >= 4 a 128-row tile takes one pass of its rows
// instead of S / 2 passes, each pass a dependent round of gathers.  The
// tile's Q rows land in LDS (sQ) for a coalesced store and for the Gram
// epilogue.
#pragma once
#include "dev_common.hpp"

namespace mb {

template <int S, int T, int SL>
struct SpmmTile {
    static constexpr int V = S >= 4 ? S / 2 : 1;       // adjacent columns per lane
    static constexpr int CPR = S / V;                  // lanes per row and slot
    static constexpr int LPR = CPR * SL;               // lanes per row
    static constexpr int RPP = MB_BLOCK / LPR;         // rows per pass
    static constexpr int NR = (T + RPP - 1) / RPP;     // passes per tile
    static constexpr int NZC = 8 * T;                  // nonzeros per LDS chunk
    static constexpr int U = (V >= 4 ? 4 : 8) / SL;    // gathers in flight per lane
    // LDS: row pointers, chunk of column indices and values, Q tile
    static constexpr int LDS_BYTES = 4 * (T + 1) + 4 * NZC + 8 * NZC + 8 * T * S;
};

template <int V>
__device__ __forceinline__ void spmm_load_cols(const double* p, double* x) {
    if constexpr (V == 1) {
        x[0] = p[0];
    } else {
#pragma unroll
        for (int h = 0; h < V / 2; ++h) {
            const double2 t = reinterpret_cast<const double2*>(p)[h];
            x[2 * h] = t.x;
            x[2 * h + 1] = t.y;
        }
    }
}

// Computes the tile's rows [r0, r0 + rows) of Q into sQ (T x S, rows >= `rows`
// zero).  All threads of the block call it; it ends with a barrier.
template <int S, int T, int SL>
__device__ __forceinline__ void spmm_tile(const int32_t* __restrict__ rowptr,
                                          const int32_t* __restrict__ colind,
                                          const double* __restrict__ vals,
                                          const double* __restrict__ P, int64_t r0, int rows,
                                          int32_t* sRp, int32_t* sC, double* sV, double* sQ) {
    using TL = SpmmTile<S, T, SL>;
    constexpr int V = TL::V, CPR = TL::CPR, RPP = TL::RPP, NR = TL::NR, NZC = TL::NZC;
    constexpr int U = TL::U;
    const int tid = threadIdx.x;
    const int grp = tid / TL::LPR, lane = tid % TL::LPR;
    const int slot = lane / CPR, jv = (lane % CPR) * V;
    // each staging copy issues all of a thread's loads before its LDS stores
    // (one memory round trip; addresses clamped inside the arrays)
    constexpr int RPT = (T + 1 + MB_BLOCK - 1) / MB_BLOCK;
    constexpr int CPT = (NZC + MB_BLOCK - 1) / MB_BLOCK;
    int rpv[RPT];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int e = tid + q * MB_BLOCK;
        rpv[q] = rowptr[r0 + (e <= rows ? e : 0)];
    }
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int e = tid + q * MB_BLOCK;
        if (e <= rows) sRp[e] = rpv[q];
    }
    __syncthreads();
    const int nz0 = sRp[0];
    const int nzt = sRp[rows] - nz0;
    double acc[NR][V];
#pragma unroll
    for (int i = 0; i < NR; ++i)
#pragma unroll
        for (int q = 0; q < V; ++q) acc[i][q] = 0.0;
    for (int cb = 0; cb < nzt; cb += NZC) {
        const int cn = min(NZC, nzt - cb);
        int cc[CPT];
        double cv[CPT];
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            const int e = tid + q * MB_BLOCK;
            const int64_t g = (int64_t)nz0 + cb + (e < cn ? e : 0);
            cc[q] = colind[g];
            cv[q] = vals[g];
        }
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            const int e = tid + q * MB_BLOCK;
            if (e < cn) {
                sC[e] = cc[q];
                sV[e] = cv[q];
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            const int rl = i * RPP + grp;
            if (rl >= rows) continue;
            const int kb = sRp[rl] - nz0, ke = sRp[rl + 1] - nz0;
            // this slot's nonzeros kb + slot + m*SL that fall in [cb, cb + cn)
            int k = kb + slot;
            if (k < cb) k += ((cb - k + SL - 1) / SL) * SL;
            const int kend = min(ke, cb + cn);
            for (; k < kend; k += U * SL) {
                int c[U];
                double v[U], x[U][V];
                // every slot's column and value first (a slot past the row
                // reads the row's last entry, in bounds, unused), then the
                // gathers, then the sums in order
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int kk = k + u * SL;
                    const int kc = (kk < kend ? kk : kend - 1) - cb;
                    c[u] = sC[kc];
                    v[u] = sV[kc];
                }
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (k + u * SL < kend) spmm_load_cols<V>(P + (int64_t)c[u] * S + jv, x[u]);
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (k + u * SL < kend) {
#pragma unroll
                        for (int q = 0; q < V; ++q) acc[i][q] += v[u] * x[u][q];
                    }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        const int rl = i * RPP + grp;
#pragma unroll
        for (int q = 0; q < V; ++q) {
            double a = acc[i][q];
#pragma unroll
            for (int off = CPR; off < TL::LPR; off <<= 1) a += __shfl_xor(a, off, 64);
            if (slot == 0 && rl < T) sQ[rl * S + jv + q] = rl < rows ? a : 0.0;
        }
    }
    __syncthreads();
}

}  // namespace mb

// Block product of the sparse path: Q = A~ P for CSR A~ and row-major P with
// S columns, fused with the per-workgroup lower triangle of P^T Q
// (Alg. 1, line Xi).  A is read once for all S columns: the nonzeros of a row
// are spread over a group of G lanes as (slot, column) pairs, each slot walks
// every (G/S)-th nonzero and gathers one contiguous S-wide row of P per
// nonzero, and the slots are combined by a butterfly.  Q goes through LDS so
// that its store is a linear, coalesced copy and the Gram epilogue reads the
// tile from LDS.
#include "kernels.hpp"

#include <algorithm>

namespace mb {

template <int S, int G>
__global__ __launch_bounds__(MB_BLOCK) void k_spmm(const int32_t* __restrict__ rowptr,
                                                   const int32_t* __restrict__ colind,
                                                   const double* __restrict__ vals, int64_t n,
                                                   const double* __restrict__ P,
                                                   double* __restrict__ Q,
                                                   double* __restrict__ part,
                                                   const DevState* __restrict__ st) {
    static_assert(G % S == 0 && G <= 64 && (64 % G) == 0, "lanes per row");
    if (st && st->done) return;
    constexpr int RPP = MB_BLOCK / G;                 // rows per pass
    constexpr int T = spmm_tile(S, G);                // tile rows
    constexpr int PASSES = T / RPP;
    constexpr int SLOTS = G / S;
    constexpr int U = SLOTS >= 8 ? 1 : 8 / SLOTS;     // gathers in flight per lane
    constexpr int E = tri_count(S);
    __shared__ double sP[T * S];
    __shared__ double sQ[T * S];
    __shared__ double red[MB_BLOCK];

    const int tid = threadIdx.x;
    const int grp = tid / G, lane = tid % G;
    const int slot = lane / S, j = lane % S;
    const int64_t ntiles = (n + T - 1) / T;
    const TileRange tr = tile_range(ntiles);

    TileSums<E> gs;
    int gi[TileSums<E>::EPT], gj[TileSums<E>::EPT];
    if (part) {
        gs.init();
#pragma unroll
        for (int k = 0; k < TileSums<E>::EPT; ++k) {
            gi[k] = gj[k] = 0;
            if (gs.ent[k] >= 0) tri_ij(gs.ent[k], gi[k], gj[k]);
        }
    }

    for (int64_t tile = tr.first; tile < tr.end; tile += tr.step) {
        const int64_t r0 = tile * T;
        const int rows = (int)min((int64_t)T, n - r0);
        for (int p = 0; p < PASSES; ++p) {
            const int rl = p * RPP + grp;
            double acc = 0.0;
            if (rl < rows) {
                const int64_t r = r0 + rl;
                const int ke = rowptr[r + 1];
                // this lane's nonzeros kb+slot, kb+slot+SLOTS, ... in batches of
                // U independent gathers, added in order
                for (int k = rowptr[r] + slot; k < ke; k += U * SLOTS) {
                    int c[U];
                    double v[U], x[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int kk = k + u * SLOTS;
                        const bool ok = kk < ke;
                        c[u] = ok ? colind[kk] : 0;
                        v[u] = ok ? vals[kk] : 0.0;
                    }
#pragma unroll
                    for (int u = 0; u < U; ++u) x[u] = P[(int64_t)c[u] * S + j];
#pragma unroll
                    for (int u = 0; u < U; ++u)
                        if (k + u * SLOTS < ke) acc += v[u] * x[u];
                }
            }
#pragma unroll
            for (int off = S; off < G; off <<= 1) acc += __shfl_xor(acc, off, 64);
            if (slot == 0) sQ[rl * S + j] = acc;
        }
        if (part) {
            const double* Pt = P + r0 * S;
            for (int e = tid; e < T * S; e += MB_BLOCK) sP[e] = (e < rows * S) ? Pt[e] : 0.0;
        }
        __syncthreads();
        double* Qt = Q + r0 * S;
        for (int e = tid; e < rows * S; e += MB_BLOCK) Qt[e] = sQ[e];
        if (part) {
            gs.add_rows(rows, [&](int k, int r) { return sP[r * S + gi[k]] * sQ[r * S + gj[k]]; });
        }
        __syncthreads();
    }
    if (part) gs.finish(red, part + (int64_t)blockIdx.x * E);
}

bool spmm_valid_G(int S, int G) {
    return G >= S && G <= 64 && (G & (G - 1)) == 0;
}

int spmm_default_G(int S) {
    int G = 2 * S;
    return G > 64 ? 64 : G;
}

template <int S, int G>
static hipError_t spmm_one(int nwg, const CsrDev& A, const double* P, double* Q, double* part,
                           const DevState* st, hipStream_t stream) {
    hipLaunchKernelGGL((k_spmm<S, G>), dim3(nwg), dim3(MB_BLOCK), 0, stream, A.rowptr, A.colind,
                       A.vals, A.n, P, Q, part, st);
    return hipGetLastError();
}

template <int S>
static hipError_t spmm_s(int G, int nwg, const CsrDev& A, const double* P, double* Q,
                         double* part, const DevState* st, hipStream_t stream) {
    switch (G) {
#define MB_G(g)                                                                   \
    case g:                                                                       \
        if constexpr (g >= S) return spmm_one<S, g>(nwg, A, P, Q, part, st, stream); \
        break;
        MB_G(1) MB_G(2) MB_G(4) MB_G(8) MB_G(16) MB_G(32) MB_G(64)
#undef MB_G
    }
    return hipErrorInvalidValue;
}

hipError_t launch_spmm(int S, int G, int nwg, const CsrDev& A, const double* P, double* Q,
                       double* part, const DevState* st, hipStream_t stream) {
    if (!spmm_valid_G(S, G)) return hipErrorInvalidValue;
    switch (S) {
        case 1: return spmm_s<1>(G, nwg, A, P, Q, part, st, stream);
        case 2: return spmm_s<2>(G, nwg, A, P, Q, part, st, stream);
        case 4: return spmm_s<4>(G, nwg, A, P, Q, part, st, stream);
        case 8: return spmm_s<8>(G, nwg, A, P, Q, part, st, stream);
        case 16: return spmm_s<16>(G, nwg, A, P, Q, part, st, stream);
        case 32: return spmm_s<32>(G, nwg, A, P, Q, part, st, stream);
    }
    return hipErrorInvalidValue;
}

// residual of the original system, one row per 8-lane group: b - A x, sum of squares
__global__ __launch_bounds__(MB_BLOCK) void k_resid_csr(const int32_t* __restrict__ rowptr,
                                                        const int32_t* __restrict__ colind,
                                                        const double* __restrict__ vals, int64_t n,
                                                        const double* __restrict__ b,
                                                        const double* __restrict__ x,
                                                        double* __restrict__ part) {
    constexpr int G = 8, RPP = MB_BLOCK / G;
    __shared__ double red[MB_BLOCK];
    const int grp = threadIdx.x / G, lane = threadIdx.x % G;
    double s2 = 0.0;
    const int64_t ntiles = (n + RPP - 1) / RPP;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t r = tile * RPP + grp;
        double acc = 0.0;
        if (r < n)
            for (int k = rowptr[r] + lane; k < rowptr[r + 1]; k += G) acc += vals[k] * x[colind[k]];
#pragma unroll
        for (int off = 1; off < G; off <<= 1) acc += __shfl_xor(acc, off, 64);
        if (r < n && lane == 0) {
            const double e = b[r] - acc;
            s2 += e * e;
        }
    }
    red[threadIdx.x] = s2;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int t = 0; t < MB_BLOCK; ++t) s += red[t];
        part[blockIdx.x] = s;
    }
}

hipError_t launch_resid_csr(int nwg, const CsrDev& A, const double* b, const double* x,
                            double* part, hipStream_t s) {
    hipLaunchKernelGGL(k_resid_csr, dim3(nwg), dim3(MB_BLOCK), 0, s, A.rowptr, A.colind, A.vals,
                       A.n, b, x, part);
    return hipGetLastError();
}

// diagonal of CSR A and the scaling D = diag(sqrt(a_jj)) (Sec. 1)
__global__ void k_diag_csr(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colind,
                           const double* __restrict__ vals, int64_t n, int jacobi,
                           double* __restrict__ d, DevState* st) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * blockDim.x) {
        double a = 0.0;
        for (int k = rowptr[r]; k < rowptr[r + 1]; ++k)
            if (colind[k] == r) a += vals[k];
        double dr = 1.0;
        if (jacobi) {
            if (!(a > 0.0) || !finite_d(a)) {
                st->done = DONE_NOTSPD;
                dr = 1.0;
            } else {
                dr = sqrt(a);
            }
        }
        d[r] = dr;
    }
}

hipError_t launch_diag_csr(const CsrDev& A, int jacobi, double* d, DevState* st, hipStream_t s) {
    int nb = (int)std::min<int64_t>((A.n + MB_BLOCK - 1) / MB_BLOCK, 4096);
    hipLaunchKernelGGL(k_diag_csr, dim3(nb), dim3(MB_BLOCK), 0, s, A.rowptr, A.colind, A.vals, A.n,
                       jacobi, d, st);
    return hipGetLastError();
}

// A~ = D^-1 A D^-1 entry by entry, a_rc / (d_r d_c)
__global__ void k_scale_csr(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colind,
                            const double* __restrict__ vals, int64_t n, const double* __restrict__ d,
                            double* __restrict__ out) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * blockDim.x) {
        const double dr = d[r];
        for (int k = rowptr[r]; k < rowptr[r + 1]; ++k) out[k] = vals[k] / (dr * d[colind[k]]);
    }
}

hipError_t launch_scale_csr(const CsrDev& A, const double* d, double* vals_s, hipStream_t s) {
    int nb = (int)std::min<int64_t>((A.n + MB_BLOCK - 1) / MB_BLOCK, 8192);
    hipLaunchKernelGGL(k_scale_csr, dim3(nb), dim3(MB_BLOCK), 0, s, A.rowptr, A.colind, A.vals, A.n,
                       d, vals_s);
    return hipGetLastError();
}

}  // namespace mb

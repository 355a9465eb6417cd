// Block product of the sparse path: Q = A~ P for CSR A~ and row-major P with
// S columns, fused with the per-workgroup lower triangle of P^T Q (the Gram
// of Alg. 1's step coefficient).  Each tile of T rows is computed by
// spmm_tile (CSR slice staged through LDS, A read once for all S columns);
// the Gram is an epilogue on the LDS tiles.  (T, SL, grid) are the tuned
// shape: T rows per tile, SL lanes-groups (slots) per row.
#include "kernels.hpp"

#include <algorithm>

#include "dev_spmm.hpp"

namespace mb {

template <int S, int T, int SL>
__global__ __launch_bounds__(MB_BLOCK) void k_spmm(const int32_t* __restrict__ rowptr,
                                                   const int32_t* __restrict__ colind,
                                                   const double* __restrict__ vals, int64_t n,
                                                   const double* __restrict__ P,
                                                   double* __restrict__ Q,
                                                   double* __restrict__ part,
                                                   const DevState* __restrict__ st) {
    using TL = SpmmTile<S, T, SL>;
    if (st && st->done) return;
    constexpr int E = tri_count(S);
    constexpr bool MF = S >= 8;                 // Gram on the matrix cores
    __shared__ int32_t sRp[T + 1];
    __shared__ int32_t sC[TL::NZC];
    __shared__ double sV[TL::NZC];
    __shared__ double sQ[T * S];
    __shared__ double sP[MF ? 1 : T * S];
    __shared__ double red[MB_BLOCK];
    const int tid = threadIdx.x;
    const int64_t ntiles = (n + T - 1) / T;
    const TileRange tr = tile_range(ntiles);

    TileSums<E> gs;
    GramMfma<S> gm;
    int gi[TileSums<E>::EPT], gj[TileSums<E>::EPT];
    if (part) {
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
    }
    for (int64_t tile = tr.first; tile < tr.end; tile += tr.step) {
        const int64_t r0 = tile * T;
        const int rows = (int)min((int64_t)T, n - r0);
        spmm_tile<S, T, SL>(rowptr, colind, vals, P, r0, rows, sRp, sC, sV, sQ);
        const double* Pt = P + r0 * S;
        if (part && !MF)
            for (int e = tid; e < T * S; e += MB_BLOCK) sP[e] = (e < rows * S) ? Pt[e] : 0.0;
        double* Qt = Q + r0 * S;
        for (int e = tid; e < rows * S; e += MB_BLOCK) Qt[e] = sQ[e];
        if (part) {
            if constexpr (MF) {
                gm.add_tile(rows, [&](int r, int c) { return Pt[r * S + c]; },
                            [&](int r, int c) { return sQ[r * S + c]; });
            } else {
                __syncthreads();
                gs.add_rows(rows, [&](int k, int r) { return sP[r * S + gi[k]] * sQ[r * S + gj[k]]; });
            }
        }
        __syncthreads();
    }
    if (part) {
        if constexpr (MF) gm.finish(sQ, part + (int64_t)blockIdx.x * E);
        else gs.finish(red, part + (int64_t)blockIdx.x * E);
    }
}

// ---- shapes compiled per width: tile rows x slots
bool spmm_valid_shape(int S, int T, int SL) {
    if (!(SL == 1 || SL == 2) || S * SL > 64) return false;
    if (!(T == 32 || T == 64 || T == 128 || T == 256)) return false;
    return T * S <= 1024;
}

void spmm_default_shape(int S, int* T, int* SL) {
    *SL = 1;
    *T = S <= 4 ? 128 : (S == 8 ? 64 : 32);
}

template <int S, int T, int SL>
static hipError_t spmm_one(int nwg, const CsrDev& A, const double* P, double* Q, double* part,
                           const DevState* st, hipStream_t stream) {
    hipLaunchKernelGGL((k_spmm<S, T, SL>), dim3(nwg), dim3(MB_BLOCK), 0, stream, A.rowptr,
                       A.colind, A.vals, A.n, P, Q, part, st);
    return hipGetLastError();
}

template <int S, int T>
static hipError_t spmm_t(int SL, int nwg, const CsrDev& A, const double* P, double* Q,
                         double* part, const DevState* st, hipStream_t stream) {
    if constexpr (T * S <= 1024) {
        if (SL == 1) return spmm_one<S, T, 1>(nwg, A, P, Q, part, st, stream);
        if constexpr (S * 2 <= 64)
            if (SL == 2) return spmm_one<S, T, 2>(nwg, A, P, Q, part, st, stream);
    }
    return hipErrorInvalidValue;
}

template <int S>
static hipError_t spmm_s(int T, int SL, int nwg, const CsrDev& A, const double* P, double* Q,
                         double* part, const DevState* st, hipStream_t stream) {
    switch (T) {
        case 32: return spmm_t<S, 32>(SL, nwg, A, P, Q, part, st, stream);
        case 64: return spmm_t<S, 64>(SL, nwg, A, P, Q, part, st, stream);
        case 128: return spmm_t<S, 128>(SL, nwg, A, P, Q, part, st, stream);
        case 256: return spmm_t<S, 256>(SL, nwg, A, P, Q, part, st, stream);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_spmm(int S, int T, int SL, int nwg, const CsrDev& A, const double* P, double* Q,
                       double* part, const DevState* st, hipStream_t stream) {
    if (!spmm_valid_shape(S, T, SL)) return hipErrorInvalidValue;
    switch (S) {
        case 1: return spmm_s<1>(T, SL, nwg, A, P, Q, part, st, stream);
        case 2: return spmm_s<2>(T, SL, nwg, A, P, Q, part, st, stream);
        case 4: return spmm_s<4>(T, SL, nwg, A, P, Q, part, st, stream);
        case 8: return spmm_s<8>(T, SL, nwg, A, P, Q, part, st, stream);
        case 16: return spmm_s<16>(T, SL, nwg, A, P, Q, part, st, stream);
        case 32: return spmm_s<32>(T, SL, nwg, A, P, Q, part, st, stream);
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

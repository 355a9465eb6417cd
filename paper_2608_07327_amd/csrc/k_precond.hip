// Block-Jacobi preconditioner setup: the inverse of every diagonal block of
// bs consecutive rows of the scaled matrix (the preconditioner M of the
// preconditioned form that Sec. 2 says the method admits).
//
// One block per bs lanes: lane i owns row i of its block.  The block is
// staged in LDS (a partial last block is padded with identity rows and
// columns, so every block runs the same bs steps), factored A_k = L L^T by a
// right-looking Cholesky, each lane forms one column of L^-1 by forward
// substitution, and each lane then writes row i of A_k^-1 = L^-T L^-1.
#include <algorithm>

#include "kernels.hpp"

namespace mb {

constexpr int BJ_THREADS = 128;

template <int BS>
__global__ __launch_bounds__(BJ_THREADS) void k_bjac_setup(int64_t n, const int32_t* __restrict__ rowptr,
                                                           const int32_t* __restrict__ colind,
                                                           const double* __restrict__ vals,
                                                           const double* __restrict__ dense,
                                                           int64_t lda, double* __restrict__ inv,
                                                           DevState* __restrict__ st) {
    constexpr int NB = BJ_THREADS / BS;  // blocks per workgroup
    __shared__ double a[NB][BS][BS + 1];
    const int t = threadIdx.x, lb = t / BS, i = t % BS;
    const int64_t nblk = (n + BS - 1) / BS;
    for (int64_t k0 = (int64_t)blockIdx.x * NB; k0 < nblk; k0 += (int64_t)gridDim.x * NB) {
        const int64_t k = k0 + lb;
        const int64_t lo = k * BS, r = lo + i;
        const bool real = k < nblk && r < n;
        double (*A)[BS + 1] = a[lb];
#pragma unroll
        for (int c = 0; c < BS; ++c) A[i][c] = (!real && c == i) ? 1.0 : 0.0;
        if (real) {
            if (dense) {
                for (int c = 0; c < BS; ++c)
                    if (lo + c < n) A[i][c] = dense[(lo + c) * lda + r];
            } else {
                for (int32_t e = rowptr[r]; e < rowptr[r + 1]; ++e) {
                    const int64_t c = (int64_t)colind[e] - lo;
                    if (c >= 0 && c < BS) A[i][c] += vals[e];
                }
            }
        }
        __syncthreads();
        // right-looking Cholesky, lower factor in place
        bool ok = true;
#pragma unroll 1
        for (int kk = 0; kk < BS; ++kk) {
            const double piv = A[kk][kk];
            ok = ok && piv > 0.0 && finite_d(piv);
            const double lkk = sqrt(piv);
            __syncthreads();
            if (i == kk) A[kk][kk] = lkk;
            if (i > kk) A[i][kk] = A[i][kk] / lkk;
            __syncthreads();
            if (i > kk) {
                const double lik = A[i][kk];
                for (int jj = kk + 1; jj <= i; ++jj) A[i][jj] -= lik * A[jj][kk];
            }
            __syncthreads();
        }
        if (!ok && real && i == 0) st->done = DONE_NOTSPD;
        // column i of L^-1 (rows >= i)
        double x[BS];
#pragma unroll
        for (int rr = 0; rr < BS; ++rr) {
            double v = (rr == i) ? 1.0 : 0.0;
#pragma unroll
            for (int c = 0; c < rr; ++c)
                if (c >= i) v -= A[rr][c] * x[c];
            x[rr] = (rr < i) ? 0.0 : v / A[rr][rr];
        }
        __syncthreads();
#pragma unroll
        for (int rr = 0; rr < BS; ++rr)
            if (rr >= i) A[rr][i] = x[rr];
        __syncthreads();
        // row i of L^-T L^-1: sum over k >= max(i, j) of Linv[k][i] Linv[k][j]
        if (real) {
            double* out = inv + r * BS;
#pragma unroll
            for (int j = 0; j < BS; ++j) {
                double v = 0.0;
#pragma unroll
                for (int kk = 0; kk < BS; ++kk)
                    if (kk >= i && kk >= j) v += A[kk][i] * A[kk][j];
                out[j] = (lo + j < n) ? v : 0.0;
            }
        }
        __syncthreads();
    }
}

template <int BS>
static hipError_t bjac_launch(int64_t n, const int32_t* rowptr, const int32_t* colind,
                              const double* vals, const double* dense, int64_t lda, double* inv,
                              DevState* st, hipStream_t s) {
    constexpr int NB = BJ_THREADS / BS;
    const int64_t nblk = (n + BS - 1) / BS;
    const int g = (int)std::max<int64_t>(1, std::min<int64_t>((nblk + NB - 1) / NB, 8192));
    hipLaunchKernelGGL(k_bjac_setup<BS>, dim3(g), dim3(BJ_THREADS), 0, s, n, rowptr, colind, vals,
                       dense, lda, inv, st);
    return hipGetLastError();
}

static hipError_t bjac_dispatch(int bs, int64_t n, const int32_t* rowptr, const int32_t* colind,
                                const double* vals, const double* dense, int64_t lda, double* inv,
                                DevState* st, hipStream_t s) {
    switch (bs) {
        case 4: return bjac_launch<4>(n, rowptr, colind, vals, dense, lda, inv, st, s);
        case 8: return bjac_launch<8>(n, rowptr, colind, vals, dense, lda, inv, st, s);
        case 16: return bjac_launch<16>(n, rowptr, colind, vals, dense, lda, inv, st, s);
        case 32: return bjac_launch<32>(n, rowptr, colind, vals, dense, lda, inv, st, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_bjac_setup_csr(int bs, const CsrDev& A, double* inv, DevState* st,
                                 hipStream_t s) {
    return bjac_dispatch(bs, A.n, A.rowptr, A.colind, A.vals, nullptr, 0, inv, st, s);
}

hipError_t launch_bjac_setup_dense(int bs, int64_t n, const double* A, int64_t lda, double* inv,
                                   DevState* st, hipStream_t s) {
    return bjac_dispatch(bs, n, nullptr, nullptr, nullptr, A, lda, inv, st, s);
}

}  // namespace mb

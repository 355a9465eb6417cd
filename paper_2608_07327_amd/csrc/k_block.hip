// Streaming n x S kernels of one MBPCG iteration, the setup and the
// termination of Algorithm 1, and the Chronopoulos-Gear CG baseline.
//
// Every kernel walks its rows in tiles of T rows.  A tile of a row-major
// n x S block is one contiguous run of T*S doubles, so blocks that are needed
// whole-row (P, Q, V) are staged through LDS with a linear coalesced copy, and
// the element-wise blocks (X~, R, W) are read and written in place with the
// same linear layout.  Each thread owns one column j of the tile, which keeps
// the column j of the s x s coefficients in registers for the whole kernel.
#include "dev_dd.hpp"
#include "kernels.hpp"

#include <hip/hip_bf16.h>

namespace mb {

template <int S>
struct Tiles {
    static constexpr int RPP = MB_BLOCK / S;   // rows per pass (one thread per column)
    static constexpr int T = stream_tile(S);   // 4 passes per tile
};

// For S <= 16 the direction kernel stores only P, and the update kernel forms
// W = V_prev M_prev from the previous V (kept in the W buffer) and the
// previous M: one n x S block less written per iteration.  At S = 32 the
// extra column of M does not fit the update kernel's registers, and the
// direction kernel stores W as before.
template <int S>
constexpr bool lazy_w() { return S <= 16; }

// For S <= 16 the direction update also applies X~ += P alpha (the same sum
// in the same order): it reads the P block anyway, so the update kernel need
// not read it (one n x S block less per iteration).  At S = 32 the alpha
// column would not fit the direction kernel's registers.
template <int S>
constexpr bool xt_in_dir() { return S <= 16; }

// Row rl of a tile of M^-1 X for the block-Jacobi preconditioner with blocks
// of BS rows: the tile starts at a multiple of BS (T is one), so the block of
// row r0 + rl is the tile rows (rl / BS) * BS ..; sX holds the tile of X
// (zero beyond n), inv row r the matching row of the block's inverse.
template <int S, int BS>
__device__ __forceinline__ double bj_row(const double* __restrict__ inv, int64_t r,
                                         const double* sX, int rl, int j) {
    static_assert(BS > 0 && Tiles<S>::T % BS == 0, "tiles must hold whole blocks");
    const double* iv = inv + r * BS;
    const int b0 = (rl / BS) * BS;
    double y = 0.0;
#pragma unroll
    for (int c = 0; c < BS; ++c) y += iv[c] * sX[(b0 + c) * S + j];
    return y;
}

// The same for the RT rows rl0 + k*RPP of a thread (k < RT), into y[k]: the
// inverse rows are loaded 4 entries at a time for every row before they are
// used, so the rows' loads overlap (entries added in the same order as
// bj_row; rows at or beyond `rows` read row r0 and are not used).
template <int S, int BS, int RT, int RPP>
__device__ __forceinline__ void bj_rows(const double* __restrict__ inv, int64_t r0, int rows,
                                        const double* sX, int rl0, int j, double* y) {
    static_assert(BS > 0 && Tiles<S>::T % BS == 0, "tiles must hold whole blocks");
    constexpr int G = BS < 4 ? BS : 4;
#pragma unroll
    for (int k = 0; k < RT; ++k) y[k] = 0.0;
    // a rolled loop over the groups, so that only one group's loads are in
    // registers at a time
#pragma unroll 1
    for (int c0 = 0; c0 < BS; c0 += G) {
        double iv[RT][G];
#pragma unroll
        for (int k = 0; k < RT; ++k) {
            const int rl = rl0 + k * RPP;
            const double* row = inv + (r0 + (rl < rows ? rl : 0)) * BS + c0;
#pragma unroll
            for (int c = 0; c < G; ++c) iv[k][c] = row[c];
        }
#pragma unroll
        for (int k = 0; k < RT; ++k) {
            const int b0 = ((rl0 + k * RPP) / BS) * BS;
#pragma unroll
            for (int c = 0; c < G; ++c) y[k] += iv[k][c] * sX[(b0 + c0 + c) * S + j];
        }
    }
}

// ---------------------------------------------------------------------------
// K_B: X~ += P alpha, R -= Q alpha, the column norms behind h, and
// V = W - Q Xi with the Gram V^T V (first half of the Cholesky QR).
//   X~ += P alpha,  R -= Q alpha,  V = W - Q Xi  (V overwrites W),
//   partial lower triangle of V^T V and nu_j = sum_r (d_r R_rj)^2.
// With lazy_w, W = V_prev M_prev is formed here from the W buffer (which
// holds the previous V) and the previous Cholesky-QR M.  With xt_in_dir the
// X~ update is left to the direction kernel of the same iteration.
// ---------------------------------------------------------------------------
// BS > 0 (preconditioned form): also Y = M^-1 V into Yp, and the Gram is V^T Y.
template <int S, int BS>
__global__ __launch_bounds__(MB_BLOCK) void k_update(int64_t n, const double* __restrict__ P,
                                                     const double* __restrict__ Q,
                                                     double* __restrict__ Xt,
                                                     double* __restrict__ R,
                                                     double* __restrict__ W,
                                                     const double* __restrict__ d,
                                                     double* __restrict__ part,
                                                     const DevState* __restrict__ st,
                                                     const double* __restrict__ inv,
                                                     double* __restrict__ Yp) {
    if (st->done) return;
    constexpr int RPP = Tiles<S>::RPP, T = Tiles<S>::T;
    constexpr int E = tri_count(S);
    constexpr bool LW = lazy_w<S>();
    constexpr bool XD = xt_in_dir<S>();   // X~ is updated by the direction kernel
    __shared__ double sP[XD ? 1 : T * S];
    __shared__ double sQ[T * S];
    __shared__ double sV[T * S];
    __shared__ double sY[BS > 0 ? T * S : 1];
    __shared__ double sW[LW ? T * S : 1];
    __shared__ double red[MB_BLOCK];
    const int t = threadIdx.x, j = t % S, rl0 = t / S;
    double al[S], xi[S], mp[LW ? S : 1];
#pragma unroll
    for (int l = 0; l < S; ++l) {
        al[l] = st->alpha[l * MB_SM + j];
        xi[l] = st->Xi[l * MB_SM + j];
        if constexpr (LW) mp[l] = st->M[l * MB_SM + j];   // M of the previous Cholesky QR
    }
    constexpr bool MF = S >= 8;   // V^T V on the matrix cores
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
    double nu = 0.0;
    const int64_t ntiles = (n + T - 1) / T;
    const TileRange tr = tile_range(ntiles);
    for (int64_t tile = tr.first; tile < tr.end; tile += tr.step) {
        const int64_t r0 = tile * T;
        const int rows = (int)min((int64_t)T, n - r0);
        // every load of the tile (the P, Q and previous-V tiles and this
        // thread's X~, R and d entries) is issued before the first LDS store
        constexpr int RT = T / RPP;   // rows per thread
        Stage<T * S> stp, stq, stw;
        if constexpr (!XD) stp.load(P + r0 * S, rows * S);
        stq.load(Q + r0 * S, rows * S);
        if constexpr (LW) stw.load(W + r0 * S, rows * S);   // the previous V
        // (S = 32: the row entries are loaded where they are used, for the
        // registers)
        constexpr bool PF = S <= 16;
        double xo[XD ? 1 : RT], ro[RT], wo[LW ? 1 : RT], dv[RT];
        auto row_loads = [&](int k) {
            const int rl = rl0 + k * RPP;
            const int64_t g = (r0 + (rl < rows ? rl : 0)) * S + j;
            if constexpr (!XD) xo[k] = stream_load(Xt + g);
            ro[k] = stream_load(R + g);
            if constexpr (!LW) wo[k] = W[g];
            dv[k] = d[r0 + (rl < rows ? rl : 0)];
        };
        if constexpr (PF) {
#pragma unroll
            for (int k = 0; k < RT; ++k) row_loads(k);
        }
        if constexpr (!XD) stp.store(sP);
        stq.store(sQ);
        if constexpr (LW) stw.store(sW);
        __syncthreads();
#pragma unroll
        for (int k = 0; k < RT; ++k) {
            const int rl = rl0 + k * RPP;
            double v = 0.0;
            if constexpr (!PF) row_loads(k);
            if (rl < rows) {
                const int64_t g = (r0 + rl) * S + j;
                double tx = 0.0, trr = 0.0, tv = 0.0;
#pragma unroll
                for (int l = 0; l < S; ++l) {
                    const double q = sQ[rl * S + l];
                    if constexpr (!XD) tx += sP[rl * S + l] * al[l];
                    trr += q * al[l];
                    tv += q * xi[l];
                }
                const double rn = ro[k] - trr;
                double w;
                if constexpr (LW) {
                    w = 0.0;
#pragma unroll
                    for (int l = 0; l < S; ++l) w += sW[rl * S + l] * mp[l];
                } else {
                    w = wo[k];
                }
                v = w - tv;
                if constexpr (!XD) stream_store(Xt + g, xo[k] + tx);
                stream_store(R + g, rn);
                W[g] = v;
                const double dr = dv[k] * rn;
                nu += dr * dr;
            }
            sV[rl * S + j] = v;
        }
        __syncthreads();
        if constexpr (BS > 0) {
            double y[RT];
            bj_rows<S, BS, RT, RPP>(inv, r0, rows, sV, rl0, j, y);
#pragma unroll
            for (int k = 0; k < RT; ++k) {
                const int rl = rl0 + k * RPP;
                if (rl < rows) Yp[(r0 + rl) * S + j] = y[k];
                sY[rl * S + j] = rl < rows ? y[k] : 0.0;
            }
            __syncthreads();
        }
        const double* sG = BS > 0 ? sY : sV;   // second Gram operand
        if constexpr (MF)
            gm.add_tile(rows, [&](int r, int c) { return sV[r * S + c]; },
                        [&](int r, int c) { return sG[r * S + c]; });
        else
            gs.add_rows(rows, [&](int k, int r) { return sV[r * S + gi[k]] * sG[r * S + gj[k]]; });
        __syncthreads();
    }
    double* out = part + (int64_t)blockIdx.x * (E + S);
    if constexpr (MF) gm.finish(sV, out);
    else gs.finish(red, out);
    __syncthreads();
    red[t] = nu;
    column_sums<S>(red);
    if (t < S) out[E + t] = red[t];
}

// ---------------------------------------------------------------------------
// K_C: W = V M (second half of the Cholesky QR) and P = W + P Z^T.
//   W = V M  (M = inverse of the kept Cholesky factor),  P = W + P Z^T.
// W is stored only where the update kernel does not form it itself (S = 32,
// lazy_w); otherwise the W buffer keeps V for the next update.
// FIRST: the first direction block P0 = W0.  Optionally also writes P rounded to FP32 or BF16
// for the low-precision dense product.
// PREC (preconditioned form): P = Yp M + P Z^T with Yp = M^-1 V.
// ---------------------------------------------------------------------------
template <int S, int FIRST, int LO, int PREC>
__global__ __launch_bounds__(MB_BLOCK) void k_dirupdate(int64_t n, double* __restrict__ W,
                                                        double* __restrict__ P,
                                                        void* __restrict__ Plo,
                                                        const DevState* __restrict__ st,
                                                        const double* __restrict__ Yp,
                                                        double* __restrict__ Xt) {
    // XD: also X~ += P alpha of this iteration, from the P read here (P is
    // still the block the update kernel's iteration used).  When the QR tail
    // has just stopped the loop, only that X~ update is left to do.
    constexpr bool XD = !FIRST && xt_in_dir<S>();
    const int stop = st->done;
    if (stop && !(XD && st->xt_pending)) return;
    // after a resumed Cholesky QR this iteration's X~ update is already done
    const bool xd = XD && !st->xt_skip;
    constexpr int RPP = Tiles<S>::RPP, T = Tiles<S>::T;
    constexpr int RT = T / RPP;   // rows per thread
    __shared__ double sV[T * S];
    __shared__ double sP[T * S];
    __shared__ double sY[PREC ? T * S : 1];
    const int t = threadIdx.x, j = t % S, rl0 = t / S;
    double m[S], z[S], al[XD ? S : 1];
#pragma unroll
    for (int l = 0; l < S; ++l) {
        m[l] = st->M[l * MB_SM + j];
        z[l] = st->Z[j * MB_SM + l];
        if constexpr (XD) al[l] = st->alpha[l * MB_SM + j];
    }
    const int64_t ntiles = (n + T - 1) / T;
    const TileRange tr = tile_range(ntiles);
    for (int64_t tile = tr.first; tile < tr.end; tile += tr.step) {
        const int64_t r0 = tile * T;
        const int rows = (int)min((int64_t)T, n - r0);
        // all loads of the tile before the first LDS store
        Stage<T * S> stv, stp, sty;
        if (!stop) stv.load(W + r0 * S, rows * S);
        if (!FIRST) stp.load(P + r0 * S, rows * S);
        if (PREC && !stop) sty.load(Yp + r0 * S, rows * S);
        double xo[XD ? RT : 1];
        if constexpr (XD) {
            if (xd) {
#pragma unroll
                for (int k = 0; k < RT; ++k) {
                    const int rl = rl0 + k * RPP;
                    xo[k] = stream_load(Xt + (r0 + (rl < rows ? rl : 0)) * S + j);
                }
            }
        }
        if (!stop) stv.store(sV);
        if (!FIRST) stp.store(sP);
        if (PREC && !stop) sty.store(sY);
        __syncthreads();
#pragma unroll
        for (int k = 0; k < RT; ++k) {
            const int rl = rl0 + k * RPP;
            if (rl >= rows) continue;
            const int64_t g = (r0 + rl) * S + j;
            if constexpr (XD) {
                if (xd) {
                    double tx = 0.0;
#pragma unroll
                    for (int l = 0; l < S; ++l) tx += sP[rl * S + l] * al[l];
                    stream_store(Xt + g, xo[k] + tx);
                }
            }
            if (stop) continue;
            double w = 0.0;
#pragma unroll
            for (int l = 0; l < S; ++l) w += sV[rl * S + l] * m[l];
            double p = w;
            if (PREC) {
                double yw = 0.0;
#pragma unroll
                for (int l = 0; l < S; ++l) yw += sY[rl * S + l] * m[l];
                p = yw;
            }
            if (!FIRST) {
                double acc = 0.0;
#pragma unroll
                for (int l = 0; l < S; ++l) acc += sP[rl * S + l] * z[l];
                p = p + acc;
            }
            if (!lazy_w<S>()) W[g] = w;
            P[g] = p;
            if (LO == DENSE_F32) static_cast<float*>(Plo)[lo_pindex(LO, r0 + rl, j, S)] = (float)p;
            if (LO == DENSE_BF16)
                static_cast<__hip_bfloat16*>(Plo)[lo_pindex(LO, r0 + rl, j, S)] = __double2bfloat16(p);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Setup (Alg. 1, from B = [b ... b] to the first direction block P0)
// ---------------------------------------------------------------------------
// b~ = D^-1 b; partial sums of b^2 and b~^2
__global__ __launch_bounds__(MB_BLOCK) void k_rhs(int64_t n, const double* __restrict__ b,
                                                  const double* __restrict__ d,
                                                  double* __restrict__ bbar,
                                                  double* __restrict__ part) {
    __shared__ double red[2 * MB_BLOCK];
    double s0 = 0.0, s1 = 0.0;
    for (int64_t r = blockIdx.x * (int64_t)MB_BLOCK + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * MB_BLOCK) {
        const double v = b[r], vb = v / d[r];
        bbar[r] = vb;
        s0 += v * v;
        s1 += vb * vb;
    }
    red[threadIdx.x] = s0;
    red[MB_BLOCK + threadIdx.x] = s1;
    __syncthreads();
    if (threadIdx.x < 2) {
        double s = 0.0;
        for (int k = 0; k < MB_BLOCK; ++k) s += red[threadIdx.x * MB_BLOCK + k];
        part[blockIdx.x * 2 + threadIdx.x] = s;
    }
}

// U_rj = 2 u - 1 with u the top 53 bits of SplitMix64 output number j*n + r
// (Alg. 1, the random block U: iid Uniform(-1, 1)); padded columns are zero.
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t k) {
    uint64_t z = seed + (k + 1u) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

template <int S>
__global__ void k_uniform(int64_t n, int s, uint64_t seed, double* __restrict__ U) {
    const int64_t total = n * S;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = e / S;
        const int j = (int)(e % S);
        double v = 0.0;
        if (j < s) {
            const uint64_t z = splitmix64_at(seed, (uint64_t)j * (uint64_t)n + (uint64_t)r);
            v = 2.0 * ((double)(z >> 11) * 0x1.0p-53) - 1.0;
        }
        U[e] = v;
    }
}

template <int S>
__global__ void k_pad_block(int64_t n, int s, const double* __restrict__ in, double* __restrict__ U) {
    const int64_t total = n * S;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = e / S;
        const int j = (int)(e % S);
        U[e] = j < s ? in[r * s + j] : 0.0;
    }
}

// partial sums over rows of sum_j Y_rj^2 (||A U||_F^2)
template <int S>
__global__ __launch_bounds__(MB_BLOCK) void k_ynorm(int64_t n, const double* __restrict__ Y,
                                                    double* __restrict__ part) {
    __shared__ double red[MB_BLOCK];
    double s2 = 0.0;
    for (int64_t r = blockIdx.x * (int64_t)MB_BLOCK + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * MB_BLOCK) {
        double a = 0.0;
#pragma unroll
        for (int j = 0; j < S; ++j) a += Y[r * S + j] * Y[r * S + j];
        s2 += a;
    }
    red[threadIdx.x] = s2;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int k = 0; k < MB_BLOCK; ++k) s += red[k];
        part[blockIdx.x] = s;
    }
}

// X0 = gamma U;  R0 = B~ - gamma (A U);  X~0 = 0   (initial guess and residual)
template <int S>
__global__ void k_init(int64_t n, int s, const double* __restrict__ U, const double* __restrict__ Y,
                       const double* __restrict__ bbar, double* __restrict__ X0,
                       double* __restrict__ Xt, double* __restrict__ R,
                       const DevState* __restrict__ st) {
    if (st->done) return;
    const double g = st->gamma;
    const int64_t total = n * S;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(e % S);
        X0[e] = g * U[e];
        Xt[e] = 0.0;
        R[e] = j < s ? bbar[e / S] - g * Y[e] : 0.0;
    }
}

// partial lower triangle of X^T X and nu_j = sum_r (d_r X_rj)^2 (same layout as k_update)
// BS > 0 (preconditioned form): also Y = M^-1 X into Yp, and the Gram is X^T Y.
template <int S, int BS>
__global__ __launch_bounds__(MB_BLOCK) void k_gram_nu(int64_t n, const double* __restrict__ X,
                                                      const double* __restrict__ d,
                                                      double* __restrict__ part,
                                                      const double* __restrict__ inv,
                                                      double* __restrict__ Yp) {
    constexpr int RPP = Tiles<S>::RPP, T = Tiles<S>::T;
    constexpr int E = tri_count(S);
    __shared__ double sX[T * S];
    __shared__ double sY[BS > 0 ? T * S : 1];
    __shared__ double red[MB_BLOCK];
    const int t = threadIdx.x, j = t % S, rl0 = t / S;
    constexpr bool MF = S >= 8;
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
    double nu = 0.0;
    const int64_t ntiles = (n + T - 1) / T;
    const TileRange tr = tile_range(ntiles);
    for (int64_t tile = tr.first; tile < tr.end; tile += tr.step) {
        const int64_t r0 = tile * T;
        const int rows = (int)min((int64_t)T, n - r0);
        for (int e = t; e < T * S; e += MB_BLOCK) sX[e] = e < rows * S ? X[r0 * S + e] : 0.0;
        __syncthreads();
        for (int rl = rl0; rl < rows; rl += RPP) {
            const double v = d[r0 + rl] * sX[rl * S + j];
            nu += v * v;
        }
        if constexpr (BS > 0) {
            for (int rl = rl0; rl < T; rl += RPP) {
                double y = 0.0;
                if (rl < rows) {
                    y = bj_row<S, BS>(inv, r0 + rl, sX, rl, j);
                    Yp[(r0 + rl) * S + j] = y;
                }
                sY[rl * S + j] = y;
            }
            __syncthreads();
        }
        const double* sG = BS > 0 ? sY : sX;
        if constexpr (MF)
            gm.add_tile(rows, [&](int r, int c) { return sX[r * S + c]; },
                        [&](int r, int c) { return sG[r * S + c]; });
        else
            gs.add_rows(rows, [&](int k, int r) { return sX[r * S + gi[k]] * sG[r * S + gj[k]]; });
        __syncthreads();
    }
    double* out = part + (int64_t)blockIdx.x * (E + S);
    if constexpr (MF) gm.finish(sX, out);
    else gs.finish(red, out);
    __syncthreads();
    red[t] = nu;
    column_sums<S>(red);
    if (t < S) out[E + t] = red[t];
}

// ---------------------------------------------------------------------------
// Termination (least-squares combination of Alg. 1, Proposition 1): the
// double-double Gram of [B^, b] with B^ = B - D R formed entry by entry as
// b_r - (d_r R_rj) (one pass over R); columns j >= s are zero.
// ---------------------------------------------------------------------------
template <int S>
__global__ __launch_bounds__(MB_BLOCK) void k_ls_gram(int64_t n, const double* __restrict__ b,
                                                      const double* __restrict__ R,
                                                      const double* __restrict__ d,
                                                      double* __restrict__ part,
                                                      const DevState* __restrict__ st) {
    constexpr int NC = S + 1;
    constexpr int T = 64;
    constexpr int E = tri_count(NC);
    __shared__ double sM[T * NC];
    __shared__ double red[2 * MB_BLOCK];
    const int t = threadIdx.x;
    const int s = st->s;
    TileSumsDD<E> gs;
    gs.init();
    int gi[TileSumsDD<E>::EPT], gj[TileSumsDD<E>::EPT];
#pragma unroll
    for (int k = 0; k < TileSumsDD<E>::EPT; ++k) {
        gi[k] = gj[k] = 0;
        if (gs.ent[k] >= 0) tri_ij(gs.ent[k], gi[k], gj[k]);
    }
    const int64_t ntiles = (n + T - 1) / T;
    const TileRange tr = tile_range(ntiles);
    for (int64_t tile = tr.first; tile < tr.end; tile += tr.step) {
        const int64_t r0 = tile * T;
        const int rows = (int)min((int64_t)T, n - r0);
        for (int e = t; e < T * S; e += MB_BLOCK) {
            const int rl = e / S, j = e % S;
            sM[rl * NC + j] = (rl < rows && j < s) ? bhat_entry(b[r0 + rl], d[r0 + rl], R[r0 * S + e])
                                                   : 0.0;
        }
        for (int rl = t; rl < T; rl += MB_BLOCK) sM[rl * NC + S] = rl < rows ? b[r0 + rl] : 0.0;
        __syncthreads();
        gs.add_rows(rows, [&](int k, int r) {
            return make_double2(sM[r * NC + gi[k]], sM[r * NC + gj[k]]);
        });
        __syncthreads();
    }
    gs.finish(red, part + (int64_t)blockIdx.x * 2 * E);
}

// x = D^-1 (X~ + X0) c^ and r = b - B^ c^ (each sum over the columns in
// column order, every product and sum rounded as written), partial ||r||^2
template <int S>
__global__ __launch_bounds__(MB_BLOCK) void k_ls_apply(int64_t n, const double* __restrict__ Xt,
                                                       const double* __restrict__ X0,
                                                       const double* __restrict__ R,
                                                       const double* __restrict__ b,
                                                       const double* __restrict__ d,
                                                       double* __restrict__ x,
                                                       double* __restrict__ part,
                                                       const DevState* __restrict__ st) {
#pragma clang fp contract(off)
    __shared__ double red[MB_BLOCK];
    double c[S];
#pragma unroll
    for (int j = 0; j < S; ++j) c[j] = st->chat[j];
    const int s = st->s;
    double s2 = 0.0;
    for (int64_t r = blockIdx.x * (int64_t)MB_BLOCK + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * MB_BLOCK) {
        double ax = 0.0, ab = 0.0;
        const double dr = d[r], br = b[r];
#pragma unroll
        for (int j = 0; j < S; ++j) {
            if (j < s) {
                ax += (Xt[r * S + j] + X0[r * S + j]) * c[j];
                ab += bhat_entry(br, dr, R[r * S + j]) * c[j];
            }
        }
        x[r] = ax / dr;
        const double res = br - ab;
        s2 += res * res;
    }
    red[threadIdx.x] = s2;
    __syncthreads();
    if (threadIdx.x == 0) {
        double v = 0.0;
        for (int k = 0; k < MB_BLOCK; ++k) v += red[k];
        part[blockIdx.x] = v;
    }
}

// fallback to the best column: x = D^-1 (X~ + X0)_h when the combination is
// not accepted (force: unconditionally, for the true-residual comparison)
template <int S>
__global__ void k_select(int64_t n, const double* __restrict__ Xt, const double* __restrict__ X0,
                         const double* __restrict__ d, double* __restrict__ x,
                         const DevState* __restrict__ st, int force) {
    if (!force && st->accepted) return;
    const int h = st->h;
    const bool ready = st->ready;  // a system that failed in setup returns x = 0
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * blockDim.x)
        x[r] = ready ? (Xt[r * S + h] + X0[r * S + h]) / d[r] : 0.0;
}

// ---------------------------------------------------------------------------
// Chronopoulos-Gear CG: p = r + beta p; s = w + beta s; x += alpha p;
// r -= alpha s; partials of ||D r||^2 and r^T r.
// ---------------------------------------------------------------------------
__global__ void k_cg_init(int64_t n, const double* __restrict__ bbar, double* __restrict__ x,
                          double* __restrict__ r, double* __restrict__ p, double* __restrict__ sv) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        x[i] = 0.0;
        r[i] = bbar[i];
        p[i] = 0.0;
        sv[i] = 0.0;
    }
}

// Rows go in chunks of MB_BLOCK (one per workgroup and pass), so a chunk holds
// whole preconditioner blocks.  BS > 0 (preconditioned form): p = u + beta p,
// then u = M^-1 r from the new r (into u), partials (||D r||^2, r^T u).
template <int BS>
__global__ __launch_bounds__(MB_BLOCK) void k_cg_update(int64_t n, double* __restrict__ p,
                                                        double* __restrict__ sv,
                                                        double* __restrict__ x,
                                                        double* __restrict__ r,
                                                        const double* __restrict__ w,
                                                        const double* __restrict__ d,
                                                        double* __restrict__ part,
                                                        const DevState* __restrict__ st,
                                                        const double* __restrict__ inv,
                                                        double* __restrict__ u) {
    static_assert(MB_BLOCK % (BS > 0 ? BS : 1) == 0, "chunks must hold whole blocks");
    if (st->done) return;
    __shared__ double red[2 * MB_BLOCK];
    __shared__ double sR[BS > 0 ? MB_BLOCK : 1];
    const int t = threadIdx.x;
    const double alpha = st->cg_alpha, beta = st->cg_beta;
    double e2 = 0.0, g2 = 0.0;
    for (int64_t base = blockIdx.x * (int64_t)MB_BLOCK; base < n;
         base += (int64_t)gridDim.x * MB_BLOCK) {
        const int64_t i = base + t;
        const bool in = i < n;
        double rn = 0.0;
        if (in) {
            const double pn = (BS > 0 ? u[i] : r[i]) + beta * p[i];
            const double sn = w[i] + beta * sv[i];
            x[i] = x[i] + alpha * pn;
            rn = r[i] - alpha * sn;
            p[i] = pn;
            sv[i] = sn;
            r[i] = rn;
            const double dr = d[i] * rn;
            e2 += dr * dr;
            if (BS == 0) g2 += rn * rn;
        }
        if constexpr (BS > 0) {
            sR[t] = rn;
            __syncthreads();
            if (in) {
                const double* iv = inv + i * BS;
                const int b0 = (t / BS) * BS;
                double un = 0.0;
#pragma unroll
                for (int c = 0; c < BS; ++c) un += iv[c] * sR[b0 + c];
                u[i] = un;
                g2 += rn * un;
            }
            __syncthreads();
        }
    }
    red[threadIdx.x] = e2;
    red[MB_BLOCK + threadIdx.x] = g2;
    __syncthreads();
    if (threadIdx.x < 2) {
        double s = 0.0;
        for (int k = 0; k < MB_BLOCK; ++k) s += red[threadIdx.x * MB_BLOCK + k];
        part[blockIdx.x * 2 + threadIdx.x] = s;
    }
}

// u = M^-1 r and partials (||D r||^2, r^T u): the start of the preconditioned CG
template <int BS>
__global__ __launch_bounds__(MB_BLOCK) void k_cg_prec(int64_t n, const double* __restrict__ r,
                                                      const double* __restrict__ d,
                                                      double* __restrict__ part,
                                                      const double* __restrict__ inv,
                                                      double* __restrict__ u) {
    __shared__ double red[2 * MB_BLOCK];
    __shared__ double sR[MB_BLOCK];
    const int t = threadIdx.x;
    double e2 = 0.0, g2 = 0.0;
    for (int64_t base = blockIdx.x * (int64_t)MB_BLOCK; base < n;
         base += (int64_t)gridDim.x * MB_BLOCK) {
        const int64_t i = base + t;
        const bool in = i < n;
        const double ri = in ? r[i] : 0.0;
        sR[t] = ri;
        __syncthreads();
        if (in) {
            const double* iv = inv + i * BS;
            const int b0 = (t / BS) * BS;
            double un = 0.0;
#pragma unroll
            for (int c = 0; c < BS; ++c) un += iv[c] * sR[b0 + c];
            u[i] = un;
            const double dr = d[i] * ri;
            e2 += dr * dr;
            g2 += ri * un;
        }
        __syncthreads();
    }
    red[t] = e2;
    red[MB_BLOCK + t] = g2;
    __syncthreads();
    if (t < 2) {
        double s = 0.0;
        for (int k = 0; k < MB_BLOCK; ++k) s += red[t * MB_BLOCK + k];
        part[blockIdx.x * 2 + t] = s;
    }
}

__global__ void k_export_x(int64_t n, int S, int s, const double* __restrict__ Xt,
                           const double* __restrict__ X0, double* __restrict__ out) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n * s;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = e / s;
        const int j = (int)(e % s);
        out[e] = Xt[r * S + j] + X0[r * S + j];
    }
}

__global__ void k_unscale(int64_t n, const double* __restrict__ xs, const double* __restrict__ d,
                          double* __restrict__ x) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        x[i] = xs[i] / d[i];
}

__global__ void k_stream_copy(const double4* __restrict__ src, double4* __restrict__ dst,
                              int64_t count) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

__global__ void k_copy_bytes(const unsigned char* __restrict__ src, unsigned char* __restrict__ dst,
                             int64_t count) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// n x S block rounded to FP32 or BF16 in the low-precision P layout, rows n ..
// lo_rows_padded(n) zero (initial block of a low-precision product)
template <int LO>
__global__ void k_block_to_lo(int64_t n, int S, const double* __restrict__ src,
                              void* __restrict__ dst) {
    const int64_t count = lo_rows_padded(n) * S;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = i / S;
        const int j = (int)(i % S);
        const double v = k < n ? src[i] : 0.0;
        const int64_t o = lo_pindex(LO, k, j, S);
        if (LO == DENSE_F32) static_cast<float*>(dst)[o] = (float)v;
        else static_cast<__hip_bfloat16*>(dst)[o] = __double2bfloat16(v);
    }
}

// x += alpha d (iterative refinement update, FP64; alpha = -1 takes it back)
__global__ void k_axpy_ir(int64_t n, double* __restrict__ x, const double* __restrict__ d,
                          double alpha) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        x[i] = x[i] + alpha * d[i];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline int grid_for(int64_t work, int cap) {
    int64_t g = (work + MB_BLOCK - 1) / MB_BLOCK;
    if (g < 1) g = 1;
    return (int)(g < cap ? g : cap);
}

#define MB_DISPATCH_S(S, CALL)          \
    switch (S) {                        \
        case 1: { constexpr int SS = 1; CALL; } \
        case 2: { constexpr int SS = 2; CALL; } \
        case 4: { constexpr int SS = 4; CALL; } \
        case 8: { constexpr int SS = 8; CALL; } \
        case 16: { constexpr int SS = 16; CALL; } \
        case 32: { constexpr int SS = 32; CALL; } \
    }                                   \
    return hipErrorInvalidValue;

// block size of the preconditioner (0: none) as a compile-time BB
#define MB_DISPATCH_BS(BS, CALL)                \
    switch (BS) {                               \
        case 0: { constexpr int BB = 0; CALL; }  \
        case 4: { constexpr int BB = 4; CALL; }  \
        case 8: { constexpr int BB = 8; CALL; }  \
        case 16: { constexpr int BB = 16; CALL; } \
        case 32: { constexpr int BB = 32; CALL; } \
    }                                           \
    return hipErrorInvalidValue;

template <int S>
static hipError_t update_s(int nwg, int64_t n, const double* P, const double* Q, double* Xt,
                           double* R, double* W, const double* d, double* part,
                           const DevState* st, hipStream_t stream, const BjArgs& bj) {
    MB_DISPATCH_BS(bj.bs, {
        hipLaunchKernelGGL((k_update<S, BB>), dim3(nwg), dim3(MB_BLOCK), 0, stream, n, P, Q, Xt, R,
                           W, d, part, st, bj.inv, bj.Y);
        return hipGetLastError();
    })
}

hipError_t launch_update(int S, int nwg, int64_t n, const double* P, const double* Q, double* Xt,
                         double* R, double* W, const double* d, double* part, const DevState* st,
                         hipStream_t stream, const BjArgs& bj) {
    MB_DISPATCH_S(S, return update_s<SS>(nwg, n, P, Q, Xt, R, W, d, part, st, stream, bj))
}

template <int S, int FIRST>
static hipError_t dirupdate_sf(int nwg, int64_t n, double* W, double* P, void* Plo, DenseKind lo,
                               const DevState* st, hipStream_t stream, const double* Yp,
                               double* Xt) {
    if (Yp) {
        if (lo != DENSE_F64) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_dirupdate<S, FIRST, DENSE_F64, 1>), dim3(nwg), dim3(MB_BLOCK), 0,
                           stream, n, W, P, Plo, st, Yp, Xt);
    } else if (lo == DENSE_F32) {
        hipLaunchKernelGGL((k_dirupdate<S, FIRST, DENSE_F32, 0>), dim3(nwg), dim3(MB_BLOCK), 0,
                           stream, n, W, P, Plo, st, Yp, Xt);
    } else if (lo == DENSE_BF16) {
        hipLaunchKernelGGL((k_dirupdate<S, FIRST, DENSE_BF16, 0>), dim3(nwg), dim3(MB_BLOCK), 0,
                           stream, n, W, P, Plo, st, Yp, Xt);
    } else {
        hipLaunchKernelGGL((k_dirupdate<S, FIRST, DENSE_F64, 0>), dim3(nwg), dim3(MB_BLOCK), 0,
                           stream, n, W, P, Plo, st, Yp, Xt);
    }
    return hipGetLastError();
}

template <int S>
static hipError_t dirupdate_s(int nwg, int64_t n, double* W, double* P, void* Plo, DenseKind lo,
                              int first, const DevState* st, hipStream_t stream, const double* Yp,
                              double* Xt) {
    return first ? dirupdate_sf<S, 1>(nwg, n, W, P, Plo, lo, st, stream, Yp, Xt)
                 : dirupdate_sf<S, 0>(nwg, n, W, P, Plo, lo, st, stream, Yp, Xt);
}

hipError_t launch_dirupdate(int S, int nwg, int64_t n, double* W, double* P, void* Plo,
                            DenseKind lo_kind, int first, const DevState* st, hipStream_t stream,
                            const double* Yp, double* Xt) {
    MB_DISPATCH_S(S, return dirupdate_s<SS>(nwg, n, W, P, Plo, lo_kind, first, st, stream, Yp, Xt))
}

// workgroups of the FP64 update / direction kernels (no preconditioner) that
// fit on one CU; 0 on error or an unknown width
static int occ_of(const void* fn) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, MB_BLOCK, 0) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return per_cu;
}

int update_blocks_per_cu(int S) {
    switch (S) {
        case 1: return occ_of((const void*)k_update<1, 0>);
        case 2: return occ_of((const void*)k_update<2, 0>);
        case 4: return occ_of((const void*)k_update<4, 0>);
        case 8: return occ_of((const void*)k_update<8, 0>);
        case 16: return occ_of((const void*)k_update<16, 0>);
        case 32: return occ_of((const void*)k_update<32, 0>);
    }
    return 0;
}

int dirupdate_blocks_per_cu(int S) {
    switch (S) {
        case 1: return occ_of((const void*)k_dirupdate<1, 0, DENSE_F64, 0>);
        case 2: return occ_of((const void*)k_dirupdate<2, 0, DENSE_F64, 0>);
        case 4: return occ_of((const void*)k_dirupdate<4, 0, DENSE_F64, 0>);
        case 8: return occ_of((const void*)k_dirupdate<8, 0, DENSE_F64, 0>);
        case 16: return occ_of((const void*)k_dirupdate<16, 0, DENSE_F64, 0>);
        case 32: return occ_of((const void*)k_dirupdate<32, 0, DENSE_F64, 0>);
    }
    return 0;
}

hipError_t launch_rhs(int nwg, int64_t n, const double* b, const double* d, double* bbar,
                      double* part, hipStream_t s) {
    hipLaunchKernelGGL(k_rhs, dim3(nwg), dim3(MB_BLOCK), 0, s, n, b, d, bbar, part);
    return hipGetLastError();
}

hipError_t launch_uniform(int S, int64_t n, int s, uint64_t seed, double* U, hipStream_t st) {
    const int g = grid_for(n * S, 8192);
    MB_DISPATCH_S(S, {
        hipLaunchKernelGGL(k_uniform<SS>, dim3(g), dim3(MB_BLOCK), 0, st, n, s, seed, U);
        return hipGetLastError();
    })
}

hipError_t launch_pad_block(int S, int64_t n, int s, const double* Uin, double* U, hipStream_t st) {
    const int g = grid_for(n * S, 8192);
    MB_DISPATCH_S(S, {
        hipLaunchKernelGGL(k_pad_block<SS>, dim3(g), dim3(MB_BLOCK), 0, st, n, s, Uin, U);
        return hipGetLastError();
    })
}

hipError_t launch_ynorm(int S, int nwg, int64_t n, const double* Y, double* part, hipStream_t s) {
    MB_DISPATCH_S(S, {
        hipLaunchKernelGGL(k_ynorm<SS>, dim3(nwg), dim3(MB_BLOCK), 0, s, n, Y, part);
        return hipGetLastError();
    })
}

hipError_t launch_init(int S, int64_t n, int s, const double* U, const double* Y,
                       const double* bbar, double* X0, double* Xt, double* R, const DevState* st,
                       hipStream_t stream) {
    const int g = grid_for(n * S, 8192);
    MB_DISPATCH_S(S, {
        hipLaunchKernelGGL(k_init<SS>, dim3(g), dim3(MB_BLOCK), 0, stream, n, s, U, Y, bbar, X0, Xt,
                           R, st);
        return hipGetLastError();
    })
}

template <int S>
static hipError_t gram_nu_s(int nwg, int64_t n, const double* X, const double* d, double* part,
                            hipStream_t stream, const BjArgs& bj) {
    MB_DISPATCH_BS(bj.bs, {
        hipLaunchKernelGGL((k_gram_nu<S, BB>), dim3(nwg), dim3(MB_BLOCK), 0, stream, n, X, d, part,
                           bj.inv, bj.Y);
        return hipGetLastError();
    })
}

hipError_t launch_gram_nu(int S, int nwg, int64_t n, const double* X, const double* d, double* part,
                          hipStream_t stream, const BjArgs& bj) {
    MB_DISPATCH_S(S, return gram_nu_s<SS>(nwg, n, X, d, part, stream, bj))
}

hipError_t launch_ls_gram(int S, int nwg, int64_t n, const double* b, const double* R,
                          const double* d, double* part, const DevState* st, hipStream_t s) {
    MB_DISPATCH_S(S, {
        hipLaunchKernelGGL(k_ls_gram<SS>, dim3(nwg), dim3(MB_BLOCK), 0, s, n, b, R, d, part, st);
        return hipGetLastError();
    })
}

hipError_t launch_ls_apply(int S, int nwg, int64_t n, const double* Xt, const double* X0,
                           const double* R, const double* b, const double* d, double* x,
                           double* part, const DevState* st, hipStream_t s) {
    MB_DISPATCH_S(S, {
        hipLaunchKernelGGL(k_ls_apply<SS>, dim3(nwg), dim3(MB_BLOCK), 0, s, n, Xt, X0, R, b, d, x,
                           part, st);
        return hipGetLastError();
    })
}

hipError_t launch_select(int S, int64_t n, const double* Xt, const double* X0, const double* d,
                         double* x, const DevState* st, int force, hipStream_t s) {
    const int g = grid_for(n, 4096);
    MB_DISPATCH_S(S, {
        hipLaunchKernelGGL(k_select<SS>, dim3(g), dim3(MB_BLOCK), 0, s, n, Xt, X0, d, x, st,
                           force);
        return hipGetLastError();
    })
}

hipError_t launch_cg_init(int64_t n, const double* bbar, double* x, double* r, double* p,
                          double* sv, hipStream_t s) {
    hipLaunchKernelGGL(k_cg_init, dim3(grid_for(n, 4096)), dim3(MB_BLOCK), 0, s, n, bbar, x, r, p,
                       sv);
    return hipGetLastError();
}

hipError_t launch_cg_update(int nwg, int64_t n, double* p, double* sv, double* x, double* r,
                            const double* w, const double* d, double* part, const DevState* st,
                            hipStream_t s, const BjArgs& bj) {
    MB_DISPATCH_BS(bj.bs, {
        hipLaunchKernelGGL(k_cg_update<BB>, dim3(nwg), dim3(MB_BLOCK), 0, s, n, p, sv, x, r, w, d,
                           part, st, bj.inv, bj.Y);
        return hipGetLastError();
    })
}

hipError_t launch_cg_prec(int nwg, int64_t n, const double* r, const double* d, double* part,
                          const BjArgs& bj, hipStream_t s) {
    if (bj.bs == 0) return hipErrorInvalidValue;
    MB_DISPATCH_BS(bj.bs, {
        hipLaunchKernelGGL(k_cg_prec<(BB > 0 ? BB : 4)>, dim3(nwg), dim3(MB_BLOCK), 0, s, n, r, d,
                           part, bj.inv, bj.Y);
        return hipGetLastError();
    })
}

hipError_t launch_export_x(int S, int64_t n, int s, const double* Xt, const double* X0, double* out,
                           hipStream_t st) {
    hipLaunchKernelGGL(k_export_x, dim3(grid_for(n * s, 4096)), dim3(MB_BLOCK), 0, st, n, S, s, Xt,
                       X0, out);
    return hipGetLastError();
}

hipError_t launch_unscale(int64_t n, const double* xs, const double* d, double* x, hipStream_t s) {
    hipLaunchKernelGGL(k_unscale, dim3(grid_for(n, 4096)), dim3(MB_BLOCK), 0, s, n, xs, d, x);
    return hipGetLastError();
}

hipError_t launch_block_to_lo(DenseKind kind, int64_t n, int S, const double* src, void* dst,
                             hipStream_t s) {
    const int64_t count = lo_rows_padded(n) * S;
    if (kind == DENSE_F32)
        hipLaunchKernelGGL(k_block_to_lo<DENSE_F32>, dim3(grid_for(count, 8192)), dim3(MB_BLOCK), 0,
                           s, n, S, src, dst);
    else if (kind == DENSE_BF16)
        hipLaunchKernelGGL(k_block_to_lo<DENSE_BF16>, dim3(grid_for(count, 8192)), dim3(MB_BLOCK),
                           0, s, n, S, src, dst);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_axpy_ir(int64_t n, double* x, const double* d, double alpha, hipStream_t s) {
    hipLaunchKernelGGL(k_axpy_ir, dim3(grid_for(n, 4096)), dim3(MB_BLOCK), 0, s, n, x, d, alpha);
    return hipGetLastError();
}

hipError_t launch_stream_copy(void* dst, const void* src, int64_t bytes, hipStream_t s) {
    if ((bytes % 32) == 0 && ((uintptr_t)dst % 32) == 0 && ((uintptr_t)src % 32) == 0) {
        const int64_t cnt = bytes / 32;
        hipLaunchKernelGGL(k_stream_copy, dim3(grid_for(cnt, 8192)), dim3(MB_BLOCK), 0, s,
                           (const double4*)src, (double4*)dst, cnt);
    } else {
        hipLaunchKernelGGL(k_copy_bytes, dim3(grid_for(bytes, 8192)), dim3(MB_BLOCK), 0, s,
                           (const unsigned char*)src, (unsigned char*)dst, bytes);
    }
    return hipGetLastError();
}

}  // namespace mb

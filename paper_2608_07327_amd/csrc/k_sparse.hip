// Block product of the sparse path: Q = A~ P for CSR A~ and row-major P with
// S columns, fused with the per-workgroup lower triangle of P^T Q (the Gram
// whose inverse is Alg. 1's step matrix Xi).
//
// A tile of T rows has its row pointers and then its CSR slice (column
// indices and values, one contiguous range) staged in LDS with coalesced
// loads, so A is read from HBM once per product for all S columns.  A row is
// handled by LPR = (S / V) * SL lanes: lane (slot, jv) accumulates the V
// adjacent columns jv .. jv+V-1 of P (16-byte loads for V = 2, 4) over every
// SL-th nonzero of the row, with U gathers in flight; for S > 2 the tile's own
// rows of P are staged in LDS (the Gram's operand) and a nonzero whose
// column falls inside the tile reads its P row from there.  Q leaves with
// non-temporal vector stores: for S <= 2 from the lanes' registers, for
// S > 2 from the tile's Q rows in LDS (the Gram's other operand), one
// contiguous range, so that every store instruction fills whole lines.
//
// Gram epilogue, chosen by width so that it costs few registers (the kernel
// lives on occupancy: its gathers' latency is hidden by other wavefronts):
//  - S <= 2: each lane keeps the S x V block of P^T Q that its rows feed,
//    from its own P row; reduced over lanes and waves once per workgroup.
//  - S = 4: the tile's P rows (staged in LDS next to the row pointers) and Q
//    rows (from the lanes) feed a per-thread fixed-order sum of one entry.
//  - S >= 8: the same LDS tiles feed the 16 x 16 x 4 FP64 MFMA.
// The tuned shape is (T, SL, V, U, W) plus the grid size.
#include "kernels.hpp"

#include <algorithm>
#include <tuple>


namespace mb {

template <int S_, int T_, int SL_, int V_, int U_, int W_ = 0>
struct BpShape {
    static constexpr int S = S_, T = T_, SL = SL_, V = V_, U = U_;
    static constexpr int W = W_;                       // requested waves per SIMD (0: free)
    static constexpr int CPR = S / V;                  // lanes per row and slot
    static constexpr int LPR = CPR * SL;               // lanes per row
    static constexpr int RPP = MB_BLOCK / LPR;         // rows per pass of the block
    static constexpr int NR = (T + RPP - 1) / RPP;     // passes per tile
    static constexpr int NZC = 8 * T;                  // nonzeros per LDS chunk
    static constexpr bool REG = S <= 2;                // Gram in lane registers
    static constexpr bool MF = S >= 8;                 // Gram on the matrix cores
    static_assert(S % V == 0 && LPR <= 64 && (V == 1 || V == 2 || V == 4), "shape");
};

template <int V>
__device__ __forceinline__ void load_cols(const double* p, double* x) {
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

// Q rows leave with non-temporal stores: nothing in the product reads them
// again, and holding them in the L2 would evict rows of P that later tiles
// gather
template <int V>
__device__ __forceinline__ void store_cols(double* p, const double* x) {
    if constexpr (V == 1) {
        __builtin_nontemporal_store(x[0], p);
    } else {
        typedef double d2 __attribute__((ext_vector_type(2)));
#pragma unroll
        for (int h = 0; h < V / 2; ++h) {
            d2 t;
            t.x = x[2 * h];
            t.y = x[2 * h + 1];
            __builtin_nontemporal_store(t, reinterpret_cast<d2*>(p) + h);
        }
    }
}

template <class B>
__global__ __launch_bounds__(MB_BLOCK) __attribute__((amdgpu_waves_per_eu(B::W > 0 ? B::W : 1)))
void k_spmm(const int32_t* __restrict__ rowptr,
                                                   const int32_t* __restrict__ colind,
                                                   const double* __restrict__ vals, int64_t n,
                                                   const double* __restrict__ P,
                                                   double* __restrict__ Q,
                                                   double* __restrict__ part,
                                                   const DevState* __restrict__ st) {
    constexpr int S = B::S, T = B::T, SL = B::SL, V = B::V, U = B::U;
    constexpr int RPP = B::RPP, NR = B::NR, NZC = B::NZC;
    constexpr bool REG = B::REG, MF = B::MF;
    constexpr int RPT = (T + 1 + MB_BLOCK - 1) / MB_BLOCK;   // row pointers per thread
    constexpr int PPT = (T * S + MB_BLOCK - 1) / MB_BLOCK;   // staged P entries per thread
    constexpr int CPT = (NZC + MB_BLOCK - 1) / MB_BLOCK;     // CSR entries per thread and chunk
    constexpr int E = tri_count(S);
    if (st && st->done) return;
    __shared__ int32_t sRp[T + 1];
    __shared__ int32_t sC[NZC];
    __shared__ double sV[NZC];
    __shared__ double sQ[REG ? 1 : T * S];
    __shared__ double sP[REG ? 1 : T * S];
    __shared__ double red[REG ? (MB_BLOCK / 64) * S * S : (S * S > MB_BLOCK ? S * S : MB_BLOCK)];
    const int tid = threadIdx.x;
    const int grp = tid / B::LPR, lane = tid % B::LPR;
    const int slot = lane / B::CPR, jv = (lane % B::CPR) * V;
    const bool gram = part != nullptr;

    double g[REG ? S : 1][V];          // register Gram: G[i][jv + q]
#pragma unroll
    for (int i = 0; i < (REG ? S : 1); ++i)
#pragma unroll
        for (int q = 0; q < V; ++q) g[i][q] = 0.0;
    TileSums<E> gs;
    int gi[TileSums<E>::EPT], gj[TileSums<E>::EPT];
    GramMfma<S> gm;
    if constexpr (MF) {
        gm.init();
    } else if constexpr (!REG) {
        gs.init();
#pragma unroll
        for (int k = 0; k < TileSums<E>::EPT; ++k) {
            gi[k] = gj[k] = 0;
            if (gs.ent[k] >= 0) tri_ij(gs.ent[k], gi[k], gj[k]);
        }
    }

    // Software pipeline over this workgroup's tiles: while a tile's gathers
    // are in flight, the next tile's row pointers, P tile and CSR-slice
    // bounds are loaded, and its first CSR chunk is loaded while the tile's
    // Q rows are stored and its Gram is formed; every copy issues all of a
    // thread's loads before its first LDS store (fixed per-thread counts,
    // addresses clamped inside the arrays).
    const int64_t ntiles = (n + T - 1) / T;
    const TileRange tr = tile_range(ntiles);
    int rpv[RPT];                      // row pointers of the tile in flight
    double ppv[REG ? 1 : PPT];         // its P tile (Gram operand)
    int cc[CPT];                       // its first CSR chunk
    double cv[CPT];
    int h_nzb = 0, h_nze = 0;          // its CSR range
    auto fetch_head = [&](int64_t tl) {
        const int64_t q0 = tl * T;
        const int qrows = (int)min((int64_t)T, n - q0);
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int e = tid + q * MB_BLOCK;
            rpv[q] = rowptr[q0 + (e <= qrows ? e : 0)];
        }
        if constexpr (!REG) {
#pragma unroll
            for (int q = 0; q < PPT; ++q) {
                const int e = tid + q * MB_BLOCK;
                const bool in = e < qrows * S;
                const double v = P[q0 * S + (in ? e : 0)];
                ppv[q] = in ? v : 0.0;
            }
        }
        h_nzb = rowptr[q0];
        h_nze = rowptr[q0 + qrows];
    };
    // CSR entries [g0, g0 + cnt) into cc/cv; S >= 2: the CSR slice is not
    // read again before a whole block-CG iteration has evicted it, and
    // non-temporal loads keep P in the last-level cache instead (S = 1, CG,
    // moves so little per iteration that A itself may stay cached)
    auto fetch_csr = [&](int64_t g0, int cnt) {
        if (cnt <= 0) return;
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            const int e = tid + q * MB_BLOCK;
            const int64_t g = g0 + (e < cnt ? e : 0);
            if constexpr (S >= 2) {
                cc[q] = stream_load(colind + g);
                cv[q] = stream_load(vals + g);
            } else {
                cc[q] = colind[g];
                cv[q] = vals[g];
            }
        }
    };
    auto put_csr = [&](int cnt) {
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            const int e = tid + q * MB_BLOCK;
            if (e < cnt) {
                sC[e] = cc[q];
                sV[e] = cv[q];
            }
        }
    };
    if (tr.first < tr.end) {
        fetch_head(tr.first);
        fetch_csr(h_nzb, min(NZC, h_nze - h_nzb));
    }
    for (int64_t tile = tr.first; tile < tr.end; tile += tr.step) {
        const int64_t r0 = tile * T;
        const int rows = (int)min((int64_t)T, n - r0);
        const double* Pt = P + r0 * S;
        const int nz0 = h_nzb;
        const int nzt = h_nze - h_nzb;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int e = tid + q * MB_BLOCK;
            if (e <= rows) sRp[e] = rpv[q];
        }
        if constexpr (!REG) {
#pragma unroll
            for (int q = 0; q < PPT; ++q) {
                const int e = tid + q * MB_BLOCK;
                if (e < T * S) sP[e] = ppv[q];
            }
        }
        put_csr(min(NZC, nzt));
        double pr[REG ? NR : 1][S];    // register Gram: this lane's P rows
        __syncthreads();
        const int64_t nxt = tile + tr.step;
        if (nxt < tr.end) fetch_head(nxt);
        if (gram) {
            if constexpr (REG) {
#pragma unroll
                for (int i = 0; i < NR; ++i) {
                    const int rl = i * RPP + grp;
                    if (rl < rows && slot == 0) {
                        load_cols<S>(Pt + (int64_t)rl * S, pr[i]);
                    } else {
#pragma unroll
                        for (int c = 0; c < S; ++c) pr[i][c] = 0.0;
                    }
                }
            }
        }
        double acc[NR][V];
#pragma unroll
        for (int i = 0; i < NR; ++i)
#pragma unroll
            for (int q = 0; q < V; ++q) acc[i][q] = 0.0;
        for (int cb = 0; cb < nzt; cb += NZC) {
            const int cn = min(NZC, nzt - cb);
            if (cb > 0) {
                // rows longer than the chunk: later chunks are loaded here
                fetch_csr((int64_t)nz0 + cb, cn);
                put_csr(cn);
                __syncthreads();
            }
#pragma unroll
            for (int i = 0; i < NR; ++i) {
                const int rl = i * RPP + grp;
                if (rl >= rows) continue;
                const int kb = sRp[rl] - nz0, ke = sRp[rl + 1] - nz0;
                // this slot's nonzeros kb + slot + m*SL inside [cb, cb + cn)
                int k = kb + slot;
                if (k < cb) k += ((cb - k + SL - 1) / SL) * SL;
                const int kend = min(ke, cb + cn);
                for (; k < kend; k += U * SL) {
                    double v[U], x[U][V];
                    unsigned lc[U];
                    // gathers of the columns outside this tile's rows, all
                    // issued before the first is consumed; a column inside
                    // the tile reads its P row from LDS when it is consumed
                    // (after the gathers have landed: an LDS read into the
                    // registers of a gather in flight would make the
                    // compiler wait for every gather issued before it)
                    int c[U];
                    // every slot's column and value first (a slot past the
                    // row reads the row's last entry, in bounds, unused), so
                    // that one LDS round trip serves all of them
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int kk = k + u * SL;
                        const int kc = (kk < kend ? kk : kend - 1) - cb;
                        c[u] = sC[kc];
                        v[u] = sV[kc];
                    }
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        lc[u] = REG ? ~0u : (unsigned)(c[u] - (int)r0);
                        if (k + u * SL < kend && (REG || lc[u] >= (unsigned)rows))
                            load_cols<V>(P + (int64_t)c[u] * S + jv, x[u]);
                    }
#pragma unroll
                    for (int u = 0; u < U; ++u)
                        if (k + u * SL < kend) {
                            if (!REG && lc[u] < (unsigned)rows) {
#pragma unroll
                                for (int q = 0; q < V; ++q) x[u][q] = sP[lc[u] * S + jv + q];
                            }
#pragma unroll
                            for (int q = 0; q < V; ++q) acc[i][q] += v[u] * x[u][q];
                        }
                }
            }
            __syncthreads();
        }
        // the next tile's first CSR chunk (its bounds came with its head)
        if (nxt < tr.end) fetch_csr(h_nzb, min(NZC, h_nze - h_nzb));

#pragma unroll
        for (int i = 0; i < NR; ++i) {
            const int rl = i * RPP + grp;
#pragma unroll
            for (int q = 0; q < V; ++q) {
                double a = acc[i][q];
#pragma unroll
                for (int off = B::CPR; off < B::LPR; off <<= 1) a += __shfl_xor(a, off, 64);
                acc[i][q] = a;
            }
            if (slot == 0 && rl < T) {
                if constexpr (REG) {
                    if (rl < rows) store_cols<V>(Q + (r0 + rl) * S + jv, acc[i]);
#pragma unroll
                    for (int c = 0; c < S; ++c)
#pragma unroll
                        for (int q = 0; q < V; ++q) g[c][q] += pr[i][c] * acc[i][q];
                } else {
#pragma unroll
                    for (int q = 0; q < V; ++q) sQ[rl * S + jv + q] = rl < rows ? acc[i][q] : 0.0;
                }
            }
        }
        if constexpr (!REG) {
            // the tile's Q rows are one contiguous range of rows * S values:
            // they leave LDS with 16-byte stores that fill whole lines
            __syncthreads();
            for (int e = 2 * tid; e < rows * S; e += 2 * MB_BLOCK) store_cols<2>(Q + r0 * S + e, &sQ[e]);
            if (gram) {
                if constexpr (MF)
                    gm.add_tile(rows, [&](int r, int c) { return sP[r * S + c]; },
                                [&](int r, int c) { return sQ[r * S + c]; });
                else
                    gs.add_rows(rows, [&](int k, int r) { return sP[r * S + gi[k]] * sQ[r * S + gj[k]]; });
            }
        }
        __syncthreads();
    }
    if (!gram) return;

    if constexpr (REG) {
        // sum over the row groups of the wave (lanes with equal slot and jv)
#pragma unroll
        for (int c = 0; c < S; ++c)
#pragma unroll
            for (int q = 0; q < V; ++q) {
                double x = g[c][q];
#pragma unroll
                for (int off = B::LPR; off < 64; off <<= 1) x += __shfl_xor(x, off, 64);
                g[c][q] = x;
            }
        const int wave = tid >> 6;
        if ((tid & 63) < B::LPR && slot == 0) {
#pragma unroll
            for (int c = 0; c < S; ++c)
#pragma unroll
                for (int q = 0; q < V; ++q) red[wave * S * S + c * S + jv + q] = g[c][q];
        }
        __syncthreads();
        for (int e = tid; e < E; e += MB_BLOCK) {
            int i, j;
            tri_ij(e, i, j);
            double s = red[i * S + j];
#pragma unroll
            for (int w = 1; w < MB_BLOCK / 64; ++w) s += red[w * S * S + i * S + j];
            part[(int64_t)blockIdx.x * E + e] = s;
        }
    } else if constexpr (MF) {
        gm.finish(red, part + (int64_t)blockIdx.x * E);
    } else {
        gs.finish(red, part + (int64_t)blockIdx.x * E);
    }
}

// ---- compiled shapes (S, T, SL, V, U[, W]); W asks the compiler to fit W
// wavefronts per SIMD (fewer registers, more gathers in flight per CU)
using BpShapes = std::tuple<
    BpShape<1, 64, 1, 1, 8>, BpShape<1, 128, 1, 1, 8>, BpShape<1, 256, 1, 1, 8>,
    BpShape<1, 64, 2, 1, 4>, BpShape<1, 128, 2, 1, 4>, BpShape<1, 256, 2, 1, 4>,
    BpShape<2, 64, 1, 2, 8>, BpShape<2, 128, 1, 2, 8>, BpShape<2, 256, 1, 2, 8>,
    BpShape<2, 128, 1, 2, 4>, BpShape<2, 256, 1, 2, 4>, BpShape<2, 128, 2, 2, 4>,
    BpShape<2, 128, 1, 2, 8, 8>,
    BpShape<4, 64, 1, 2, 4>, BpShape<4, 128, 1, 2, 4>, BpShape<4, 64, 1, 2, 8>,
    BpShape<4, 128, 1, 2, 8>, BpShape<4, 128, 1, 4, 4>, BpShape<4, 256, 1, 4, 4>,
    BpShape<4, 128, 2, 2, 4>,
    BpShape<4, 64, 1, 2, 8, 8>, BpShape<4, 128, 1, 2, 8, 6>, BpShape<4, 64, 1, 4, 4, 8>,
    BpShape<4, 128, 1, 4, 4, 6>,
    BpShape<8, 32, 1, 2, 8>, BpShape<8, 64, 1, 2, 8>, BpShape<8, 64, 1, 2, 4>,
    BpShape<8, 128, 1, 2, 4>, BpShape<8, 64, 1, 4, 4>, BpShape<8, 128, 1, 4, 4>,
    BpShape<8, 32, 1, 2, 8, 8>, BpShape<8, 64, 1, 2, 8, 6>, BpShape<8, 64, 1, 4, 4, 6>,
    BpShape<16, 32, 1, 2, 8>, BpShape<16, 32, 1, 2, 4>, BpShape<16, 64, 1, 2, 8>,
    BpShape<16, 32, 1, 4, 4>, BpShape<16, 64, 1, 4, 4>,
    BpShape<16, 32, 1, 2, 8, 6>, BpShape<16, 32, 1, 4, 4, 6>, BpShape<16, 32, 1, 2, 4, 8>,
    BpShape<32, 32, 1, 2, 8>, BpShape<32, 32, 1, 2, 4>, BpShape<32, 32, 1, 4, 4>,
    BpShape<32, 32, 1, 2, 8, 5>, BpShape<32, 32, 1, 4, 4, 5>>;

template <class F, class... Bs>
static bool any_shape(F&& f, std::tuple<Bs...>*) {
    return (f(Bs{}) || ...);
}

template <class B>
static bool shape_is(const B&, int S, const SpmmShape& sh) {
    return B::S == S && B::T == sh.T && B::SL == sh.SL && B::V == sh.V && B::U == sh.U &&
           B::W == sh.W;
}

bool spmm_valid_shape(int S, const SpmmShape& sh) {
    return any_shape([&](auto b) { return shape_is(b, S, sh); }, (BpShapes*)nullptr);
}

int spmm_shape_list(int S, SpmmShape* out, int cap) {
    int k = 0;
    any_shape(
        [&](auto b) {
            using B = decltype(b);
            if (B::S == S && k < cap) out[k++] = SpmmShape{B::T, B::SL, B::V, B::U, B::W};
            return false;
        },
        (BpShapes*)nullptr);
    return k;
}

SpmmShape spmm_default_shape(int S) {
    switch (S) {
        case 1: return SpmmShape{128, 1, 1, 8};
        case 2: return SpmmShape{128, 1, 2, 4};
        case 4: return SpmmShape{128, 1, 2, 4};
        case 8: return SpmmShape{64, 1, 2, 4};
        case 16: return SpmmShape{32, 1, 2, 8};
        default: return SpmmShape{32, 1, 2, 8};
    }
}

int spmm_lanes_per_row(int S, const SpmmShape& sh) { return S / sh.V * sh.SL; }

int spmm_blocks_per_cu(int S, const SpmmShape& sh) {
    int per_cu = 0;
    any_shape(
        [&](auto b) {
            using B = decltype(b);
            if (!shape_is(b, S, sh)) return false;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_spmm<B>, MB_BLOCK, 0) !=
                hipSuccess) {
                (void)hipGetLastError();
                per_cu = 0;
            }
            return true;
        },
        (BpShapes*)nullptr);
    return per_cu;
}

hipError_t launch_spmm(int S, const SpmmShape& sh, int nwg, const CsrDev& A, const double* P,
                       double* Q, double* part, const DevState* st, hipStream_t stream) {
    hipError_t err = hipErrorInvalidValue;
    any_shape(
        [&](auto b) {
            using B = decltype(b);
            if (!shape_is(b, S, sh)) return false;
            hipLaunchKernelGGL((k_spmm<B>), dim3(nwg), dim3(MB_BLOCK), 0, stream, A.rowptr,
                               A.colind, A.vals, A.n, P, Q, part, st);
            err = hipGetLastError();
            return true;
        },
        (BpShapes*)nullptr);
    return err;
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

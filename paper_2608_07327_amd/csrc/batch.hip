// Batched MBPCG: many independent sparse SPD systems of uneven n and block
// width s (1..8) solved together by ONE persistent kernel, launched through a
// hipGraph.  The kernel walks the whole of Algorithm 1 -- scaling, initial
// block, the iteration loop and the least-squares termination -- for every
// system at once.  Each phase spreads its work over the grid: streaming row
// phases take (system, 1024 / S-row) items, the block products take
// (system, 128-row) items, s x s phases take one system per workgroup.
// Phases are separated by a software grid barrier; every barrier wait is
// bounded, so a grid that is not co-resident ends with an error instead of a
// hang.  Systems that finish drop out of the item loops; the loop ends when
// none is active.
#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "dev_spmm.hpp"
#include "dev_sxs.hpp"
#include "runtime.hpp"

namespace mb {

// rows per item: 1024 / S, so every item holds 1024 block entries (S = 8:
// 128 rows, S = 1: 1024 rows) and a phase moves the same bytes per item
// whatever the width
__host__ __device__ constexpr int item_rows(int S) { return 1024 / S; }
constexpr int ITEM_ELEMS = 1024;
// rows per block-product item: the product phases keep 128-row items (their
// gathers do best spread over many small items), with partial sums of their
// own
constexpr int PT = 128;
constexpr int PSTRIDE = 96;    // doubles of partial sums per item (the double-double
                               // Gram of the least squares at S = 8: 2 x 45)
constexpr int BATCH_TERM_BARRIERS = 9;  // grid barriers of the termination
constexpr int BSM = 4096;    // LDS doubles of the persistent kernel (32 KB)
static_assert(SxsWs<8>::DOUBLES <= BSM, "s x s workspace of the widest batched system");

struct BSys {
    int64_t n, rp_off, nz_off, vec_off, blk_off;
    int32_t s, S, SL, ntile, item_off, pntile, pitem_off, pad;
};

constexpr int BAR_GROUPS = 8;   // first-level arrival counters of the grid barrier

struct BCtl {
    unsigned bar_count, bar_gen;
    int abort, active;
    int loops, pad0, pad1, pad2;
    unsigned sub[BAR_GROUPS * 32];   // group g's arrival counter at sub[32 g] (own 128-byte line)
};

struct BArgs {
    int nsys, total_items, max_iter, jacobi;
    int total_pitems, pad_p;
    const int32_t* pitem_sys;   // system of each block-product item
    double* ppart;              // partial sums of the block-product items
    double tol, tau;
    uint64_t seed;
    long long spin_limit;
    const BSys* sys;
    DevState* st;
    BCtl* ctl;
    const int32_t* item_sys;
    const int32_t* rowptr;
    const int32_t* colind;
    const double* vals;
    double* vals_s;
    const double* b;
    double* x;
    double* d;
    double* bbar;
    double *U, *Y, *X0, *Xt, *R, *W, *P, *Q;
    double* part;
    long long* tstamp;   // profile: steady-clock stamp after every grid barrier (or null)
};

// The batch's arguments, written by the host before each launch.  Device
// code reads them from here (scalar loads at a fixed address) rather than
// through a reference to the kernel argument, which the compiler kept in
// per-lane scratch memory for the phase functions it does not inline.
// One batched solve at a time per process (the host serialises them).
__constant__ BArgs g_bargs;

// ---------------------------------------------------------------------------
// software grid barrier (sense by generation counter), bounded wait
// ---------------------------------------------------------------------------
__device__ bool grid_sync(BCtl* ctl, long long spin_limit, int* flag) {
    // One thread per workgroup publishes and acquires for the whole
    // workgroup (the workgroup barrier orders its other threads' accesses
    // around it): a device-scope release before it counts in and an acquire
    // after it sees the new generation.  A device-scope fence writes back or
    // invalidates the XCD's L2, so the counting and the polling use relaxed
    // atomics and the fences are issued once each, not per thread, per
    // atomic or per poll (an acquiring poll would invalidate the L2 under the
    // workgroups still at work); the last arriver of a group, and the last
    // group, acquire what the others released before they count on.
    __syncthreads();
    if (threadIdx.x == 0) {
        // two levels of arrival: workgroup b counts on its group's counter
        // (g = b mod groups), the group's last arriver on the top counter,
        // and the last group releases everyone by bumping the generation;
        // the atomics on one address are serialised, so the chain is about
        // nb / 8 + 8 long instead of nb
        const unsigned nb = gridDim.x;
        const unsigned groups = nb < (unsigned)BAR_GROUPS ? nb : (unsigned)BAR_GROUPS;
        const unsigned g = blockIdx.x % groups;
        const unsigned ng = (nb - g + groups - 1) / groups;   // workgroups of group g
        const unsigned gen = __hip_atomic_load(&ctl->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        bool last = false;
        const unsigned a1 =
            __hip_atomic_fetch_add(&ctl->sub[32 * g], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (a1 == ng - 1) {
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
            __hip_atomic_store(&ctl->sub[32 * g], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const unsigned a2 =
                __hip_atomic_fetch_add(&ctl->bar_count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (a2 == groups - 1) {
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
                __hip_atomic_store(&ctl->bar_count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_add(&ctl->bar_gen, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                last = true;
            }
        }
        if (!last) {
            long long spins = 0;
            while (__hip_atomic_load(&ctl->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                __builtin_amdgcn_s_sleep(8);
                if (++spins > spin_limit) {
                    __hip_atomic_store(&ctl->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
                if (__hip_atomic_load(&ctl->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        *flag = __hip_atomic_load(&ctl->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    const int ab = *flag;
    __syncthreads();
    return ab == 0;
}

// Polls a workgroup makes at a grid barrier before it gives up and ends the
// launch (all co-resident workgroups arrive long before).  The environment
// variable MBPCG_BATCH_SPIN_LIMIT (a positive integer) lowers the bound, so
// that a test reaches the error path with every workgroup exiting normally.
static long long batch_spin_limit() {
    if (const char* e = getenv("MBPCG_BATCH_SPIN_LIMIT")) {
        char* end = nullptr;
        const long long v = strtoll(e, &end, 10);
        if (end != e && *end == 0 && v > 0) return v;
    }
    return 1ll << 24;
}

// block-wide fixed-order sum of one value per thread, by a pairwise tree
// (result valid in thread 0)
__device__ double block_sum(double v, double* red) {
    const int t = threadIdx.x;
    red[t] = v;
    __syncthreads();
#pragma unroll
    for (int h = MB_BLOCK / 2; h >= 1; h /= 2) {
        if (t < h) red[t] += red[t + h];
        __syncthreads();
    }
    const double s = red[0];
    __syncthreads();
    return s;
}

struct Item {
    int sys;
    int it;      // global item index (its partial-sum slot)
    int64_t r0;
    int rows;
};

// block-product item (PT rows)
__device__ __forceinline__ Item pitem_of(int it) {
    const BArgs& a = g_bargs;
    Item m;
    m.sys = a.pitem_sys[it];
    m.it = it;
    const BSys& y = a.sys[m.sys];
    m.r0 = (int64_t)(it - y.pitem_off) * PT;
    m.rows = (int)min((int64_t)PT, y.n - m.r0);
    return m;
}

__device__ __forceinline__ Item item_of(int it) {
    const BArgs& a = g_bargs;
    Item m;
    m.sys = a.item_sys[it];
    m.it = it;
    const BSys& y = a.sys[m.sys];
    const int bt = item_rows(y.S);
    m.r0 = (int64_t)(it - y.item_off) * bt;
    m.rows = (int)min((int64_t)bt, y.n - m.r0);
    return m;
}

#define FOR_ITEMS for (int it_ = blockIdx.x; it_ < a.total_items; it_ += gridDim.x)
// block-product items in XCD-aware order: XCD x (workgroups blockIdx % 8 == x)
// takes the x-th eighth of the item range, so a system's items, and the P
// rows their gathers read, stay in the L2 of one XCD
#define FOR_PITEMS                                                                            \
    for (TileRange r_ = tile_range(a.total_pitems); r_.first < r_.end; r_.first += r_.step) \
        if (const int it_ = (int)r_.first; true)
#define FOR_SYS for (int sy_ = blockIdx.x; sy_ < a.nsys; sy_ += gridDim.x)
#define DISPATCH_S(Sv, CALL)                          \
    switch (Sv) {                                     \
        case 1: { constexpr int SS = 1; CALL; } break; \
        case 2: { constexpr int SS = 2; CALL; } break; \
        case 4: { constexpr int SS = 4; CALL; } break; \
        case 8: { constexpr int SS = 8; CALL; } break; \
    }

// ---------------------------------------------------------------------------
// row phases (one item: item_rows(S) rows of one system)
// ---------------------------------------------------------------------------
// D = diag(sqrt(a_jj)) (Sec. 1), b~ = D^-1 b, partial ||b||^2 and ||b~||^2
__device__ void ph_diag(const Item& m, double* sm) {
    const BArgs& a = g_bargs;
    const BSys& y = a.sys[m.sys];
    DevState* st = a.st + m.sys;
    const int32_t* rp = a.rowptr + y.rp_off;
    const int32_t* ci = a.colind + y.nz_off;
    const double* va = a.vals + y.nz_off;
    double s0 = 0.0, s1 = 0.0;
    for (int rl = threadIdx.x; rl < m.rows; rl += MB_BLOCK) {
        const int64_t r = m.r0 + rl;
        double diag = 0.0;
        for (int k = rp[r]; k < rp[r + 1]; ++k)
            if (ci[k] == r) diag += va[k];
        double dr = 1.0;
        if (a.jacobi) {
            if (!(diag > 0.0) || !finite_d(diag)) st->done = DONE_NOTSPD;
            else dr = sqrt(diag);
        }
        a.d[y.vec_off + r] = dr;
        const double bv = a.b[y.vec_off + r];
        const double bb = bv / dr;
        a.bbar[y.vec_off + r] = bb;
        s0 += bv * bv;
        s1 += bb * bb;
    }
    const int64_t it = m.it;
    const double t0 = block_sum(s0, sm);
    const double t1 = block_sum(s1, sm);
    if (threadIdx.x == 0) {
        a.ppart[it * PSTRIDE + 0] = t0;   // a block-product item (pitem_of)
        a.ppart[it * PSTRIDE + 1] = t1;
    }
}

__device__ __forceinline__ uint64_t splitmix64_at_b(uint64_t seed, uint64_t k) {
    uint64_t z = seed + (k + 1u) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// scaled values a_rc / (d_r d_c) and the Uniform(-1,1) block U (Alg. 1, the random block U)
template <int S>
__device__ void ph_scale_u(const Item& m) {
    const BArgs& a = g_bargs;
    const BSys& y = a.sys[m.sys];
    const int32_t* rp = a.rowptr + y.rp_off;
    const int32_t* ci = a.colind + y.nz_off;
    const double* va = a.vals + y.nz_off;
    double* vs = a.vals_s + y.nz_off;
    const double* d = a.d + y.vec_off;
    for (int rl = threadIdx.x; rl < m.rows; rl += MB_BLOCK) {
        const int64_t r = m.r0 + rl;
        const double dr = d[r];
        for (int k = rp[r]; k < rp[r + 1]; ++k) vs[k] = va[k] / (dr * d[ci[k]]);
    }
    const uint64_t seed = a.seed + (uint64_t)m.sys;
    double* U = a.U + y.blk_off;
    for (int e = threadIdx.x; e < m.rows * S; e += MB_BLOCK) {
        const int64_t r = m.r0 + e / S;
        const int j = e % S;
        double v = 0.0;
        if (j < y.s) {
            const uint64_t z = splitmix64_at_b(seed, (uint64_t)j * (uint64_t)y.n + (uint64_t)r);
            v = 2.0 * ((double)(z >> 11) * 0x1.0p-53) - 1.0;
        }
        U[r * S + j] = v;
    }
}

// Q = A~ P for the tile (spmm_tile, CSR slice staged in LDS); optional
// lower-triangle Gram P^T Q into part[0..E) and/or sum of Q^2 into part[2]
template <int S, int SL>
__device__ void ph_spmm(const Item& m, const double* Pb, double* Qb, bool gram,
                        bool qsq, double* sm) {
    const BArgs& a = g_bargs;
    constexpr int E = tri_count(S);
    const BSys& y = a.sys[m.sys];
    const double* P = Pb + y.blk_off;
    double* Q = Qb + y.blk_off;
    double* sQ = sm;                    // PT * 8
    double* sP = sm + PT * 8;           // PT * 8
    double* sV = sm + 2 * PT * 8;       // 8 * PT
    int32_t* sC = reinterpret_cast<int32_t*>(sm + 2 * PT * 8 + 8 * PT);   // 8 * PT ints
    int32_t* sRp = sC + 8 * PT;                                   // PT + 1 ints
    double* red = sm + BSM - MB_BLOCK;
    static_assert(2 * PT * 8 + 8 * PT + (8 * PT + PT + 2) / 2 + MB_BLOCK <= BSM, "batched LDS");
    const int tid = threadIdx.x;
    spmm_tile<S, PT, SL>(a.rowptr + y.rp_off, a.colind + y.nz_off, a.vals_s + y.nz_off, P, m.r0,
                         m.rows, sRp, sC, sV, sQ);
    if (gram) {
        // all loads first, then the LDS stores: one memory round trip
        constexpr int PPT = (PT * S + MB_BLOCK - 1) / MB_BLOCK;
        double pv[PPT];
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            const int e = tid + q * MB_BLOCK;
            const bool in = e < m.rows * S;
            const double v = P[m.r0 * S + (in ? e : 0)];
            pv[q] = in ? v : 0.0;
        }
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            const int e = tid + q * MB_BLOCK;
            if (e < PT * S) sP[e] = pv[q];
        }
    }
    double q2 = 0.0;
    for (int e = tid; e < m.rows * S; e += MB_BLOCK) {
        const double q = sQ[e];
        Q[m.r0 * S + e] = q;
        q2 += q * q;
    }
    __syncthreads();
    double* out = a.ppart + (int64_t)m.it * PSTRIDE;
    if (gram) {
        TileSums<E> gs;
        gs.init();
        int gi[TileSums<E>::EPT], gj[TileSums<E>::EPT];
#pragma unroll
        for (int k = 0; k < TileSums<E>::EPT; ++k) {
            gi[k] = gj[k] = 0;
            if (gs.ent[k] >= 0) tri_ij(gs.ent[k], gi[k], gj[k]);
        }
        gs.add_rows(m.rows, [&](int k, int r) { return sP[r * S + gi[k]] * sQ[r * S + gj[k]]; });
        gs.finish(red, out);
    }
    if (qsq) {
        const double t = block_sum(q2, red);
        if (tid == 0) out[2] = t;
    }
    __syncthreads();
}

template <int S>
__device__ void ph_spmm_dispatch(const Item& m, const double* P, double* Q,
                                 bool gram, bool qsq, double* sm) {
    const BArgs& a = g_bargs;
    if (a.sys[m.sys].SL == 2) {
        if constexpr (S * 2 <= 64) ph_spmm<S, 2>(m, P, Q, gram, qsq, sm);
    } else {
        ph_spmm<S, 1>(m, P, Q, gram, qsq, sm);
    }
}

// X0 = gamma U, X~ = 0, R = B~ - gamma Y; Gram of R and nu (setup QR partials)
template <int S>
__device__ void ph_init(const Item& m, double* sm) {
    const BArgs& a = g_bargs;
    constexpr int E = tri_count(S);
    const BSys& y = a.sys[m.sys];
    constexpr int TB = item_rows(S);   // rows per item
    const DevState* st = a.st + m.sys;
    const double g = st->gamma;
    double* sR = sm;
    double* red = sm + TB * S;
    const int64_t base = y.blk_off + m.r0 * S;
    const double* bb = a.bbar + y.vec_off + m.r0;
    const double* d = a.d + y.vec_off + m.r0;
    const int t = threadIdx.x;
    for (int e = t; e < TB * S; e += MB_BLOCK) {
        double r = 0.0;
        if (e < m.rows * S) {
            const int j = e % S;
            a.X0[base + e] = g * a.U[base + e];
            a.Xt[base + e] = 0.0;
            r = j < y.s ? bb[e / S] - g * a.Y[base + e] : 0.0;
            a.R[base + e] = r;
        }
        sR[e] = r;
    }
    __syncthreads();
    TileSums<E> gs;
    gs.init();
    int gi[TileSums<E>::EPT], gj[TileSums<E>::EPT];
#pragma unroll
    for (int k = 0; k < TileSums<E>::EPT; ++k) {
        gi[k] = gj[k] = 0;
        if (gs.ent[k] >= 0) tri_ij(gs.ent[k], gi[k], gj[k]);
    }
    gs.add_rows(m.rows, [&](int k, int r) { return sR[r * S + gi[k]] * sR[r * S + gj[k]]; });
    const int64_t it = m.it;
    double* out = a.part + it * PSTRIDE;
    gs.finish(red, out);
    for (int j = 0; j < S; ++j) {
        double v = 0.0;
        for (int rl = t; rl < m.rows; rl += MB_BLOCK) {
            const double w = d[rl] * sR[rl * S + j];
            v += w * w;
        }
        const double tot = block_sum(v, red);
        if (t == 0) out[E + j] = tot;
    }
    __syncthreads();
}

// X~ += P alpha, R -= Q alpha and V = W - Q Xi, with Gram of V and nu partials
template <int S>
__device__ void ph_update(const Item& m, double* sm) {
    const BArgs& a = g_bargs;
    constexpr int RPP = MB_BLOCK / S;
    constexpr int E = tri_count(S);
    const BSys& y = a.sys[m.sys];
    constexpr int TB = item_rows(S);   // rows per item
    const DevState* st = a.st + m.sys;
    double* sP = sm;
    double* sQ = sm + TB * S;
    double* sV = sm + 2 * TB * S;
    double* red = sm + 3 * TB * S;
    const int t = threadIdx.x, j = t % S, rl0 = t / S;
    double al[S], xi[S];
#pragma unroll
    for (int l = 0; l < S; ++l) {
        al[l] = st->alpha[l * MB_SM + j];
        xi[l] = st->Xi[l * MB_SM + j];
    }
    const int64_t base = y.blk_off + m.r0 * S;
    const double* d = a.d + y.vec_off + m.r0;
    // every load of the item (P and Q tiles, this thread's X~, R, W and d
    // entries) before the first LDS store: one memory round trip
    constexpr int RT = TB / RPP;
    Stage<TB * S> stp, stq;
    stp.load(a.P + base, m.rows * S);
    stq.load(a.Q + base, m.rows * S);
    double xo[RT], ro[RT], wo[RT], dv[RT];
#pragma unroll
    for (int k = 0; k < RT; ++k) {
        const int rl = rl0 + k * RPP;
        const int rr = rl < m.rows ? rl : 0;
        const int64_t g = base + rr * S + j;
        xo[k] = a.Xt[g];
        ro[k] = a.R[g];
        wo[k] = a.W[g];
        dv[k] = d[rr];
    }
    stp.store(sP);
    stq.store(sQ);
    __syncthreads();
    double nu = 0.0;
#pragma unroll
    for (int k = 0; k < RT; ++k) {
        const int rl = rl0 + k * RPP;
        double v = 0.0;
        if (rl < m.rows) {
            const int64_t g = base + rl * S + j;
            double tx = 0.0, tr = 0.0, tv = 0.0;
#pragma unroll
            for (int l = 0; l < S; ++l) {
                const double p = sP[rl * S + l], q = sQ[rl * S + l];
                tx += p * al[l];
                tr += q * al[l];
                tv += q * xi[l];
            }
            const double xn = xo[k] + tx;
            const double rn = ro[k] - tr;
            v = wo[k] - tv;
            a.Xt[g] = xn;
            a.R[g] = rn;
            a.W[g] = v;
            const double dr = dv[k] * rn;
            nu += dr * dr;
        }
        sV[rl * S + j] = v;
    }
    __syncthreads();
    TileSums<E> gs;
    gs.init();
    int gi[TileSums<E>::EPT], gj[TileSums<E>::EPT];
#pragma unroll
    for (int k = 0; k < TileSums<E>::EPT; ++k) {
        gi[k] = gj[k] = 0;
        if (gs.ent[k] >= 0) tri_ij(gs.ent[k], gi[k], gj[k]);
    }
    gs.add_rows(m.rows, [&](int k, int r) { return sV[r * S + gi[k]] * sV[r * S + gj[k]]; });
    const int64_t it = m.it;
    double* out = a.part + it * PSTRIDE;
    gs.finish(red, out);
    red[t] = nu;
    column_sums<S>(red);
    if (t < S) out[E + t] = red[t];
    __syncthreads();
}

// W = V M, P = W + P Z^T (FIRST: P = W, V read from R)
template <int S, int FIRST>
__device__ void ph_dir(const Item& m, double* sm) {
    const BArgs& a = g_bargs;
    constexpr int RPP = MB_BLOCK / S;
    const BSys& y = a.sys[m.sys];
    constexpr int TB = item_rows(S);   // rows per item
    const DevState* st = a.st + m.sys;
    double* sV = sm;
    double* sP = sm + TB * S;
    const int t = threadIdx.x, j = t % S, rl0 = t / S;
    double mm[S], z[S];
#pragma unroll
    for (int l = 0; l < S; ++l) {
        mm[l] = st->M[l * MB_SM + j];
        z[l] = st->Z[j * MB_SM + l];
    }
    const int64_t base = y.blk_off + m.r0 * S;
    const double* V = FIRST ? a.R : a.W;
    Stage<TB * S> stv, stp;   // all loads before the LDS stores
    stv.load(V + base, m.rows * S);
    if (!FIRST) stp.load(a.P + base, m.rows * S);
    stv.store(sV);
    if (!FIRST) stp.store(sP);
    __syncthreads();
    for (int rl = rl0; rl < m.rows; rl += RPP) {
        double w = 0.0;
#pragma unroll
        for (int l = 0; l < S; ++l) w += sV[rl * S + l] * mm[l];
        double p = w;
        if (!FIRST) {
            double acc = 0.0;
#pragma unroll
            for (int l = 0; l < S; ++l) acc += sP[rl * S + l] * z[l];
            p = w + acc;
        }
        a.W[base + rl * S + j] = w;
        a.P[base + rl * S + j] = p;
    }
    __syncthreads();
}

// double-double Gram of [B^, b] for the least-squares termination,
// B^ = B - D R formed entry by entry as b_r - (d_r R_rj); columns j >= s zero
template <int S>
__device__ void ph_ls_gram(const Item& m, double* sm) {
    const BArgs& a = g_bargs;
    constexpr int NC = S + 1;
    constexpr int E = tri_count(NC);
    static_assert(2 * E <= PSTRIDE, "least-squares partials per item");
    const BSys& y = a.sys[m.sys];
    constexpr int TB = item_rows(S);   // rows per item
    double* sM = sm;
    double* red = sm + TB * NC;
    static_assert(TB * NC + 2 * MB_BLOCK <= BSM, "batched LDS");
    const int t = threadIdx.x;
    const int s = y.s;
    const int64_t base = y.blk_off + m.r0 * S;
    const double* d = a.d + y.vec_off + m.r0;
    const double* b = a.b + y.vec_off + m.r0;
    for (int e = t; e < TB * S; e += MB_BLOCK) {
        const int rl = e / S, j = e % S;
        sM[rl * NC + j] = (rl < m.rows && j < s) ? bhat_entry(b[rl], d[rl], a.R[base + e]) : 0.0;
    }
    for (int rl = t; rl < TB; rl += MB_BLOCK) sM[rl * NC + S] = rl < m.rows ? b[rl] : 0.0;
    __syncthreads();
    TileSumsDD<E> gs;
    gs.init();
    int gi[TileSumsDD<E>::EPT], gj[TileSumsDD<E>::EPT];
#pragma unroll
    for (int k = 0; k < TileSumsDD<E>::EPT; ++k) {
        gi[k] = gj[k] = 0;
        if (gs.ent[k] >= 0) tri_ij(gs.ent[k], gi[k], gj[k]);
    }
    gs.add_rows(m.rows, [&](int k, int r) {
        return make_double2(sM[r * NC + gi[k]], sM[r * NC + gj[k]]);
    });
    const int64_t it = m.it;
    gs.finish(red, a.part + it * PSTRIDE);
    __syncthreads();
}

// x = D^-1 (X~ + X0) c^, r = b - B^ c^ (sums over the columns in column
// order, rounded as written), partial ||r||^2 into part[0]
template <int S>
__device__ void ph_ls_apply(const Item& m, double* sm) {
#pragma clang fp contract(off)
    const BArgs& a = g_bargs;
    const BSys& y = a.sys[m.sys];
    const DevState* st = a.st + m.sys;
    const int64_t base = y.blk_off + m.r0 * S;
    const double* d = a.d + y.vec_off + m.r0;
    const double* b = a.b + y.vec_off + m.r0;
    double* x = a.x + y.vec_off + m.r0;
    const int s = y.s;
    double c[S];
#pragma unroll
    for (int j = 0; j < S; ++j) c[j] = st->chat[j];
    double s2 = 0.0;
    for (int rl = threadIdx.x; rl < m.rows; rl += MB_BLOCK) {
        double ax = 0.0, ab = 0.0;
        const double dr = d[rl], br = b[rl];
#pragma unroll
        for (int j = 0; j < S; ++j) {
            if (j < s) {
                ax += (a.Xt[base + rl * S + j] + a.X0[base + rl * S + j]) * c[j];
                ab += bhat_entry(br, dr, a.R[base + rl * S + j]) * c[j];
            }
        }
        x[rl] = ax / dr;
        const double res = br - ab;
        s2 += res * res;
    }
    const int64_t it = m.it;
    const double tot = block_sum(s2, sm);
    if (threadIdx.x == 0) a.part[it * PSTRIDE + 0] = tot;
}

// best column when the combination was not accepted; x = 0 for b = 0
template <int S>
__device__ void ph_select(const Item& m) {
    const BArgs& a = g_bargs;
    const BSys& y = a.sys[m.sys];
    const DevState* st = a.st + m.sys;
    double* x = a.x + y.vec_off + m.r0;
    if (st->done == DONE_ZERO_RHS || !st->ready) {
        for (int rl = threadIdx.x; rl < m.rows; rl += MB_BLOCK) x[rl] = 0.0;
        return;
    }
    if (st->accepted) return;
    const int h = st->h;
    const int64_t base = y.blk_off + m.r0 * S;
    const double* d = a.d + y.vec_off + m.r0;
    for (int rl = threadIdx.x; rl < m.rows; rl += MB_BLOCK)
        x[rl] = (a.Xt[base + rl * S + h] + a.X0[base + rl * S + h]) / d[rl];
}

// ||b - A x||^2 partial on the original values into part[1]
__device__ void ph_resid(const Item& m, double* sm) {
    const BArgs& a = g_bargs;
    const BSys& y = a.sys[m.sys];
    const int32_t* rp = a.rowptr + y.rp_off;
    const int32_t* ci = a.colind + y.nz_off;
    const double* va = a.vals + y.nz_off;
    const double* x = a.x + y.vec_off;
    const double* b = a.b + y.vec_off;
    double s2 = 0.0;
    for (int rl = threadIdx.x; rl < m.rows; rl += MB_BLOCK) {
        const int64_t r = m.r0 + rl;
        double acc = 0.0;
        for (int k = rp[r]; k < rp[r + 1]; ++k) acc += va[k] * x[ci[k]];
        const double e = b[r] - acc;
        s2 += e * e;
    }
    const int64_t it = m.it;
    const double tot = block_sum(s2, sm);
    if (threadIdx.x == 0) a.ppart[it * PSTRIDE + 1] = tot;   // block-product item
}

// ||b - A x_h||^2 partial into part[2], x_h = D^-1 (X~ + X0)_h read from the
// blocks (the best column, when the accepted combination misses the tolerance)
template <int S>
__device__ void ph_resid_best(const Item& m, double* sm) {
    const BArgs& a = g_bargs;
    const BSys& y = a.sys[m.sys];
    const int32_t* rp = a.rowptr + y.rp_off;
    const int32_t* ci = a.colind + y.nz_off;
    const double* va = a.vals + y.nz_off;
    const double* b = a.b + y.vec_off;
    const double* d = a.d + y.vec_off;
    const double* Xt = a.Xt + y.blk_off;
    const double* X0 = a.X0 + y.blk_off;
    const int h = a.st[m.sys].h;
    double s2 = 0.0;
    for (int rl = threadIdx.x; rl < m.rows; rl += MB_BLOCK) {
        const int64_t r = m.r0 + rl;
        double acc = 0.0;
        for (int k = rp[r]; k < rp[r + 1]; ++k) {
            const int64_t c = ci[k];
            acc += va[k] * ((Xt[c * S + h] + X0[c * S + h]) / d[c]);
        }
        const double e = b[r] - acc;
        s2 += e * e;
    }
    const int64_t it = m.it;
    const double tot = block_sum(s2, sm);
    if (threadIdx.x == 0) a.ppart[it * PSTRIDE + 2] = tot;   // block-product item
}

// an accepted combination whose true residual misses the tolerance
__device__ inline bool needs_pick(const DevState* st) {
    return st->done == DONE_CONVERGED && st->accepted && !(st->rel_true < st->tol);
}

// the combination passed the test on B - R but gave way to the best column
__device__ inline bool was_picked(const DevState* st) {
    return st->done == DONE_CONVERGED && !st->accepted && st->ls_ok && finite_d(st->rel_ls) &&
           st->rel_ls < st->tol;
}

// sum of ppart[slot] over a system's block-product items (fixed order)
__device__ double sys_psum(const BSys& y, int slot, double* sm) {
    const BArgs& a = g_bargs;
    reduce_partials(a.ppart + (int64_t)y.pitem_off * PSTRIDE + slot, y.pntile, 1, PSTRIDE, sm,
                    sm + 8);
    return sm[0];
}

// sum of part[slot] over a system's items (fixed order), result to thread 0
__device__ double sys_sum(const BSys& y, int slot, double* sm) {
    const BArgs& a = g_bargs;
    reduce_partials(a.part + (int64_t)y.item_off * PSTRIDE + slot, y.ntile, 1, PSTRIDE, sm,
                    sm + 8);
    return sm[0];
}

// ---------------------------------------------------------------------------
// the persistent kernel
// ---------------------------------------------------------------------------
// one body for every phase: the register cap (128) keeps four waves per SIMD,
// four workgroups per CU, as many as its 32 KB of LDS allows
__global__ __launch_bounds__(MB_BLOCK) __attribute__((amdgpu_waves_per_eu(4))) void k_batch() {
    const BArgs& a = g_bargs;
    __shared__ double sm[BSM];
    __shared__ int smi[48];
    int* flag = smi + 40;
    BCtl* ctl = a.ctl;
    int nstamp = 0;
    auto stamp = [&]() {
        if (a.tstamp && blockIdx.x == 0 && threadIdx.x == 0) a.tstamp[nstamp] = wall_clock64();
        ++nstamp;
    };
    stamp();
#define SYNC_OR_QUIT \
    if (!grid_sync(ctl, a.spin_limit, flag)) return; \
    stamp();

    // --- setup: scaling, b~, ||b||
    // (the CSR row phases take the 128-row block-product items)
    FOR_PITEMS {
        const Item m = pitem_of(it_);
        ph_diag(m, sm);
    }
    SYNC_OR_QUIT
    FOR_PITEMS {
        const Item m = pitem_of(it_);
        DISPATCH_S(a.sys[m.sys].S, ph_scale_u<SS>(m))
    }
    SYNC_OR_QUIT
    // initial guess: Y = A~ U and ||Y||_F^2
    FOR_PITEMS {
        const Item m = pitem_of(it_);
        DISPATCH_S(a.sys[m.sys].S, ph_spmm_dispatch<SS>(m, a.U, a.Y, false, true, sm))
    }
    SYNC_OR_QUIT
    FOR_SYS {
        const BSys& y = a.sys[sy_];
        DevState* st = a.st + sy_;
        const double sb = sys_psum(y, 0, sm);
        __syncthreads();
        const double sbb = sys_psum(y, 1, sm);
        __syncthreads();
        const double sy = sys_psum(y, 2, sm);
        if (threadIdx.x == 0) {
            const double bn = sqrt(sb);
            st->bnorm = bn;
            st->bbar_norm = sqrt(sbb);
            if (!finite_d(bn)) st->done = DONE_NONFINITE;
            else if (bn == 0.0) st->done = DONE_ZERO_RHS;
            else if (!st->done) {
                const double g = sqrt((double)y.s * sbb) / sqrt(sy);
                st->gamma = g;
                if (!finite_d(g)) st->done = DONE_NONFINITE;
            }
        }
        __syncthreads();
    }
    SYNC_OR_QUIT
    // scaled right-hand sides, R0 and the partials of the first QR
    FOR_ITEMS {
        const Item m = item_of(it_);
        if (a.st[m.sys].done) continue;
        DISPATCH_S(a.sys[m.sys].S, ph_init<SS>(m, sm))
    }
    SYNC_OR_QUIT
    FOR_SYS {
        const BSys& y = a.sys[sy_];
        DevState* st = a.st + sy_;
        if (st->done) continue;
        DISPATCH_S(y.S, tail_qr_body<SS>(a.part + (int64_t)y.item_off * PSTRIDE, y.ntile, PSTRIDE,
                                         st, nullptr, 1, sm, smi))
        __syncthreads();
    }
    SYNC_OR_QUIT
    FOR_ITEMS {
        const Item m = item_of(it_);
        if (a.st[m.sys].done) continue;
        DISPATCH_S(a.sys[m.sys].S, (ph_dir<SS, 1>(m, sm)))
    }
    FOR_SYS {
        if (threadIdx.x == 0 && !a.st[sy_].done)
            __hip_atomic_fetch_add(&ctl->active, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    SYNC_OR_QUIT

    // --- the iteration loop (Xi to the new Sigma) for every active system
    for (int64_t loop = 0; loop <= (int64_t)a.max_iter + 1; ++loop) {
        FOR_PITEMS {
            const Item m = pitem_of(it_);
            if (a.st[m.sys].done) continue;
            DISPATCH_S(a.sys[m.sys].S, ph_spmm_dispatch<SS>(m, a.P, a.Q, true, false, sm))
        }
        SYNC_OR_QUIT
        FOR_SYS {
            const BSys& y = a.sys[sy_];
            DevState* st = a.st + sy_;
            if (st->done) continue;
            DISPATCH_S(y.S, tail_xi_body<SS>(a.ppart + (int64_t)y.pitem_off * PSTRIDE, y.pntile,
                                             PSTRIDE, st, sm, smi))
            __syncthreads();
            if (threadIdx.x == 0 && st->done)
                __hip_atomic_fetch_add(&ctl->active, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __syncthreads();
        }
        SYNC_OR_QUIT
        FOR_ITEMS {
            const Item m = item_of(it_);
            if (a.st[m.sys].done) continue;
            DISPATCH_S(a.sys[m.sys].S, ph_update<SS>(m, sm))
        }
        SYNC_OR_QUIT
        FOR_SYS {
            const BSys& y = a.sys[sy_];
            DevState* st = a.st + sy_;
            if (st->done) continue;
            int fin = 0;
            DISPATCH_S(y.S, fin = tail_qr_body<SS>(a.part + (int64_t)y.item_off * PSTRIDE, y.ntile,
                                                   PSTRIDE, st, nullptr, 0, sm, smi))
            __syncthreads();
            if (threadIdx.x == 0 && fin)
                __hip_atomic_fetch_add(&ctl->active, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __syncthreads();
        }
        SYNC_OR_QUIT
        if (threadIdx.x == 0)
            flag[1] = __hip_atomic_load(&ctl->active, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const int still = flag[1];
        __syncthreads();
        if (still <= 0) break;
        FOR_ITEMS {
            const Item m = item_of(it_);
            if (a.st[m.sys].done) continue;
            DISPATCH_S(a.sys[m.sys].S, (ph_dir<SS, 0>(m, sm)))
        }
        SYNC_OR_QUIT
        if (blockIdx.x == 0 && threadIdx.x == 0) ctl->loops = (int)(loop + 1);
    }

    // --- termination (least-squares combination)
    FOR_ITEMS {
        const Item m = item_of(it_);
        if (a.st[m.sys].done != DONE_CONVERGED) continue;
        DISPATCH_S(a.sys[m.sys].S, ph_ls_gram<SS>(m, sm))
    }
    SYNC_OR_QUIT
    FOR_SYS {
        const BSys& y = a.sys[sy_];
        DevState* st = a.st + sy_;
        if (st->done != DONE_CONVERGED) continue;
        DISPATCH_S(y.S, tail_ls_body<SS>(a.part + (int64_t)y.item_off * PSTRIDE, y.ntile, PSTRIDE,
                                         y.n, st, sm, smi))
        __syncthreads();
    }
    SYNC_OR_QUIT
    FOR_ITEMS {
        const Item m = item_of(it_);
        if (a.st[m.sys].done != DONE_CONVERGED) continue;
        DISPATCH_S(a.sys[m.sys].S, ph_ls_apply<SS>(m, sm))
    }
    SYNC_OR_QUIT
    FOR_SYS {
        const BSys& y = a.sys[sy_];
        DevState* st = a.st + sy_;
        if (st->done != DONE_CONVERGED) {
            if (threadIdx.x == 0) st->accepted = 0;
            continue;
        }
        const double s2 = sys_sum(y, 0, sm);
        if (threadIdx.x == 0) {
            const double rel = sqrt(s2) / st->bnorm;
            st->rel_ls = rel;
            st->accepted = st->ls_ok && finite_d(rel) && rel < st->tol;
        }
        __syncthreads();
    }
    SYNC_OR_QUIT
    FOR_ITEMS {
        const Item m = item_of(it_);
        DISPATCH_S(a.sys[m.sys].S, ph_select<SS>(m))
    }
    SYNC_OR_QUIT
    FOR_PITEMS {
        const Item m = pitem_of(it_);
        ph_resid(m, sm);
    }
    SYNC_OR_QUIT
    FOR_SYS {
        const BSys& y = a.sys[sy_];
        DevState* st = a.st + sy_;
        const double s2 = sys_psum(y, 1, sm);
        if (threadIdx.x == 0) st->rel_true = st->done == DONE_ZERO_RHS ? 0.0 : sqrt(s2) / st->bnorm;
        __syncthreads();
    }
    SYNC_OR_QUIT
    FOR_PITEMS {
        const Item m = pitem_of(it_);
        if (!needs_pick(a.st + m.sys)) continue;
        DISPATCH_S(a.sys[m.sys].S, ph_resid_best<SS>(m, sm))
    }
    SYNC_OR_QUIT
    FOR_SYS {
        const BSys& y = a.sys[sy_];
        DevState* st = a.st + sy_;
        if (!needs_pick(st)) continue;
        const double s2 = sys_psum(y, 2, sm);
        if (threadIdx.x == 0) {
            const double rel_h = sqrt(s2) / st->bnorm;
            if (rel_h < st->rel_true) {
                st->accepted = 0;
                st->rel_true = rel_h;
            }
        }
        __syncthreads();
    }
    SYNC_OR_QUIT
    FOR_ITEMS {
        const Item m = item_of(it_);
        if (!was_picked(a.st + m.sys)) continue;
        DISPATCH_S(a.sys[m.sys].S, ph_select<SS>(m))
    }
    stamp();
#undef SYNC_OR_QUIT
}

// the leading `head_words` 32-bit words of every system's state, packed for one
// copy out
__global__ void k_batch_state_pack(int nsys, const DevState* __restrict__ st, int head_words,
                                   uint32_t* __restrict__ out) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)nsys * head_words;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / head_words;
        const int w = (int)(e % head_words);
        out[e] = reinterpret_cast<const uint32_t*>(st + i)[w];
    }
}

__global__ void k_batch_state_init(int nsys, DevState* st, const BSys* sys, int max_iter,
                                   double tol, double tau) {
    const int i = blockIdx.x;
    if (i >= nsys) return;
    DevState* s = st + i;
    double* raw = reinterpret_cast<double*>(s);
    const int nd = (int)(sizeof(DevState) / sizeof(double));
    for (int e = threadIdx.x; e < nd; e += blockDim.x) raw[e] = 0.0;
    __syncthreads();
    if (threadIdx.x == 0) {
        s->s = sys[i].s;
        s->max_iter = max_iter;
        s->tol = tol;
        s->tol0 = tol;
        s->tau = tau;
        s->width = sys[i].s;
    }
    if (threadIdx.x < MB_SM) s->active[threadIdx.x] = threadIdx.x < sys[i].s;
}

// ---------------------------------------------------------------------------
// host side: a batch context uploads the systems once and keeps its captured
// graph; each solve writes the kernel's arguments, resets the per-system
// states and replays the graph
// ---------------------------------------------------------------------------
struct BatchBufs {
    std::vector<void*> ptrs;
    ~BatchBufs() {
        for (void* p : ptrs) (void)hipFree(p);
    }
    template <class T>
    hipError_t alloc(T** p, size_t count) {
        hipError_t e = hipMalloc((void**)p, sizeof(T) * std::max<size_t>(count, 1));
        if (e == hipSuccess) ptrs.push_back((void*)*p);
        return e;
    }
};

// row-length class of a system (average nonzeros per row) for the choice of
// lane groups per row: [0, 16), [16, 48), [48, ...)
static int row_class(int64_t n, int64_t nnz) {
    const double r = (double)nnz / (double)std::max<int64_t>(n, 1);
    return r < 16.0 ? 0 : (r < 48.0 ? 1 : 2);
}
// untuned: a second lane group per row for long rows
static int default_slots(int cls) { return cls == 0 ? 1 : 2; }

// tuned lane groups per row, per (padded width, row class), kept for the
// process: a later batch whose classes are all known skips those trials
static std::mutex g_tune_mu;
static std::map<std::pair<int, int>, int> g_slot_cache;

// the kernel's arguments live in one device symbol: one batched solve at a
// time in this process
static std::mutex g_batch_mu;

struct BatchCtx {
    int device = 0;
    int nsys = 0;
    mbpcg_mem mem = MBPCG_MEM_DEVICE;
    std::vector<mbpcg_system> sys;   // the caller's descriptors (x receives the results)
    std::vector<BSys> hs;
    int items = 0, pitems = 0;
    BatchBufs B;
    BArgs a;                 // device pointers; the per-solve fields are set by each solve
    BSys* d_sys = nullptr;
    double* d_x = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr, ev0 = nullptr, ev1 = nullptr;
    int resident = 0;        // workgroups that fit on the GPU at once
    int grid = 0;            // grid of the persistent kernel
    hipGraphExec_t exec = nullptr;
    int exec_grid = 0;
    long long* d_ts = nullptr;
    int64_t ts_cap = 0;
    std::string err;
    ~BatchCtx() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (d_ts) (void)hipFree(d_ts);
        if (ev) (void)hipEventDestroy(ev);
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
        if (stream) (void)hipStreamDestroy(stream);
    }
};

BatchCtx* batch_new() { return new (std::nothrow) BatchCtx; }
void batch_delete(BatchCtx* c) { delete c; }
const char* batch_error(const BatchCtx* c) { return c ? c->err.c_str() : ""; }

#define BCK(expr)                                                              \
    do {                                                                       \
        hipError_t _e = (expr);                                                \
        if (_e != hipSuccess) {                                                \
            (void)hipGetLastError(); /* reported through the status */         \
            c.err = std::string(#expr) + ": " + hipGetErrorString(_e);        \
            return _e == hipErrorOutOfMemory ? MBPCG_ERR_OOM : MBPCG_ERR_HIP;  \
        }                                                                      \
    } while (0)

mbpcg_status batch_create(BatchCtx& c, int32_t nsys, const mbpcg_system* systems, mbpcg_mem mem,
                          hipStream_t user_stream) {
    c.nsys = nsys;
    c.mem = mem;
    c.sys.assign(systems, systems + nsys);
    c.hs.resize(nsys);
    std::vector<int32_t> item_sys, pitem_sys;
    int64_t rp = 0, nz = 0, vec = 0, blk = 0;
    int items = 0, pitems = 0;
    for (int i = 0; i < nsys; ++i) {
        const mbpcg_system& y = systems[i];
        BSys& b = c.hs[i];
        b.n = y.n;
        b.rp_off = rp;
        b.nz_off = nz;
        b.vec_off = vec;
        b.blk_off = blk;
        b.s = y.s;
        b.S = padded_width(y.s);
        b.SL = default_slots(row_class(y.n, y.nnz));
        b.ntile = (int)((y.n + item_rows(b.S) - 1) / item_rows(b.S));
        b.item_off = items;
        b.pntile = (int)((y.n + PT - 1) / PT);
        b.pitem_off = pitems;
        b.pad = 0;
        for (int t = 0; t < b.ntile; ++t) item_sys.push_back(i);
        for (int t = 0; t < b.pntile; ++t) pitem_sys.push_back(i);
        items += b.ntile;
        pitems += b.pntile;
        rp += y.n + 1;
        nz += y.nnz;
        vec += y.n;
        blk += y.n * b.S;
        if (items >= INT32_MAX / 2 || pitems >= INT32_MAX / 2) {
            c.err = "batch too large";
            return MBPCG_ERR_UNSUPPORTED;
        }
    }
    c.items = items;
    c.pitems = pitems;
    BCK(hipGetDevice(&c.device));
    BCK(hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking));
    BCK(hipEventCreateWithFlags(&c.ev, hipEventDisableTiming));
    BCK(hipEventCreate(&c.ev0));
    BCK(hipEventCreate(&c.ev1));
    BCK(hipEventRecord(c.ev, user_stream));
    BCK(hipStreamWaitEvent(c.stream, c.ev, 0));

    BArgs& a = c.a;
    memset(&a, 0, sizeof(a));
    int32_t *d_rp, *d_ci, *d_items, *d_pitems;
    double *d_va, *d_vs, *d_b, *d_d, *d_bb;
    DevState* d_st;
    BCtl* d_ctl;
    BatchBufs& B = c.B;
    BCK(B.alloc(&d_rp, rp));
    BCK(B.alloc(&d_ci, nz));
    BCK(B.alloc(&d_va, nz));
    BCK(B.alloc(&d_vs, nz));
    BCK(B.alloc(&d_b, vec));
    BCK(B.alloc(&c.d_x, vec));
    BCK(B.alloc(&d_d, vec));
    BCK(B.alloc(&d_bb, vec));
    BCK(B.alloc(&d_items, items));
    BCK(B.alloc(&d_pitems, pitems));
    BCK(B.alloc(&c.d_sys, nsys));
    BCK(B.alloc(&d_st, nsys));
    BCK(B.alloc(&d_ctl, 1));
    double* blocks[8];
    for (auto& q : blocks) BCK(B.alloc(&q, blk));
    double *d_part, *d_ppart;
    BCK(B.alloc(&d_part, (size_t)items * PSTRIDE));
    BCK(B.alloc(&d_ppart, (size_t)pitems * PSTRIDE));

    const hipMemcpyKind kind = mem == MBPCG_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    for (int i = 0; i < nsys; ++i) {
        const mbpcg_system& y = systems[i];
        const BSys& b = c.hs[i];
        BCK(hipMemcpyAsync(d_rp + b.rp_off, y.rowptr, sizeof(int32_t) * (y.n + 1), kind, c.stream));
        if (y.nnz > 0) {
            BCK(hipMemcpyAsync(d_ci + b.nz_off, y.colind, sizeof(int32_t) * y.nnz, kind, c.stream));
            BCK(hipMemcpyAsync(d_va + b.nz_off, y.vals, sizeof(double) * y.nnz, kind, c.stream));
        }
        BCK(hipMemcpyAsync(d_b + b.vec_off, y.b, sizeof(double) * y.n, kind, c.stream));
    }
    BCK(hipMemcpyAsync(d_items, item_sys.data(), sizeof(int32_t) * items, hipMemcpyHostToDevice,
                       c.stream));
    BCK(hipMemcpyAsync(d_pitems, pitem_sys.data(), sizeof(int32_t) * pitems,
                       hipMemcpyHostToDevice, c.stream));
    BCK(hipMemcpyAsync(c.d_sys, c.hs.data(), sizeof(BSys) * nsys, hipMemcpyHostToDevice, c.stream));
    BCK(hipStreamSynchronize(c.stream));

    a.nsys = nsys;
    a.total_items = items;
    a.total_pitems = pitems;
    a.pitem_sys = d_pitems;
    a.ppart = d_ppart;
    a.spin_limit = batch_spin_limit();
    a.sys = c.d_sys;
    a.st = d_st;
    a.ctl = d_ctl;
    a.item_sys = d_items;
    a.rowptr = d_rp;
    a.colind = d_ci;
    a.vals = d_va;
    a.vals_s = d_vs;
    a.b = d_b;
    a.x = c.d_x;
    a.d = d_d;
    a.bbar = d_bb;
    a.U = blocks[0];
    a.Y = blocks[1];
    a.X0 = blocks[2];
    a.Xt = blocks[3];
    a.R = blocks[4];
    a.W = blocks[5];
    a.P = blocks[6];
    a.Q = blocks[7];
    a.part = d_part;

    // grid: every workgroup co-resident (the barrier needs it)
    int per_cu = 0, cus = 0;
    BCK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch, MB_BLOCK, 0));
    BCK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c.device));
    if (per_cu < 1) {
        c.err = "batched kernel does not fit on a compute unit";
        return MBPCG_ERR_HIP;
    }
    c.resident = per_cu * cus;
    c.grid = std::max(1, std::min(std::max(items, pitems), c.resident));
    return MBPCG_OK;
}

// lane groups per row of every system of class (S, cls); uploads the table
static mbpcg_status set_slots(BatchCtx& c, int S, int cls, int SL) {
    for (int i = 0; i < c.nsys; ++i)
        if (c.hs[i].S == S && row_class(c.sys[i].n, c.sys[i].nnz) == cls) c.hs[i].SL = SL;
    BCK(hipMemcpyAsync(c.d_sys, c.hs.data(), sizeof(BSys) * c.nsys, hipMemcpyHostToDevice,
                       c.stream));
    BCK(hipStreamSynchronize(c.stream));
    return MBPCG_OK;
}

mbpcg_status batch_solve(BatchCtx& c, const mbpcg_params& p, mbpcg_info* per_system,
                         hipStream_t user_stream, double* kernel_ms) {
    std::lock_guard<std::mutex> lk(g_batch_mu);
    BCK(hipSetDevice(c.device));
    const auto t0 = std::chrono::steady_clock::now();
    BCK(hipEventRecord(c.ev, user_stream));
    BCK(hipStreamWaitEvent(c.stream, c.ev, 0));
    const int nsys = c.nsys;
    BArgs& a = c.a;
    // profile: one steady-clock stamp per grid barrier (setup 7, 5 per
    // iteration, 4 in the last, termination 9, plus start and end)
    const int64_t max_loops = std::min<int64_t>(p.max_iter, INT32_MAX) + 2;
    const int64_t nstamps = 1 + 7 + 5 * max_loops + 4 + BATCH_TERM_BARRIERS + 1;
    if (p.profile && nstamps > c.ts_cap) {
        if (c.d_ts) (void)hipFree(c.d_ts);
        c.d_ts = nullptr;
        c.ts_cap = 0;
        BCK(hipMalloc(&c.d_ts, sizeof(long long) * nstamps));
        c.ts_cap = nstamps;
    }
    a.max_iter = (int)p.max_iter;
    a.jacobi = p.precond == MBPCG_PRECOND_JACOBI;
    a.tol = p.tol;
    a.tau = p.tau > 0 ? p.tau : 1e-12;
    a.seed = p.seed;
    a.tstamp = p.profile ? c.d_ts : nullptr;
    a.spin_limit = batch_spin_limit();
    BCK(hipMemsetAsync(a.ctl, 0, sizeof(BCtl), c.stream));
    hipLaunchKernelGGL(k_batch_state_init, dim3(nsys), dim3(MB_BLOCK), 0, c.stream, nsys, a.st,
                       c.d_sys, (int)p.max_iter, p.tol, a.tau);
    BCK(hipGetLastError());
    BCK(hipMemcpyToSymbolAsync(HIP_SYMBOL(g_bargs), &a, sizeof(BArgs), 0, hipMemcpyHostToDevice,
                               c.stream));
    // the persistent kernel, captured once per grid and replayed
    if (!c.exec || c.exec_grid != c.grid) {
        if (c.exec) (void)hipGraphExecDestroy(c.exec);
        c.exec = nullptr;
        hipStream_t cs = nullptr;
        BCK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        hipGraph_t graph = nullptr;
        hipError_t be = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (be == hipSuccess) {
            hipLaunchKernelGGL(k_batch, dim3(c.grid), dim3(MB_BLOCK), 0, cs);
            const hipError_t le = hipGetLastError();
            const hipError_t ce = hipStreamEndCapture(cs, &graph);
            be = le != hipSuccess ? le : ce;
        }
        (void)hipStreamDestroy(cs);
        if (be != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            c.err = std::string("capture of the batched kernel failed: ") + hipGetErrorString(be);
            return MBPCG_ERR_HIP;
        }
        const hipError_t ie = hipGraphInstantiate(&c.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ie != hipSuccess) {
            c.exec = nullptr;
            c.err = std::string("instantiate: ") + hipGetErrorString(ie);
            return MBPCG_ERR_HIP;
        }
        c.exec_grid = c.grid;
    }
    BCK(hipEventRecord(c.ev0, c.stream));
    BCK(hipGraphLaunch(c.exec, c.stream));
    BCK(hipEventRecord(c.ev1, c.stream));
    BCK(hipEventSynchronize(c.ev1));
    float kms = 0.f;
    BCK(hipEventElapsedTime(&kms, c.ev0, c.ev1));
    const double ms_kernel = kms;
    if (kernel_ms) *kernel_ms = ms_kernel;

    BCtl hctl;
    BCK(hipMemcpy(&hctl, a.ctl, sizeof(BCtl), hipMemcpyDeviceToHost));
    if (hctl.abort) {
        c.err = "batched kernel: grid barrier wait exceeded its bound (grid not co-resident?)";
        return MBPCG_ERR_HIP;
    }
    // results
    const size_t head = offsetof(DevState, Xi);
    static_assert(offsetof(DevState, Xi) % 4 == 0, "state head");
    std::vector<char> hst(head * (size_t)nsys);
    uint32_t* d_pack = reinterpret_cast<uint32_t*>(a.part);   // the partials are free now
    hipLaunchKernelGGL(k_batch_state_pack, dim3(std::min(nsys, 1024)), dim3(MB_BLOCK), 0, c.stream,
                       nsys, a.st, (int)(head / 4), d_pack);
    BCK(hipGetLastError());
    BCK(hipMemcpyAsync(hst.data(), d_pack, head * (size_t)nsys, hipMemcpyDeviceToHost, c.stream));
    const hipMemcpyKind back = c.mem == MBPCG_MEM_HOST ? hipMemcpyDeviceToHost
                                                       : hipMemcpyDeviceToDevice;
    for (int i = 0; i < nsys; ++i)
        BCK(hipMemcpyAsync(c.sys[i].x, c.d_x + c.hs[i].vec_off, sizeof(double) * c.sys[i].n, back,
                           c.stream));
    BCK(hipStreamSynchronize(c.stream));
    // phase totals as in mbpcg_info.ms_phase: 0 block product, 1 Xi tail,
    // 2 update, 3 QR tail, 4 direction update, 5 termination, 6 setup
    double ph_ms[7] = {0, 0, 0, 0, 0, 0, 0};
    if (p.profile) {
        const int64_t L = hctl.loops;
        const int64_t used = 1 + 7 + 5 * L + 4 + BATCH_TERM_BARRIERS + 1;
        std::vector<long long> ts(used);
        BCK(hipMemcpy(ts.data(), c.d_ts, sizeof(long long) * used, hipMemcpyDeviceToHost));
        int khz = 0;
        BCK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, c.device));
        const double ms_per_tick = khz > 0 ? 1.0 / khz : 0.0;
        auto span = [&](int64_t i) { return (double)(ts[i] - ts[i - 1]) * ms_per_tick; };
        for (int64_t i = 1; i <= 7; ++i) ph_ms[6] += span(i);
        for (int64_t it = 0; it <= L; ++it)
            for (int q = 0; q < (it < L ? 5 : 4); ++q) ph_ms[q] += span(8 + 5 * it + q);
        for (int64_t i = 8 + 5 * L + 4; i < used; ++i) ph_ms[5] += span(i);
    }
    const double ms_all =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    mbpcg_status worst = MBPCG_OK;
    for (int i = 0; i < nsys; ++i) {
        DevState s;
        memcpy(&s, hst.data() + head * i, head);
        mbpcg_status st;
        switch (s.done) {
            case DONE_CONVERGED: case DONE_ZERO_RHS: st = MBPCG_OK; break;
            case DONE_MAXITER: st = MBPCG_NOT_CONVERGED; break;
            case DONE_BREAKDOWN: st = MBPCG_ERR_BREAKDOWN; break;
            case DONE_NOTSPD: st = MBPCG_ERR_NOT_SPD; break;
            case DONE_NONFINITE: st = MBPCG_ERR_NONFINITE; break;
            default: st = MBPCG_NOT_CONVERGED; break;
        }
        if (st != MBPCG_OK && (worst == MBPCG_OK || st < 0)) worst = st;
        if (per_system) {
            mbpcg_info& f = per_system[i];
            memset(&f, 0, sizeof(f));
            f.iterations = s.iter;
            f.best_column = s.h;
            f.final_width = s.width;
            f.deflations = s.deflations;
            f.used_fallback = (s.done == DONE_ZERO_RHS) ? 0 : (s.accepted ? 0 : 1);
            f.rel_res_best_basis = s.nu_h;
            f.rel_res_ls = s.done == DONE_CONVERGED ? s.rel_ls : NAN;
            f.rel_res_true = s.rel_true;
            f.ms_total = ms_all;
            f.ms_per_iter = hctl.loops > 0 ? ms_kernel / hctl.loops : 0.0;
            double acc = 0.0;
            for (int q = 0; q < 7; ++q) {
                f.ms_phase[q] = ph_ms[q];
                acc += ph_ms[q];
            }
            f.ms_phase[7] = p.profile ? std::max(0.0, ms_kernel - acc) : ms_kernel;
            f.status = st;
        }
    }
    return worst;
}

// Timed trials of the persistent kernel's free parameters: lane groups per
// row for each (width, row class) present -- tried flipped one class at a
// time, kept when faster -- and then the grid (all co-resident workgroups,
// three quarters, half).  Trials are solves capped at a few iterations.  The
// per-class choice is kept for the process; a batch whose classes are all
// known skips those trials.
mbpcg_status batch_tune(BatchCtx& c, const mbpcg_params& p, mbpcg_batch_tuning* out) {
    mbpcg_params q = p;
    q.max_iter = std::min<int64_t>(p.max_iter, 12);
    q.profile = 0;
    std::vector<std::pair<int, int>> classes;
    for (int i = 0; i < c.nsys; ++i) {
        const std::pair<int, int> k{c.hs[i].S, row_class(c.sys[i].n, c.sys[i].nnz)};
        if (std::find(classes.begin(), classes.end(), k) == classes.end()) classes.push_back(k);
    }
    std::sort(classes.begin(), classes.end());
    int trials = 0;
    auto trial = [&](double* ms) -> mbpcg_status {
        ++trials;
        double best = 1e30;
        for (int r = 0; r < 2; ++r) {   // the faster of two runs
            double t = 0.0;
            const mbpcg_status st = batch_solve(c, q, nullptr, c.stream, &t);
            if (st != MBPCG_OK && st != MBPCG_NOT_CONVERGED && st != MBPCG_ERR_NOT_SPD &&
                st != MBPCG_ERR_BREAKDOWN && st != MBPCG_ERR_NONFINITE)
                return st;
            best = std::min(best, t);
        }
        *ms = best;
        return MBPCG_OK;
    };
    bool all_known = true;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        for (const auto& k : classes) {
            auto it = g_slot_cache.find(k);
            if (it == g_slot_cache.end()) all_known = false;
        }
        for (const auto& k : classes) {
            auto it = g_slot_cache.find(k);
            const int SL = it != g_slot_cache.end() ? it->second : default_slots(k.second);
            for (int i = 0; i < c.nsys; ++i)
                if (c.hs[i].S == k.first && row_class(c.sys[i].n, c.sys[i].nnz) == k.second)
                    c.hs[i].SL = SL;
        }
    }
    BCK(hipMemcpyAsync(c.d_sys, c.hs.data(), sizeof(BSys) * c.nsys, hipMemcpyHostToDevice,
                       c.stream));
    BCK(hipStreamSynchronize(c.stream));
    double best = 0.0;
    mbpcg_status st = trial(&best);
    if (st != MBPCG_OK) return st;
    if (!all_known) {
        for (const auto& k : classes) {
            int cur = 1;
            for (int i = 0; i < c.nsys; ++i)
                if (c.hs[i].S == k.first && row_class(c.sys[i].n, c.sys[i].nnz) == k.second)
                    cur = c.hs[i].SL;
            const int alt = cur == 1 ? 2 : 1;
            if ((st = set_slots(c, k.first, k.second, alt)) != MBPCG_OK) return st;
            double t = 0.0;
            if ((st = trial(&t)) != MBPCG_OK) return st;
            if (t < 0.99 * best) {
                best = t;
            } else if ((st = set_slots(c, k.first, k.second, cur)) != MBPCG_OK) {
                return st;
            }
        }
        std::lock_guard<std::mutex> lk(g_tune_mu);
        for (const auto& k : classes)
            for (int i = 0; i < c.nsys; ++i)
                if (c.hs[i].S == k.first && row_class(c.sys[i].n, c.sys[i].nnz) == k.second) {
                    g_slot_cache[k] = c.hs[i].SL;
                    break;
                }
    }
    const int full = std::max(1, std::min(std::max(c.items, c.pitems), c.resident));
    int best_grid = c.grid;
    for (int g : {full, full * 3 / 4 / 8 * 8, full / 2 / 8 * 8}) {
        if (g < 8 || g == c.grid) continue;
        const int keep = c.grid;
        c.grid = g;
        double t = 0.0;
        if ((st = trial(&t)) != MBPCG_OK) {
            c.grid = keep;   // the context stays on a grid that was tuned
            return st;
        }
        if (t < 0.99 * best) {
            best = t;
            best_grid = g;
        }
        c.grid = keep;
    }
    c.grid = best_grid;
    if (out) {
        *out = mbpcg_batch_tuning{};
        out->workgroups = c.grid;
        out->classes = (int32_t)classes.size();
        for (const auto& k : classes)
            for (int i = 0; i < c.nsys; ++i)
                if (c.hs[i].S == k.first && row_class(c.sys[i].n, c.sys[i].nnz) == k.second) {
                    out->two_slot_classes += c.hs[i].SL == 2;
                    break;
                }
        out->trials = trials;
        out->ms = best;
    }
    return MBPCG_OK;
}

#undef BCK

// one call: upload, solve, free
mbpcg_status batch_entry(int32_t nsys, const mbpcg_system* systems, const mbpcg_params& p,
                         mbpcg_info* per_system, mbpcg_mem mem, hipStream_t user_stream,
                         std::string& err) {
    BatchCtx c;
    mbpcg_status st = batch_create(c, nsys, systems, mem, user_stream);
    if (st == MBPCG_OK) st = batch_solve(c, p, per_system, user_stream, nullptr);
    if (!c.err.empty()) err = c.err;
    return st;
}

}  // namespace mb

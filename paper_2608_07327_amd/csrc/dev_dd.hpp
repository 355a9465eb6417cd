// Double-double (unevaluated sum hi + lo of two FP64 numbers, about 106
// significant bits) arithmetic for the least-squares termination.  The
// error-free transformations are Knuth's two-sum, Dekker's fast two-sum and
// the FMA form of the exact product; addition, multiplication, division and
// square root follow the usual double-double algorithms (Dekker 1971;
// Bailey's QD library description, Hida, Li & Bailey 2001).  FMA contraction
// is switched off inside every function: the transformations are exact only
// when each operation is rounded as written.
#pragma once
#include "dev_common.hpp"

namespace mb {

struct dd {
    double hi, lo;
};

__device__ __forceinline__ dd dd_from(double a) { return dd{a, 0.0}; }

__device__ __forceinline__ dd two_sum(double a, double b) {
#pragma clang fp contract(off)
    const double s = a + b;
    const double bb = s - a;
    return dd{s, (a - (s - bb)) + (b - bb)};
}

// |a| >= |b| (or a == 0)
__device__ __forceinline__ dd fast_two_sum(double a, double b) {
#pragma clang fp contract(off)
    const double s = a + b;
    return dd{s, b - (s - a)};
}

__device__ __forceinline__ dd two_prod(double a, double b) {
#pragma clang fp contract(off)
    const double p = a * b;
    return dd{p, __fma_rn(a, b, -p)};
}

__device__ __forceinline__ dd dd_add(dd a, dd b) {
#pragma clang fp contract(off)
    dd s = two_sum(a.hi, b.hi);
    const dd t = two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = fast_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return fast_two_sum(s.hi, s.lo);
}

__device__ __forceinline__ dd dd_neg(dd a) { return dd{-a.hi, -a.lo}; }
__device__ __forceinline__ dd dd_sub(dd a, dd b) { return dd_add(a, dd_neg(b)); }

// symmetric in its arguments: the cross terms are rounded and added in an
// order that does not depend on which operand is first
__device__ __forceinline__ dd dd_mul(dd a, dd b) {
#pragma clang fp contract(off)
    dd p = two_prod(a.hi, b.hi);
    const double x = a.hi * b.lo, y = a.lo * b.hi;
    p.lo += x + y;
    return fast_two_sum(p.hi, p.lo);
}

// a + x * y with x, y plain doubles (accumulation of exact products)
__device__ __forceinline__ dd dd_add_prod(dd a, double x, double y) {
    return dd_add(a, two_prod(x, y));
}

__device__ __forceinline__ dd dd_div(dd a, dd b) {
#pragma clang fp contract(off)
    const double q1 = a.hi / b.hi;
    dd r = dd_sub(a, dd_mul(dd_from(q1), b));
    const double q2 = r.hi / b.hi;
    r = dd_sub(r, dd_mul(dd_from(q2), b));
    const double q3 = r.hi / b.hi;
    const dd q = fast_two_sum(q1, q2);
    return dd_add(q, dd_from(q3));
}

// a >= 0; one Newton step on the FP64 square root
__device__ __forceinline__ dd dd_sqrt(dd a) {
#pragma clang fp contract(off)
    if (!(a.hi > 0.0)) return dd{0.0, 0.0};
    const double q = sqrt(a.hi);
    const dd r = dd_sub(a, two_prod(q, q));
    return fast_two_sum(q, r.hi / (2.0 * q));
}

__device__ __forceinline__ double dd_to_double(dd a) { return a.hi + a.lo; }

__device__ __forceinline__ bool dd_finite(dd a) { return finite_d(a.hi) && finite_d(a.lo); }

// lane broadcast of a double-double from a compile-time lane
__device__ __forceinline__ double lane_bcast_d(double v, int lane) {
    const long long x = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(x & 0xffffffffll), lane);
    const int hi = __builtin_amdgcn_readlane((int)(x >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ dd lane_bcast_dd(dd v, int lane) {
    return dd{lane_bcast_d(v.hi, lane), lane_bcast_d(v.lo, lane)};
}

// ---------------------------------------------------------------------------
// Per-workgroup double-double sums of ETOT entries over the rows of a tile
// (the layout of TileSums): entry e of thread t, TPE threads per entry when
// there are fewer entries than threads.  finish() writes hi at out[2 e] and
// lo at out[2 e + 1], after a pairwise tree over the TPE threads of an
// entry (fixed order).
// ---------------------------------------------------------------------------
template <int ETOT>
struct TileSumsDD {
    static constexpr int TPE = ETOT >= MB_BLOCK ? 1 : floor_pow2(MB_BLOCK / ETOT);
    static constexpr int EPT = TPE == 1 ? (ETOT + MB_BLOCK - 1) / MB_BLOCK : 1;
    dd acc[EPT];
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
                const int e = t + k * MB_BLOCK;
                ent[k] = e < ETOT ? e : -1;
            }
        }
#pragma unroll
        for (int k = 0; k < EPT; ++k) acc[k] = dd{0.0, 0.0};
    }

    // f(k, r) -> (x, y): the product x * y is added exactly
    template <class F>
    __device__ __forceinline__ void add_rows(int rows, F f) {
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
            if (ent[k] < 0) continue;
            dd a = acc[k];
            for (int r = sub; r < rows; r += TPE) {
                const double2 xy = f(k, r);
                a = dd_add_prod(a, xy.x, xy.y);
            }
            acc[k] = a;
        }
    }

    // lds: 2 * MB_BLOCK doubles.  Ends with a barrier.
    __device__ __forceinline__ void finish(double* lds, double* out) {
        if (TPE > 1) {
            __syncthreads();
            lds[2 * threadIdx.x] = acc[0].hi;
            lds[2 * threadIdx.x + 1] = acc[0].lo;
            __syncthreads();
            const int q = threadIdx.x % TPE;
#pragma unroll
            for (int h = TPE / 2; h >= 1; h /= 2) {
                if (q < h) {
                    const int o = threadIdx.x + h;
                    const dd v = dd_add(dd{lds[2 * threadIdx.x], lds[2 * threadIdx.x + 1]},
                                        dd{lds[2 * o], lds[2 * o + 1]});
                    lds[2 * threadIdx.x] = v.hi;
                    lds[2 * threadIdx.x + 1] = v.lo;
                }
                __syncthreads();
            }
            const int e = threadIdx.x;
            if (e < ETOT) {
                out[2 * e] = lds[2 * e * TPE];
                out[2 * e + 1] = lds[2 * e * TPE + 1];
            }
            __syncthreads();
        } else {
#pragma unroll
            for (int k = 0; k < EPT; ++k)
                if (ent[k] >= 0) {
                    out[2 * ent[k]] = acc[k].hi;
                    out[2 * ent[k] + 1] = acc[k].lo;
                }
        }
    }
};

// Fixed-order double-double sum of nwg partials (entry e of partial w at
// part[w * stride + 2 e], lo at + 1) into out_hi/out_lo[0..E).  Threads take
// an entry and a contiguous chunk of partials each, then a pairwise tree over
// the chunks.  tmp must hold 2 * blockDim doubles.  Ends with a barrier.
__device__ __forceinline__ void reduce_partials_dd(const double* __restrict__ part, int nwg, int E,
                                                   int stride, double* out_hi, double* out_lo,
                                                   double* tmp) {
    const int B = blockDim.x, t = threadIdx.x;
    int tpe = 1;
    while (tpe * 2 * E <= B) tpe *= 2;
    if (E > B) {
        for (int e = t; e < E; e += B) {
            dd a{0.0, 0.0};
            for (int w = 0; w < nwg; ++w)
                a = dd_add(a, dd{part[(int64_t)w * stride + 2 * e], part[(int64_t)w * stride + 2 * e + 1]});
            out_hi[e] = a.hi;
            out_lo[e] = a.lo;
        }
        __syncthreads();
        return;
    }
    const int e = t % E, q = t / E;
    if (q < tpe) {
        const int chunk = (nwg + tpe - 1) / tpe;
        const int w0 = min(nwg, q * chunk), w1 = min(nwg, w0 + chunk);
        dd a{0.0, 0.0};
        for (int w = w0; w < w1; ++w)
            a = dd_add(a, dd{part[(int64_t)w * stride + 2 * e], part[(int64_t)w * stride + 2 * e + 1]});
        tmp[2 * (q * E + e)] = a.hi;
        tmp[2 * (q * E + e) + 1] = a.lo;
    }
    __syncthreads();
    for (int h = tpe / 2; h >= 1; h /= 2) {
        if (q < h) {
            const int i0 = 2 * (q * E + e), i1 = 2 * ((q + h) * E + e);
            const dd v = dd_add(dd{tmp[i0], tmp[i0 + 1]}, dd{tmp[i1], tmp[i1 + 1]});
            tmp[i0] = v.hi;
            tmp[i0 + 1] = v.lo;
        }
        __syncthreads();
    }
    if (t < E) {
        out_hi[t] = tmp[2 * t];
        out_lo[t] = tmp[2 * t + 1];
    }
    __syncthreads();
}

// One entry of B^ = B - D R (the least-squares matrix of the termination),
// b_r - (d_r R_rj) with both operations rounded: the product is not fused
// into the subtraction.
__device__ __forceinline__ double bhat_entry(double b, double d, double r) {
#pragma clang fp contract(off)
    const double ro = d * r;
    return b - ro;
}

}  // namespace mb

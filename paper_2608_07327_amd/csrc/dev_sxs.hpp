// s x s FP64 work of an MBPCG iteration, as device functions run by one
// workgroup (all threads call them; they contain barriers).  Each takes the
// partial sums of its reduction (nwg slots, `stride` doubles apart) and LDS
// workspace from the caller, so the single-system tail kernels and the
// batched persistent kernel share them.  The factorisations are sequential
// stages separated by barriers; thread i owns row (or column) i.
#pragma once
#include "dev_common.hpp"
#include "dev_dd.hpp"

namespace mb {

// ---------------------------------------------------------------------------
// The factorisations run on wavefront 0 with lane i holding row i of the
// working matrix in registers (S <= 32 < 64 lanes); a pivot or a finished
// column entry reaches the other lanes by readlane with a compile-time lane
// index, so there is no barrier inside the elimination.  Results go to LDS
// and the callers' remaining S^3 products use every thread.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double lane_bcast(double v, int lane) {
    const long long x = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(x & 0xffffffffll), lane);
    const int hi = __builtin_amdgcn_readlane((int)(x >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// lower Cholesky C = L L^T (S x S, reads the lower triangle) into L (upper
// part zero).  Returns nonzero when a pivot is not positive and finite.
template <int S>
__device__ int chol_lower(const double* C, double* L, int* flag) {
    const int t = threadIdx.x;
    if (t < 64) {
        const int i = t < S ? t : S - 1;
        double w[S];
#pragma unroll
        for (int k = 0; k < S; ++k) w[k] = C[(i >= k ? i : k) * S + (i >= k ? k : i)];
        int bad = 0;
#pragma unroll
        for (int j = 0; j < S; ++j) {
            double d = lane_bcast(w[j], j);
            if (!(d > 0.0) || !finite_d(d)) {
                bad = 1;
                d = 1.0;
            }
            const double ljj = sqrt(d);
            const double lij = t == j ? ljj : (t > j ? w[j] / ljj : 0.0);
            w[j] = lij;
#pragma unroll
            for (int k = j + 1; k < S; ++k) w[k] -= lij * lane_bcast(lij, k);
        }
        if (t < S) {
#pragma unroll
            for (int k = 0; k < S; ++k) L[t * S + k] = k <= t ? w[k] : 0.0;
        }
        if (t == 0) *flag = bad;
    }
    __syncthreads();
    const int f = *flag;
    __syncthreads();
    return f;
}

// L^-1 of a lower-triangular L in LDS, one column per lane (forward
// substitution on e_c; reads of L are wavefront broadcasts).
template <int S>
__device__ void lower_inverse(const double* L, double* Li) {
    const int c = threadIdx.x;
    if (c < S) {
        double x[S];
#pragma unroll
        for (int i = 0; i < S; ++i) {
            double v = i == c ? 1.0 : 0.0;
#pragma unroll
            for (int m = 0; m < i; ++m) v -= L[i * S + m] * x[m];
            x[i] = v / L[i * S + i];
        }
#pragma unroll
        for (int i = 0; i < S; ++i) Li[i * S + c] = x[i];
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Cholesky QR factor with column dropping (Sec. 3 uses single-pass Cholesky
// QR; the paper only needs independent columns).  G = U^T U column by column;
// column l is kept iff G_ll > 0, finite, and delta_l > tau G_ll with
// delta_l = G_ll - sum_{kept q < l} U_ql^2 (the pivot of the Schur complement
// left by the kept columns).  Writes U (upper, dropped rows zero), keep[S],
// Z = U (upper trapezoidal) and M = inverse of the kept block (dropped rows
// and columns zero).  Returns the number of kept columns.
// ---------------------------------------------------------------------------
template <int S>
__device__ int cholqr_factor(const double* G, double tau, double* U, int* keep, double* Z,
                             double* M, int* cnt) {
    const int t = threadIdx.x;
    if (t < 64) {
        const int i = t < S ? t : S - 1;
        double w[S];
#pragma unroll
        for (int k = 0; k < S; ++k) w[k] = G[i * S + k];
        const double gdiag = G[i * S + i];
        int kept = 0;
#pragma unroll
        for (int l = 0; l < S; ++l) {
            const double g = lane_bcast(gdiag, l);
            const double dl = lane_bcast(w[l], l);
            const bool k = (g > 0.0) && finite_d(dl) && (dl > tau * g);   // wave-uniform
            double u = 0.0;
            if (k) {
                const double ul = sqrt(dl);
                u = t == l ? ul : (t > l ? w[l] / ul : 0.0);
#pragma unroll
                for (int a = l + 1; a < S; ++a) w[a] -= u * lane_bcast(u, a);
                ++kept;
            }
            if (t < S) U[l * S + t] = u;
            if (t == 0) keep[l] = k ? 1 : 0;
        }
        if (t == 0) *cnt = kept;
    }
    __syncthreads();
    // M = (kept block of U)^-1, one column per lane by back substitution
    if (t < S) {
        const int c = t;
        double x[S];
#pragma unroll
        for (int a = S - 1; a >= 0; --a) {
            double v = a == c ? 1.0 : 0.0;
#pragma unroll
            for (int b2 = a + 1; b2 < S; ++b2) v -= U[a * S + b2] * x[b2];
            x[a] = (keep[a] && keep[c] && a <= c) ? v / U[a * S + a] : 0.0;
        }
#pragma unroll
        for (int a = 0; a < S; ++a) M[a * S + c] = x[a];
    }
    for (int e = t; e < S * S; e += blockDim.x) {
        const int r = e / S, j = e % S;
        Z[e] = (keep[r] && j >= r) ? U[e] : 0.0;
    }
    __syncthreads();
    return *cnt;
}

// reduction workspace: max(E, threads of any caller)
template <int E>
struct RedWs {
    static constexpr int N = E > TAIL_THREADS ? E : TAIL_THREADS;
};

// doubles / ints of LDS workspace each body needs
template <int S>
struct SxsWs {
    static constexpr int XI = 2 * RedWs<tri_count(S)>::N + 4 * S * S;
    static constexpr int QR = 2 * RedWs<tri_count(S) + S>::N + 5 * S * S;
    static constexpr int LS = 2 * tri_count(S + 1) + 2 * TAIL_THREADS + 2 * (S + 1) * (S + 1) +
                              2 * (S + 1);
    static constexpr int DOUBLES = XI > QR ? (XI > LS ? XI : LS) : (QR > LS ? QR : LS);
    static constexpr int INTS = S + 8;   // >= S + 2 for the least squares
};

// ---------------------------------------------------------------------------
// step matrix: C = P^T A P from partials; inactive columns get an identity
// row/column; Xi = C^-1 through C = L L^T; alpha = Xi Sigma.
// ---------------------------------------------------------------------------
template <int S>
__device__ void tail_xi_body(const double* __restrict__ part, int nwg, int stride,
                             DevState* __restrict__ st, double* sm, int* smi) {
    constexpr int E = tri_count(S);
    constexpr int RN = RedWs<E>::N;
    double* tri = sm;
    double* tmp = sm + RN;
    double* C = sm + 2 * RN;
    double* L = C + S * S;
    double* Li = L + S * S;
    double* Xi = Li + S * S;
    const int t = threadIdx.x;
    reduce_partials(part, nwg, E, stride, tri, tmp);
    for (int e = t; e < S * S; e += blockDim.x) {
        const int i = e / S, j = e % S;
        const int a = i >= j ? i : j, b = i >= j ? j : i;
        double v = tri[a * (a + 1) / 2 + b];
        if (!st->active[i] || !st->active[j]) v = (i == j) ? 1.0 : 0.0;
        C[e] = v;
    }
    __syncthreads();
    if (S >= 16 && (int)blockDim.x >= S * S) {   // uniform across the workgroup
        // Wide blocks: Gauss-Jordan elimination without pivoting, one thread
        // per entry, in place.  On an SPD matrix its pivots are those of the
        // Cholesky factorisation (squared diagonal of L), so a pivot that is
        // not positive and finite means C is not SPD, as there.  S steps of
        // two barriers replace the sequential Cholesky, triangular inverse
        // and L^-T L^-1 of the narrow path; the result is symmetrised.
        const int i = t / S, j = t % S;
        const bool mine = t < S * S;
        bool bad = false;
        for (int k = 0; k < S; ++k) {
            double p = C[k * S + k];
            const double aik = mine ? C[i * S + k] : 0.0;
            const double akj = mine ? C[k * S + j] : 0.0;
            __syncthreads();
            if (!(p > 0.0) || !finite_d(p)) {
                bad = true;
                p = 1.0;
            }
            const double rp = 1.0 / p;
            if (mine) {
                double v;
                if (i == k && j == k) v = rp;
                else if (i == k) v = akj * rp;
                else if (j == k) v = -aik * rp;
                else v = C[t] - aik * (akj * rp);
                C[t] = v;
            }
            __syncthreads();
        }
        if (bad) {
            if (t == 0) st->done = DONE_NOTSPD;
            return;
        }
        if (mine) {
            Xi[t] = 0.5 * (C[i * S + j] + C[j * S + i]);
            L[t] = st->Sigma[i * MB_SM + j];   // Sigma staged in LDS
        }
        __syncthreads();
        if (mine) {
            double v = 0.0;
#pragma unroll 8
            for (int l = 0; l < S; ++l) v += Xi[i * S + l] * L[l * S + j];
            st->alpha[i * MB_SM + j] = v;
            st->Xi[i * MB_SM + j] = Xi[t];
        }
        (void)Li;
        return;
    } else {
        if (chol_lower<S>(C, L, smi)) {
            if (t == 0) st->done = DONE_NOTSPD;
            return;
        }
        // L^-1, one column per lane
        lower_inverse<S>(L, Li);
        // Xi = L^-T L^-1
        for (int e = t; e < S * S; e += blockDim.x) {
            const int i = e / S, j = e % S;
            const int k0 = i > j ? i : j;
            double v = 0.0;
            for (int k = k0; k < S; ++k) v += Li[k * S + i] * Li[k * S + j];
            Xi[e] = v;
        }
        __syncthreads();
        for (int e = t; e < S * S; e += blockDim.x) {
            const int i = e / S, j = e % S;
            double v = 0.0;
            for (int l = 0; l < S; ++l) v += Xi[i * S + l] * st->Sigma[l * MB_SM + j];
            st->alpha[i * MB_SM + j] = v;
            st->Xi[i * MB_SM + j] = Xi[e];
        }
    }
}

// ---------------------------------------------------------------------------
// best column h, stop test, second half of the Cholesky QR, Sigma update; or,
// with setup, the first Cholesky QR (W0, Sigma0).  Partials hold the lower triangle of V^T V and then
// nu_j = sum_r (d_r R_rj)^2.  Returns 1 when this call finished the system
// (converged, stalled or failed), else 0.
// ---------------------------------------------------------------------------
template <int S>
__device__ int tail_qr_body(const double* __restrict__ part, int nwg, int stride,
                            DevState* __restrict__ st, double* __restrict__ hist, int setup,
                            double* sm, int* smi) {
    // setup 2: resume after a least squares that did not finish the solve --
    // the best column and the stop test of this iteration are done, only the
    // Cholesky QR is left (the direction kernel then leaves X~ alone)
    const int resume = setup == 2;
    if (resume) setup = 0;
    constexpr int E = tri_count(S);
    constexpr int ET = E + S;
    constexpr int RN = RedWs<ET>::N;
    double* red = sm;
    double* tmp = sm + RN;
    double* G = sm + 2 * RN;
    double* U = G + S * S;
    double* Z = U + S * S;
    double* M = Z + S * S;
    double* Sg = M + S * S;
    int* keep = smi;
    int* cnt = smi + S;
    int* stop = smi + S + 1;
    const int t = threadIdx.x;
    reduce_partials(part, nwg, ET, stride, red, tmp);
    if (!resume && t < st->s) st->nu[t] = sqrt(red[E + t]) / st->bnorm;
    if (t == 0 && resume) {
        st->xt_skip = 1;
        *stop = 0;
    } else if (t == 0) {
        // best column in the original residual norm (Sec. 1: R = D R~)
        const int s = st->s;
        int h = 0;
        double best = red[E];
        for (int j = 1; j < s; ++j) {
            if (red[E + j] < best) {
                best = red[E + j];
                h = j;
            }
        }
        const double nu_h = sqrt(best) / st->bnorm;
        st->h = h;
        st->nu_h = nu_h;
        int stp = 0;
        if (!setup) {
            const int it = st->iter + 1;
            st->iter = it;
            if (hist && it <= st->n_hist) hist[it - 1] = nu_h;
            if (!finite_d(nu_h)) {
                st->done = DONE_NONFINITE;
                stp = 1;
            } else if (nu_h < st->tol0) {
                st->done = st->ls_inloop ? DONE_LS : DONE_CONVERGED;
                stp = 1;
            }
        }
        *stop = stp;
    }
    __syncthreads();
    if (*stop) return 1;
    for (int e = t; e < S * S; e += blockDim.x) {
        const int i = e / S, j = e % S;
        const int a = i >= j ? i : j, b = i >= j ? j : i;
        G[e] = red[a * (a + 1) / 2 + b];
    }
    __syncthreads();
    const int k = cholqr_factor<S>(G, st->tau, U, keep, Z, M, cnt);
    // Sigma staged in LDS (G is free once the factor is done)
    if (!setup)
        for (int e = t; e < S * S; e += blockDim.x) G[e] = st->Sigma[(e / S) * MB_SM + e % S];
    __syncthreads();
    for (int e = t; e < S * S; e += blockDim.x) {
        const int i = e / S, j = e % S;
        double v;
        if (setup) {
            v = Z[e];
        } else {
            v = 0.0;
            for (int l = 0; l < S; ++l) v += Z[i * S + l] * G[l * S + j];
        }
        Sg[e] = v;
    }
    __syncthreads();
    for (int e = t; e < S * S; e += blockDim.x) {
        const int i = e / S, j = e % S;
        st->Sigma[i * MB_SM + j] = Sg[e];
        st->Z[i * MB_SM + j] = Z[e];
        st->M[i * MB_SM + j] = M[e];
    }
    if (t < S) st->active[t] = keep[t];
    int fin = 0;
    if (k == 0) fin = 1;
    else if (!setup && st->iter >= st->max_iter) fin = 1;
    if (t == 0) {
        if (setup) st->ready = 1;
        const int before = setup ? st->s : st->width;
        st->deflations += before - k;
        st->width = k;
        if (k == 0) st->done = setup ? DONE_CONVERGED : DONE_BREAKDOWN;
        else if (!setup && st->iter >= st->max_iter) st->done = DONE_MAXITER;
    }
    return fin;
}

// ---------------------------------------------------------------------------
// Least squares of the termination (Alg. 1, the combination c^ of the
// columns of B^ = B - D R, which equals A X by Proposition 1):
// c^ = argmin ||b - B^ c||.  The partials hold the double-double Gram of
// [B^_0 .. B^_{S-1}, b] (columns j >= s zero).  It is factored G = U^T U
// column by column in double-double, leaving out column j when its part
// independent of the columns kept before it is not above 1e-12 of its norm
// (pivot delta_j <= 1e-24 G_jj), when its norm is zero, or when n columns are
// kept already; a left-out column gets coefficient 0.  This is the basic
// solution that Householder QR of B^ with the same rule gives: in exact
// arithmetic the pivots are the squared norms of the independent parts.
// The Gram in double-double (about 106 bits) keeps the independent parts,
// which are about |R| / |b| of a column's norm, well resolved although the
// Gram squares the condition number of B^.  The last column's entries of U
// are z = U_JJ^-T B^_J^T b, and U_JJ c_J = z.
// ---------------------------------------------------------------------------
template <int S>
__device__ void tail_ls_body(const double* __restrict__ part, int nwg, int stride, int64_t n,
                             DevState* __restrict__ st, double* sm, int* smi) {
    constexpr int NC = S + 1;
    constexpr int E = tri_count(NC);
    double* ghi = sm;
    double* glo = sm + E;
    double* tmp = sm + 2 * E;                       // 2 * blockDim doubles
    double* uhi = sm + 2 * E + 2 * TAIL_THREADS;    // U, row l at [l * NC]
    double* ulo = uhi + NC * NC;
    double* chi = ulo + NC * NC;                    // c^ (double-double)
    double* clo = chi + NC;
    int* keep = smi;                                // [S]
    int* flags = smi + S;                           // [0] kept, [1] ok
    const int t = threadIdx.x;
    reduce_partials_dd(part, nwg, E, stride, ghi, glo, tmp);
    const int s = st->s;
    if (t < 64) {
        const int i = t < NC ? t : NC - 1;   // lanes past the last row mirror it (discarded)
        dd w[NC];
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            const int a = i >= k ? i : k, b = i >= k ? k : i;
            w[k] = dd{ghi[a * (a + 1) / 2 + b], glo[a * (a + 1) / 2 + b]};
        }
        int kept = 0;
        bool ok = true;
#pragma unroll
        for (int l = 0; l < S; ++l) {
            const double g = ghi[l * (l + 1) / 2 + l];   // squared norm of column l
            const dd dl = lane_bcast_dd(w[l], l);        // pivot left by the kept columns
            if (l < s && !finite_d(g)) ok = false;
            const bool k = l < s && g > 0.0 && finite_d(g) && dd_finite(dl) &&
                           dl.hi > 1e-24 * g && kept < n;   // wave-uniform
            if (k) {
                const dd ull = dd_sqrt(dl);
                dd ci{0.0, 0.0};
                if (i == l) ci = ull;
                else if (i > l) ci = dd_div(w[l], ull);
                if (t < NC) {
                    uhi[l * NC + i] = ci.hi;
                    ulo[l * NC + i] = ci.lo;
                }
#pragma unroll
                for (int q = l + 1; q < NC; ++q) w[q] = dd_sub(w[q], dd_mul(ci, lane_bcast_dd(ci, q)));
                ++kept;
            }
            if (t == 0) keep[l] = k ? 1 : 0;
        }
        if (t == 0) {
            flags[0] = kept;
            flags[1] = ok ? 1 : 0;
        }
    }
    __syncthreads();
    // back substitution U_JJ c_J = z over the kept columns: lane l holds the
    // running right-hand side of row l, c_q reaches the other lanes by readlane
    if (t < 64) {
        const int l = t < S ? t : S - 1;
        const bool mine = t < S && keep[l];
        dd acc = mine ? dd{uhi[l * NC + S], ulo[l * NC + S]} : dd{0.0, 0.0};
        dd cl{0.0, 0.0};
#pragma unroll
        for (int q = S - 1; q >= 0; --q) {
            if (!keep[q]) continue;   // wave-uniform
            dd cq{0.0, 0.0};
            if (t == q) cq = dd_div(acc, dd{uhi[q * NC + q], ulo[q * NC + q]});
            cq = lane_bcast_dd(cq, q);
            if (t == q) cl = cq;
            if (mine && l < q) acc = dd_sub(acc, dd_mul(dd{uhi[l * NC + q], ulo[l * NC + q]}, cq));
        }
        if (t < S) {
            chi[t] = cl.hi;
            clo[t] = cl.lo;
        }
    }
    __syncthreads();
    if (t == 0) {
        bool ok = flags[1] && flags[0] > 0;
        for (int j = 0; j < S; ++j) {
            const double cj = keep[j] ? dd_to_double(dd{chi[j], clo[j]}) : 0.0;
            if (!finite_d(cj)) ok = false;
            st->chat[j] = cj;
        }
        st->y0 = 0.0;
        st->ls_ok = ok ? 1 : 0;
        st->ls_width = flags[0];
    }
    __syncthreads();
}

}  // namespace mb

// s x s FP64 work of an MBPCG iteration, as device functions run by one
// workgroup (all threads call them; they contain barriers).  Each takes the
// partial sums of its reduction (nwg slots, `stride` doubles apart) and LDS
// workspace from the caller, so the single-system tail kernels and the
// batched persistent kernel share them.  The factorisations are sequential
// stages separated by barriers; thread i owns row (or column) i.
#pragma once
#include "dev_common.hpp"

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
    static constexpr int LS = 2 * RedWs<tri_count(S + 1)>::N + 2 * (S + 1) * (S + 1) + 2 * (S + 1);
    static constexpr int DOUBLES = XI > QR ? (XI > LS ? XI : LS) : (QR > LS ? QR : LS);
    static constexpr int INTS = S + 8;
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
    if (t < st->s) st->nu[t] = sqrt(red[E + t]) / st->bnorm;
    if (t == 0) {
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
                st->done = DONE_CONVERGED;
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
// Least squares of the termination (the combination c^).  Columns m_0 = b,
// m_{j+1} = D R_j; K = M^T M (lower triangle from partials).  Minimise
// ||M y|| subject to sum y = 1: with Delta = diag(||m_i||), K~ = Delta^-1 K
// Delta^-1 and w = Delta^-1 1, y = Delta^-1 z / (w^T z) where K~ z = w,
// solved by Cholesky over the independent columns (same dropping rule as
// the Cholesky QR).  c_j = y_{j+1}.  Since b - B^ c = (1 - sum c) b + D R c,
// this is the minimiser of ||b - B^ c||.
// ---------------------------------------------------------------------------
template <int S>
__device__ void tail_ls_body(const double* __restrict__ part, int nwg, int stride,
                             DevState* __restrict__ st, double* sm, int* smi) {
    constexpr int NC = S + 1;
    constexpr int E = tri_count(NC);
    constexpr int RN = RedWs<E>::N;
    double* red = sm;
    double* tmp = sm + RN;
    double* K = sm + 2 * RN;
    double* Lk = K + NC * NC;
    double* dn = Lk + NC * NC;
    double* z = dn + NC;
    int* keep = smi;
    const int t = threadIdx.x;
    reduce_partials(part, nwg, E, stride, red, tmp);
    if (t < NC) dn[t] = sqrt(red[t * (t + 1) / 2 + t]);
    __syncthreads();
    for (int e = t; e < NC * NC; e += blockDim.x) {
        const int i = e / NC, j = e % NC;
        const int a = i >= j ? i : j, b = i >= j ? j : i;
        const double den = dn[i] * dn[j];
        K[e] = den > 0.0 ? red[a * (a + 1) / 2 + b] / den : 0.0;
        Lk[e] = 0.0;
    }
    __syncthreads();
    for (int l = 0; l < NC; ++l) {
        if (t == 0) {
            const double g = K[l * NC + l];
            double dl = g;
            for (int q = 0; q < l; ++q)
                if (keep[q]) dl -= Lk[l * NC + q] * Lk[l * NC + q];
            const int k = (dn[l] > 0.0) && (g > 0.0) && finite_d(dl) && (dl > st->tau * g);
            keep[l] = k;
            Lk[l * NC + l] = k ? sqrt(dl) : 1.0;
        }
        __syncthreads();
        if (keep[l] && t > l && t < NC) {
            double v = K[t * NC + l];
            for (int q = 0; q < l; ++q)
                if (keep[q]) v -= Lk[t * NC + q] * Lk[l * NC + q];
            Lk[t * NC + l] = v / Lk[l * NC + l];
        }
        __syncthreads();
    }
    if (t == 0) {
        // forward L y = w, backward L^T z = y (kept columns only); y in z's slot first
        int kept = 0;
        for (int i = 0; i < NC; ++i) {
            z[i] = 0.0;
            if (!keep[i]) continue;
            ++kept;
            double v = 1.0 / dn[i];
            for (int q = 0; q < i; ++q)
                if (keep[q]) v -= Lk[i * NC + q] * z[q];
            z[i] = v / Lk[i * NC + i];
        }
        for (int i = NC - 1; i >= 0; --i) {
            if (!keep[i]) continue;
            double v = z[i];
            for (int q = i + 1; q < NC; ++q)
                if (keep[q]) v -= Lk[q * NC + i] * z[q];
            z[i] = v / Lk[i * NC + i];
        }
        double wz = 0.0;
        for (int i = 0; i < NC; ++i)
            if (keep[i]) wz += z[i] / dn[i];
        bool ok = wz > 0.0 && finite_d(wz);
        for (int i = 0; i < NC; ++i) {
            const double yi = keep[i] ? (z[i] / wz) / dn[i] : 0.0;
            if (!finite_d(yi)) ok = false;
            if (i == 0) st->y0 = yi;
            else st->chat[i - 1] = yi;
        }
        st->ls_ok = ok ? 1 : 0;
        st->ls_width = kept;
    }
    __syncthreads();
}

}  // namespace mb

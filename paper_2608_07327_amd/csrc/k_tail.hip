// One-workgroup tail kernels: add up the per-workgroup partial sums of a
// reduction in a fixed order, then do the s x s FP64 work of the iteration.
// The s x s factorisations run on one wavefront: step j is a barrier-separated
// stage and lane i owns row (or column) i.
#include "kernels.hpp"

namespace mb {

#define TAIL_THREADS 256

// ---------------------------------------------------------------------------
// lower Cholesky C = L L^T of an S x S matrix in LDS (reads the lower triangle
// as filled in by the caller).  Returns 0 on success.
// ---------------------------------------------------------------------------
template <int S>
__device__ int chol_lower(const double* C, double* L, int* flag) {
    const int t = threadIdx.x;
    for (int e = t; e < S * S; e += blockDim.x) L[e] = 0.0;
    if (t == 0) *flag = 0;
    __syncthreads();
    for (int j = 0; j < S; ++j) {
        if (t == 0) {
            double dd = C[j * S + j];
            for (int k = 0; k < j; ++k) dd -= L[j * S + k] * L[j * S + k];
            if (!(dd > 0.0) || !finite_d(dd)) {
                *flag = 1;
                dd = 1.0;
            }
            L[j * S + j] = sqrt(dd);
        }
        __syncthreads();
        if (t > j && t < S) {
            double v = C[t * S + j];
            for (int k = 0; k < j; ++k) v -= L[t * S + k] * L[j * S + k];
            L[t * S + j] = v / L[j * S + j];
        }
        __syncthreads();
    }
    return *flag;
}

// ---------------------------------------------------------------------------
// Cholesky QR factor with column dropping (Sec. 3 uses single-pass Cholesky
// QR; the paper only needs independent columns).  G = U^T U column by column;
// column l is kept iff G_ll > 0, finite, and delta_l > tau G_ll with
// delta_l = G_ll - sum_{kept q < l} U_ql^2.  Writes U (upper, S x S),
// keep[S], Z = kept rows of U (upper trapezoidal, dropped rows zero) and
// M = inverse of the kept block (dropped rows/columns zero).  Returns the
// number of kept columns.
// ---------------------------------------------------------------------------
template <int S>
__device__ int cholqr_factor(const double* G, double tau, double* U, int* keep, double* Z,
                             double* M, int* cnt) {
    const int t = threadIdx.x;
    for (int e = t; e < S * S; e += blockDim.x) {
        U[e] = 0.0;
        M[e] = 0.0;
    }
    __syncthreads();
    for (int l = 0; l < S; ++l) {
        if (t == 0) {
            const double g = G[l * S + l];
            double dl = g;
            for (int q = 0; q < l; ++q)
                if (keep[q]) dl -= U[q * S + l] * U[q * S + l];
            const int k = (g > 0.0) && finite_d(dl) && (dl > tau * g);
            keep[l] = k;
            if (k) U[l * S + l] = sqrt(dl);
        }
        __syncthreads();
        if (keep[l] && t > l && t < S) {
            double v = G[l * S + t];
            for (int q = 0; q < l; ++q)
                if (keep[q]) v -= U[q * S + l] * U[q * S + t];
            U[l * S + t] = v / U[l * S + l];
        }
        __syncthreads();
    }
    // Z and M
    for (int e = t; e < S * S; e += blockDim.x) {
        const int i = e / S, j = e % S;
        Z[e] = (keep[i] && j >= i) ? U[e] : 0.0;
    }
    if (t < S && keep[t]) {
        const int c = t;
        M[c * S + c] = 1.0 / U[c * S + c];
        for (int a = c - 1; a >= 0; --a) {
            if (!keep[a]) continue;
            double v = 0.0;
            for (int b = a + 1; b <= c; ++b)
                if (keep[b]) v -= U[a * S + b] * M[b * S + c];
            M[a * S + c] = v / U[a * S + a];
        }
    }
    if (t == 0) {
        int k = 0;
        for (int l = 0; l < S; ++l) k += keep[l];
        *cnt = k;
    }
    __syncthreads();
    return *cnt;
}

// ---------------------------------------------------------------------------
// T_A (line Xi): C = P^T A P from partials; inactive columns get an identity
// row/column; Xi = C^-1 through C = L L^T; alpha = Xi Sigma.
// ---------------------------------------------------------------------------
template <int S>
__global__ __launch_bounds__(TAIL_THREADS) void k_tail_xi(const double* __restrict__ part, int nwg,
                                                          DevState* __restrict__ st) {
    if (st->done) return;
    constexpr int E = tri_count(S);
    __shared__ double tri[E > TAIL_THREADS ? E : TAIL_THREADS];
    __shared__ double tmp[E > TAIL_THREADS ? E : TAIL_THREADS];
    __shared__ double C[S * S], L[S * S], Li[S * S], Xi[S * S];
    __shared__ int flag;
    const int t = threadIdx.x;
    reduce_partials(part, nwg, E, tri, tmp);
    for (int e = t; e < S * S; e += TAIL_THREADS) {
        const int i = e / S, j = e % S;
        const int a = i >= j ? i : j, b = i >= j ? j : i;
        double v = tri[a * (a + 1) / 2 + b];
        if (!st->active[i] || !st->active[j]) v = (i == j) ? 1.0 : 0.0;
        C[e] = v;
    }
    __syncthreads();
    const int bad = chol_lower<S>(C, L, &flag);
    if (bad) {
        if (t == 0) st->done = DONE_NOTSPD;
        return;
    }
    // L^-1 by forward substitution, one column per lane
    for (int e = t; e < S * S; e += TAIL_THREADS) Li[e] = 0.0;
    __syncthreads();
    if (t < S) {
        const int c = t;
        Li[c * S + c] = 1.0 / L[c * S + c];
        for (int i = c + 1; i < S; ++i) {
            double v = 0.0;
            for (int k = c; k < i; ++k) v -= L[i * S + k] * Li[k * S + c];
            Li[i * S + c] = v / L[i * S + i];
        }
    }
    __syncthreads();
    // Xi = L^-T L^-1
    for (int e = t; e < S * S; e += TAIL_THREADS) {
        const int i = e / S, j = e % S;
        const int k0 = i > j ? i : j;
        double v = 0.0;
        for (int k = k0; k < S; ++k) v += Li[k * S + i] * Li[k * S + j];
        Xi[e] = v;
    }
    __syncthreads();
    for (int e = t; e < S * S; e += TAIL_THREADS) {
        const int i = e / S, j = e % S;
        double v = 0.0;
        for (int l = 0; l < S; ++l) v += Xi[i * S + l] * st->Sigma[l * MB_SM + j];
        st->alpha[i * MB_SM + j] = v;
        st->Xi[i * MB_SM + j] = Xi[e];
    }
}

// ---------------------------------------------------------------------------
// T_B (lines h, initial_tolerance, W_zeta, Sigma) and the setup QR (line
// W^0_Sigma^0).  Partials hold the lower triangle of V^T V and nu_j.
// ---------------------------------------------------------------------------
template <int S>
__global__ __launch_bounds__(TAIL_THREADS) void k_tail_qr(const double* __restrict__ part, int nwg,
                                                          DevState* __restrict__ st,
                                                          double* __restrict__ hist, int setup) {
    if (st->done) return;
    constexpr int E = tri_count(S);
    constexpr int ET = E + S;
    __shared__ double red[ET > TAIL_THREADS ? ET : TAIL_THREADS];
    __shared__ double tmp[ET > TAIL_THREADS ? ET : TAIL_THREADS];
    __shared__ double G[S * S], U[S * S], Z[S * S], M[S * S];
    __shared__ int keep[S];
    __shared__ int cnt, stop;
    const int t = threadIdx.x;
    reduce_partials(part, nwg, ET, red, tmp);
    if (t == 0) {
        // best column in the original residual norm (Sec. 1: R = D R~)
        const int s = st->s;
        int h = 0;
        double best = red[E];
        for (int j = 0; j < s; ++j) {
            const double v = sqrt(red[E + j]) / st->bnorm;
            st->nu[j] = v;
            if (j > 0 && red[E + j] < best) {
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
        stop = stp;
    }
    __syncthreads();
    if (stop) return;
    for (int e = t; e < S * S; e += TAIL_THREADS) {
        const int i = e / S, j = e % S;
        const int a = i >= j ? i : j, b = i >= j ? j : i;
        G[e] = red[a * (a + 1) / 2 + b];
    }
    __syncthreads();
    const int k = cholqr_factor<S>(G, st->tau, U, keep, Z, M, &cnt);
    // Sigma <- Z Sigma (setup: Sigma = Z)
    __shared__ double Sg[S * S];
    for (int e = t; e < S * S; e += TAIL_THREADS) {
        const int i = e / S, j = e % S;
        double v;
        if (setup) {
            v = Z[e];
        } else {
            v = 0.0;
            for (int l = 0; l < S; ++l) v += Z[i * S + l] * st->Sigma[l * MB_SM + j];
        }
        Sg[e] = v;
    }
    __syncthreads();
    for (int e = t; e < S * S; e += TAIL_THREADS) {
        const int i = e / S, j = e % S;
        st->Sigma[i * MB_SM + j] = Sg[e];
        st->Z[i * MB_SM + j] = Z[e];
        st->M[i * MB_SM + j] = M[e];
    }
    if (t < S) st->active[t] = keep[t];
    if (t == 0) {
        const int before = setup ? st->s : st->width;
        st->deflations += before - k;
        st->width = k;
        if (k == 0) st->done = setup ? DONE_CONVERGED : DONE_BREAKDOWN;
        else if (!setup && st->iter >= st->max_iter) st->done = DONE_MAXITER;
    }
}

// ---------------------------------------------------------------------------
// Least squares of the termination (line hat_c).  Columns m_0 = b,
// m_{j+1} = D R_j; K = M^T M (lower triangle from partials).  Minimise
// ||M y|| subject to sum y = 1: with Delta = diag(||m_i||), K~ = Delta^-1 K
// Delta^-1 and w = Delta^-1 1, y = Delta^-1 z / (w^T z) where K~ z = w,
// solved by Cholesky over the independent columns (same dropping rule as
// the Cholesky QR).  c_j = y_{j+1}.
// ---------------------------------------------------------------------------
template <int S>
__global__ __launch_bounds__(TAIL_THREADS) void k_tail_ls(const double* __restrict__ part, int nwg,
                                                          DevState* __restrict__ st) {
    constexpr int NC = S + 1;
    constexpr int E = tri_count(NC);
    __shared__ double red[E > TAIL_THREADS ? E : TAIL_THREADS];
    __shared__ double tmp[E > TAIL_THREADS ? E : TAIL_THREADS];
    __shared__ double K[NC * NC], Lk[NC * NC], dn[NC], z[NC];
    __shared__ int keep[NC];
    const int t = threadIdx.x;
    reduce_partials(part, nwg, E, red, tmp);
    if (t < NC) dn[t] = sqrt(red[t * (t + 1) / 2 + t]);
    __syncthreads();
    for (int e = t; e < NC * NC; e += TAIL_THREADS) {
        const int i = e / NC, j = e % NC;
        const int a = i >= j ? i : j, b = i >= j ? j : i;
        const double den = dn[i] * dn[j];
        K[e] = den > 0.0 ? red[a * (a + 1) / 2 + b] / den : 0.0;
        Lk[e] = 0.0;
    }
    __syncthreads();
    // lower Cholesky with dropping on K~ (row l of L = column l of U)
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
        // forward: L y = w over kept; backward: L^T z = y over kept
        double y[NC];
        int kept = 0;
        for (int i = 0; i < NC; ++i) {
            y[i] = 0.0;
            if (!keep[i]) continue;
            ++kept;
            double v = 1.0 / dn[i];
            for (int q = 0; q < i; ++q)
                if (keep[q]) v -= Lk[i * NC + q] * y[q];
            y[i] = v / Lk[i * NC + i];
        }
        for (int i = NC - 1; i >= 0; --i) {
            z[i] = 0.0;
            if (!keep[i]) continue;
            double v = y[i];
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
}

// ||r|| of the LS combination and the accept test (line convergence_tolerance)
__global__ void k_tail_accept(const double* __restrict__ part, int nwg, DevState* __restrict__ st) {
    __shared__ double out[1], tmp[TAIL_THREADS];
    reduce_partials(part, nwg, 1, out, tmp);
    if (threadIdx.x == 0) {
        const double rel = sqrt(out[0]) / st->bnorm;
        st->rel_ls = rel;
        st->accepted = (st->done == DONE_CONVERGED) && st->ls_ok && finite_d(rel) && (rel < st->tol);
    }
}

__global__ void k_tail_true(const double* __restrict__ part, int nwg, DevState* __restrict__ st) {
    __shared__ double out[1], tmp[TAIL_THREADS];
    reduce_partials(part, nwg, 1, out, tmp);
    if (threadIdx.x == 0) st->rel_true = sqrt(out[0]) / st->bnorm;
}

// ||b||, ||b~||, ||A U||_F -> gamma (line X^0)
__global__ void k_tail_gamma(const double* __restrict__ part_b, int nwg_b,
                             const double* __restrict__ part_y, int nwg_y,
                             DevState* __restrict__ st) {
    __shared__ double ob[2], oy[1], tmp[TAIL_THREADS];
    reduce_partials(part_b, nwg_b, 2, ob, tmp);
    reduce_partials(part_y, nwg_y, 1, oy, tmp);
    if (threadIdx.x == 0) {
        const double bn = sqrt(ob[0]);
        st->bnorm = bn;
        st->bbar_norm = sqrt(ob[1]);
        if (!finite_d(bn)) {
            st->done = DONE_NONFINITE;
        } else if (bn == 0.0) {
            st->done = DONE_ZERO_RHS;
        } else if (!st->done) {
            const double g = sqrt((double)st->s * ob[1]) / sqrt(oy[0]);
            st->gamma = g;
            if (!finite_d(g)) st->done = DONE_NONFINITE;
        }
    }
}

// CG start: gamma = r^T r (r = b~), delta = w^T r; alpha = gamma / delta
__global__ void k_tail_cg0(const double* __restrict__ part_b, int nwg_b,
                           const double* __restrict__ part_s, int nwg_s, DevState* __restrict__ st) {
    __shared__ double ob[2], os[1], tmp[TAIL_THREADS];
    reduce_partials(part_b, nwg_b, 2, ob, tmp);
    reduce_partials(part_s, nwg_s, 1, os, tmp);
    if (threadIdx.x == 0) {
        const double bn = sqrt(ob[0]);
        st->bnorm = bn;
        if (!finite_d(bn)) {
            st->done = DONE_NONFINITE;
            return;
        }
        if (bn == 0.0) {
            st->done = DONE_ZERO_RHS;
            return;
        }
        if (st->done) return;
        st->cg_gamma = ob[1];
        st->cg_alpha = ob[1] / os[0];
        st->cg_beta = 0.0;
        if (!finite_d(st->cg_alpha)) st->done = DONE_NONFINITE;
    }
}

// CG iteration tail: stop test on ||D r|| / ||b||, then beta and alpha
// (alpha = gamma' / (delta - beta gamma' / alpha)).
__global__ void k_tail_cg(const double* __restrict__ part_u, int nwg_u,
                          const double* __restrict__ part_s, int nwg_s, DevState* __restrict__ st,
                          double* __restrict__ hist) {
    if (st->done) return;
    __shared__ double ou[2], os[1], tmp[TAIL_THREADS];
    reduce_partials(part_u, nwg_u, 2, ou, tmp);
    reduce_partials(part_s, nwg_s, 1, os, tmp);
    if (threadIdx.x == 0) {
        const double rel = sqrt(ou[0]) / st->bnorm;
        const int it = st->iter + 1;
        st->iter = it;
        st->cg_rel = rel;
        st->nu_h = rel;
        if (hist && it <= st->n_hist) hist[it - 1] = rel;
        if (!finite_d(rel)) {
            st->done = DONE_NONFINITE;
        } else if (rel < st->tol) {
            st->done = DONE_CONVERGED;
        } else if (it >= st->max_iter) {
            st->done = DONE_MAXITER;
        } else {
            const double g = ou[1];
            const double beta = g / st->cg_gamma;
            st->cg_beta = beta;
            st->cg_alpha = g / (os[0] - beta * g / st->cg_alpha);
            st->cg_gamma = g;
        }
    }
}

__global__ void k_tail_norm(const double* __restrict__ part, int nwg, DevState* __restrict__ st) {
    __shared__ double out[1], tmp[TAIL_THREADS];
    reduce_partials(part, nwg, 1, out, tmp);
    if (threadIdx.x == 0) st->res_norm = sqrt(out[0]);
}

template <int S>
__global__ void k_gram_out(const double* __restrict__ part, int nwg, double* __restrict__ C) {
    constexpr int E = tri_count(S);
    __shared__ double red[E > TAIL_THREADS ? E : TAIL_THREADS];
    __shared__ double tmp[E > TAIL_THREADS ? E : TAIL_THREADS];
    reduce_partials(part, nwg, E, red, tmp);
    for (int e = threadIdx.x; e < E; e += TAIL_THREADS) {
        int i, j;
        tri_ij(e, i, j);
        C[i * S + j] = red[e];
    }
}

__global__ void k_state_init(DevState* st, int s, int max_iter, double tol, double tol0, double tau,
                             int n_hist) {
    double* raw = reinterpret_cast<double*>(st);
    const int nd = (int)(sizeof(DevState) / sizeof(double));
    for (int e = threadIdx.x; e < nd; e += blockDim.x) raw[e] = 0.0;
    __syncthreads();
    if (threadIdx.x == 0) {
        st->s = s;
        st->max_iter = max_iter;
        st->tol = tol;
        st->tol0 = tol0;
        st->tau = tau;
        st->n_hist = n_hist;
        st->width = s;
    }
    if (threadIdx.x < MB_SM) st->active[threadIdx.x] = threadIdx.x < s;
}

// ---------------------------------------------------------------------------
#define MB_TAIL_S(S, CALL)          \
    switch (S) {                    \
        case 1: { constexpr int SS = 1; CALL; } \
        case 2: { constexpr int SS = 2; CALL; } \
        case 4: { constexpr int SS = 4; CALL; } \
        case 8: { constexpr int SS = 8; CALL; } \
        case 16: { constexpr int SS = 16; CALL; } \
        case 32: { constexpr int SS = 32; CALL; } \
    }                               \
    return hipErrorInvalidValue;

hipError_t launch_tail_xi(int S, int nwg, const double* part, DevState* st, hipStream_t s) {
    MB_TAIL_S(S, {
        hipLaunchKernelGGL(k_tail_xi<SS>, dim3(1), dim3(TAIL_THREADS), 0, s, part, nwg, st);
        return hipGetLastError();
    })
}

hipError_t launch_tail_qr(int S, int nwg, const double* part, DevState* st, double* hist, int setup,
                          hipStream_t s) {
    MB_TAIL_S(S, {
        hipLaunchKernelGGL(k_tail_qr<SS>, dim3(1), dim3(TAIL_THREADS), 0, s, part, nwg, st, hist,
                           setup);
        return hipGetLastError();
    })
}

hipError_t launch_tail_ls(int S, int nwg, const double* part, DevState* st, hipStream_t s) {
    MB_TAIL_S(S, {
        hipLaunchKernelGGL(k_tail_ls<SS>, dim3(1), dim3(TAIL_THREADS), 0, s, part, nwg, st);
        return hipGetLastError();
    })
}

hipError_t launch_tail_accept(int nwg, const double* part, DevState* st, hipStream_t s) {
    hipLaunchKernelGGL(k_tail_accept, dim3(1), dim3(TAIL_THREADS), 0, s, part, nwg, st);
    return hipGetLastError();
}

hipError_t launch_tail_true(int nwg, const double* part, DevState* st, hipStream_t s) {
    hipLaunchKernelGGL(k_tail_true, dim3(1), dim3(TAIL_THREADS), 0, s, part, nwg, st);
    return hipGetLastError();
}

hipError_t launch_tail_gamma(int nwg_b, const double* part_b, int nwg_y, const double* part_y,
                             DevState* st, hipStream_t s) {
    hipLaunchKernelGGL(k_tail_gamma, dim3(1), dim3(TAIL_THREADS), 0, s, part_b, nwg_b, part_y, nwg_y,
                       st);
    return hipGetLastError();
}

hipError_t launch_tail_cg0(int nwg_b, const double* part_b, int nwg_s, const double* part_s,
                           DevState* st, hipStream_t s) {
    hipLaunchKernelGGL(k_tail_cg0, dim3(1), dim3(TAIL_THREADS), 0, s, part_b, nwg_b, part_s, nwg_s,
                       st);
    return hipGetLastError();
}

hipError_t launch_tail_cg(int nwg_u, const double* part_u, int nwg_s, const double* part_s,
                          DevState* st, double* hist, hipStream_t s) {
    hipLaunchKernelGGL(k_tail_cg, dim3(1), dim3(TAIL_THREADS), 0, s, part_u, nwg_u, part_s, nwg_s,
                       st, hist);
    return hipGetLastError();
}

hipError_t launch_tail_norm(int nwg, const double* part, DevState* st, hipStream_t s) {
    hipLaunchKernelGGL(k_tail_norm, dim3(1), dim3(TAIL_THREADS), 0, s, part, nwg, st);
    return hipGetLastError();
}

hipError_t launch_gram_out(int S, int nwg, const double* part, double* C, hipStream_t s) {
    MB_TAIL_S(S, {
        hipLaunchKernelGGL(k_gram_out<SS>, dim3(1), dim3(TAIL_THREADS), 0, s, part, nwg, C);
        return hipGetLastError();
    })
}

hipError_t launch_state_init(DevState* st, int s, int max_iter, double tol, double tol0,
                             double tau, int n_hist, hipStream_t stream) {
    hipLaunchKernelGGL(k_state_init, dim3(1), dim3(TAIL_THREADS), 0, stream, st, s, max_iter, tol,
                       tol0, tau, n_hist);
    return hipGetLastError();
}

}  // namespace mb

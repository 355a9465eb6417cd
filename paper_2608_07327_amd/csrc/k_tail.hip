// One-workgroup tail kernels (TAIL_THREADS threads): add up the per-workgroup
// partial sums of a reduction in a fixed order, then do the s x s FP64 work of
// the iteration.  The s x s factorisations run on one wavefront with lane i
// owning row (or column) i and readlane broadcasts between the steps; for
// s >= 16 the inverse of P^T A P is a Gauss-Jordan elimination with one
// thread per entry.
#include "dev_sxs.hpp"
#include "kernels.hpp"

#include <algorithm>

namespace mb {

// First stage of a two-stage fixed-order sum of per-workgroup partials:
// workgroup g adds partials [g c, (g + 1) c) of every entry (c = ceil(nwg / G))
// and writes out[g * E + e].  The one-workgroup tails then add G partials
// instead of nwg, so their latency-bound reduction no longer grows with the
// producer's grid.
__global__ __launch_bounds__(TAIL_THREADS) void k_part_reduce(const double* __restrict__ part,
                                                              int nwg, int E,
                                                              double* __restrict__ out,
                                                              const DevState* __restrict__ st) {
    if (st && st->done) return;
    __shared__ double sums[PART_REDUCE_EMAX];
    __shared__ double tmp[TAIL_THREADS];
    const int G = gridDim.x, g = blockIdx.x;
    const int c = (nwg + G - 1) / G;
    const int w0 = min(nwg, g * c), w1 = min(nwg, w0 + c);
    reduce_partials(part + (int64_t)w0 * E, w1 - w0, E, E, sums, tmp);
    for (int e = threadIdx.x; e < E; e += blockDim.x) out[(int64_t)g * E + e] = sums[e];
}

template <int S>
__global__ __launch_bounds__(TAIL_THREADS) void k_tail_xi(const double* __restrict__ part, int nwg,
                                                          DevState* __restrict__ st) {
    if (st->done) {
        if (threadIdx.x == 0) st->xt_pending = 0;
        return;
    }
    __shared__ double sm[SxsWs<S>::DOUBLES];
    __shared__ int smi[SxsWs<S>::INTS];
    if (threadIdx.x == 0) st->xt_skip = 0;
    tail_xi_body<S>(part, nwg, tri_count(S), st, sm, smi);
    __syncthreads();
    // the update runs unless this tail stopped the loop (P^T A P not SPD)
    if (threadIdx.x == 0) st->xt_pending = st->done == 0;
}

template <int S>
__global__ __launch_bounds__(TAIL_THREADS) void k_tail_qr(const double* __restrict__ part, int nwg,
                                                          DevState* __restrict__ st,
                                                          double* __restrict__ hist, int setup) {
    if (st->done) return;   // (a resume is launched with done cleared)
    __shared__ double sm[SxsWs<S>::DOUBLES];
    __shared__ int smi[SxsWs<S>::INTS];
    tail_qr_body<S>(part, nwg, tri_count(S) + S, st, hist, setup, sm, smi);
}

template <int S>
__global__ __launch_bounds__(TAIL_THREADS) void k_tail_ls(const double* __restrict__ part, int nwg,
                                                          int64_t n, DevState* __restrict__ st) {
    __shared__ double sm[SxsWs<S>::DOUBLES];
    __shared__ int smi[SxsWs<S>::INTS];
    tail_ls_body<S>(part, nwg, 2 * tri_count(S + 1), n, st, sm, smi);
}

// ||r|| of the LS combination and the accept test (the stop test on the
// combination).  After a DONE_LS stop (tol_initial > tol) the solve ends when
// the combination is accepted or the best column itself meets tol, and the
// loop resumes otherwise (done back to 0).
__global__ void k_tail_accept(const double* __restrict__ part, int nwg, DevState* __restrict__ st) {
    __shared__ double out[1], tmp[TAIL_THREADS];
    reduce_partials(part, nwg, 1, 1, out, tmp);
    if (threadIdx.x == 0) {
        const double rel = sqrt(out[0]) / st->bnorm;
        const int done = st->done;
        st->rel_ls = rel;
        const bool ok = st->ls_ok && finite_d(rel) && (rel < st->tol);
        st->accepted = (done == DONE_CONVERGED || done == DONE_LS) && ok;
        if (done == DONE_LS) st->done = (ok || st->nu_h < st->tol) ? DONE_CONVERGED : DONE_RUNNING;
    }
}

__global__ void k_tail_true(const double* __restrict__ part, int nwg, DevState* __restrict__ st) {
    __shared__ double out[1], tmp[TAIL_THREADS];
    reduce_partials(part, nwg, 1, 1, out, tmp);
    if (threadIdx.x == 0) st->rel_true = sqrt(out[0]) / st->bnorm;
}

// true residual of the best column against that of the accepted combination:
// the column replaces the combination when it is lower (the combination's
// coefficients can amplify the rounding drift between A X and B - R)
__global__ void k_tail_pick(const double* __restrict__ part, int nwg, DevState* __restrict__ st) {
    __shared__ double out[1], tmp[TAIL_THREADS];
    reduce_partials(part, nwg, 1, 1, out, tmp);
    if (threadIdx.x == 0) {
        const double rel_h = sqrt(out[0]) / st->bnorm;
        if (rel_h < st->rel_true) {
            st->accepted = 0;
            st->rel_true = rel_h;
        }
    }
}

// ||b||, ||b~||, ||A U||_F -> gamma (scale of the initial guess)
__global__ void k_tail_gamma(const double* __restrict__ part_b, int nwg_b,
                             const double* __restrict__ part_y, int nwg_y,
                             DevState* __restrict__ st) {
    __shared__ double ob[2], oy[1], tmp[TAIL_THREADS];
    reduce_partials(part_b, nwg_b, 2, 2, ob, tmp);
    reduce_partials(part_y, nwg_y, 1, 1, oy, tmp);
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
    reduce_partials(part_b, nwg_b, 2, 2, ob, tmp);
    reduce_partials(part_s, nwg_s, 1, 1, os, tmp);
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
    reduce_partials(part_u, nwg_u, 2, 2, ou, tmp);
    reduce_partials(part_s, nwg_s, 1, 1, os, tmp);
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
    reduce_partials(part, nwg, 1, 1, out, tmp);
    if (threadIdx.x == 0) st->res_norm = sqrt(out[0]);
}

template <int S>
__global__ void k_gram_out(const double* __restrict__ part, int nwg, double* __restrict__ C) {
    constexpr int E = tri_count(S);
    __shared__ double red[E > TAIL_THREADS ? E : TAIL_THREADS];
    __shared__ double tmp[E > TAIL_THREADS ? E : TAIL_THREADS];
    reduce_partials(part, nwg, E, E, red, tmp);
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
        st->ls_inloop = tol0 > tol;
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

hipError_t launch_part_reduce(int nwg, int E, const double* part, double* out, int G,
                              const DevState* st, hipStream_t s) {
    if (E > PART_REDUCE_EMAX || G < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_part_reduce, dim3(G), dim3(TAIL_THREADS), 0, s, part, nwg, E, out, st);
    return hipGetLastError();
}

// Threads of a one-workgroup tail over nwg partials of E entries: four
// wavefronts when each thread then adds at most 32 partials (fewer
// wavefronts to start and to hold at each barrier; the S = 16 inverse still
// has one thread per entry), else TAIL_THREADS.
static int tail_threads(int S, int E, int nwg) {
    constexpr int SMALL = 256;
    if (S > 16) return TAIL_THREADS;
    int tpe = 1;
    while (tpe * 2 * E <= SMALL) tpe *= 2;
    return nwg <= 32 * tpe ? SMALL : TAIL_THREADS;
}

hipError_t launch_tail_xi(int S, int nwg, const double* part, DevState* st, hipStream_t s) {
    const int nt = tail_threads(S, tri_count(S), nwg);
    MB_TAIL_S(S, {
        hipLaunchKernelGGL(k_tail_xi<SS>, dim3(1), dim3(nt), 0, s, part, nwg, st);
        return hipGetLastError();
    })
}

hipError_t launch_tail_qr(int S, int nwg, const double* part, DevState* st, double* hist, int setup,
                          hipStream_t s) {
    const int nt = tail_threads(S, tri_count(S) + S, nwg);
    MB_TAIL_S(S, {
        hipLaunchKernelGGL(k_tail_qr<SS>, dim3(1), dim3(nt), 0, s, part, nwg, st, hist, setup);
        return hipGetLastError();
    })
}

hipError_t launch_tail_ls(int S, int nwg, int64_t n, const double* part, DevState* st,
                          hipStream_t s) {
    MB_TAIL_S(S, {
        hipLaunchKernelGGL(k_tail_ls<SS>, dim3(1), dim3(TAIL_THREADS), 0, s, part, nwg, n, st);
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

hipError_t launch_tail_pick(int nwg, const double* part, DevState* st, hipStream_t s) {
    hipLaunchKernelGGL(k_tail_pick, dim3(1), dim3(TAIL_THREADS), 0, s, part, nwg, st);
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
    const int nt = std::max(tail_threads(1, 2, nwg_u), tail_threads(1, 1, nwg_s));
    hipLaunchKernelGGL(k_tail_cg, dim3(1), dim3(nt), 0, s, part_u, nwg_u, part_s, nwg_s, st, hist);
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

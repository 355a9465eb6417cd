// Host runtime: context lifetime, device buffers, the per-iteration launch
// sequence of Algorithm 1, graph capture of batches of iterations, the stop
// polling, the CG baseline and the FP64 iterative-refinement loop.
#include "runtime.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>

namespace mb {

#define CK(expr)                                                                      \
    do {                                                                              \
        hipError_t _e = (expr);                                                       \
        if (_e != hipSuccess) {                                                       \
            (void)hipGetLastError(); /* the status is ours to report, not the caller's */ \
            c.err = std::string(#expr) + " failed: " + hipGetErrorString(_e);        \
            return _e == hipErrorOutOfMemory ? MBPCG_ERR_OOM : MBPCG_ERR_HIP;         \
        }                                                                             \
    } while (0)

#define CKS(expr)                        \
    do {                                 \
        mbpcg_status _s = (expr);        \
        if (_s != MBPCG_OK) return _s;   \
    } while (0)

constexpr int NWG_MAX = 4096;

static double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

template <class T>
static void dfree(T*& p) {
    if (p) (void)hipFree((void*)p);
    p = nullptr;
}

Ctx::~Ctx() {
    if (stream) (void)hipStreamSynchronize(stream);
    for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
    graphs.clear();
    dfree(rowptr); dfree(colind); dfree(vals); dfree(vals_s);
    if (As && As != A) dfree(As);
    As = nullptr;
    dfree(A); dfree(Alo);
    dfree(d); dfree(bbar); dfree(bdev); dfree(xdev); dfree(rvec); dfree(xacc); dfree(bjinv);
    dfree(U); dfree(Y); dfree(X0); dfree(Xt); dfree(R); dfree(W); dfree(P); dfree(Q); dfree(Plo);
    dfree(qpart); dfree(part_a); dfree(part_b); dfree(part_r); dfree(part_c); dfree(st); dfree(hist);
    if (pinned) (void)hipHostFree(pinned);
    if (st_host) (void)hipHostFree(st_host);
    for (auto& e : ev_poll)
        if (e) (void)hipEventDestroy(e);
    if (ev_a) (void)hipEventDestroy(ev_a);
    if (ev_b) (void)hipEventDestroy(ev_b);
    if (ev_user) (void)hipEventDestroy(ev_user);
    for (auto e : pev) (void)hipEventDestroy(e);
    if (stream) (void)hipStreamDestroy(stream);
}

static mbpcg_status dalloc(Ctx& c, void** p, size_t bytes) {
    hipError_t e = hipMalloc(p, bytes ? bytes : 16);
    if (e == hipErrorOutOfMemory) {
        c.err = "out of device memory";
        return MBPCG_ERR_OOM;
    }
    if (e != hipSuccess) {
        c.err = std::string("hipMalloc failed: ") + hipGetErrorString(e);
        return MBPCG_ERR_HIP;
    }
    return MBPCG_OK;
}
#define DALLOC(ptr, bytes) CKS(dalloc(c, (void**)&(ptr), (bytes)))

static void drop_graphs(Ctx& c) {
    for (auto& kv : c.graphs) (void)hipGraphExecDestroy(kv.second);
    c.graphs.clear();
}

mbpcg_status ctx_init_common(Ctx& c, hipStream_t user_stream) {
    CK(hipGetDevice(&c.device));
    CK(hipDeviceGetAttribute(&c.cus, hipDeviceAttributeMultiprocessorCount, c.device));
    c.user_stream = user_stream;
    CK(hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking));
    CK(hipEventCreateWithFlags(&c.ev_poll[0], hipEventDisableTiming));
    CK(hipEventCreateWithFlags(&c.ev_poll[1], hipEventDisableTiming));
    CK(hipEventCreateWithFlags(&c.ev_user, hipEventDisableTiming));
    // timing-only events (the tuner's and the profile's) record without a
    // system-scope fence: a fence writes back and invalidates the caches
    // around the timed kernel, which the solve never does between kernels
    CK(hipEventCreateWithFlags(&c.ev_a, hipEventDisableSystemFence));
    CK(hipEventCreateWithFlags(&c.ev_b, hipEventDisableSystemFence));
    CK(hipHostMalloc((void**)&c.pinned, 4 * sizeof(int32_t), hipHostMallocDefault));
    CK(hipHostMalloc((void**)&c.st_host, sizeof(DevState), hipHostMallocDefault));
    DALLOC(c.st, sizeof(DevState));
    const size_t nb = sizeof(double) * (size_t)c.n;
    DALLOC(c.d, nb);
    DALLOC(c.bbar, nb);
    DALLOC(c.bdev, nb);
    DALLOC(c.xdev, nb);
    return MBPCG_OK;
}

static mbpcg_status ensure_blocks(Ctx& c, int S) {
    if (c.Scap >= S) return MBPCG_OK;
    drop_graphs(c);
    dfree(c.U); dfree(c.Y); dfree(c.X0); dfree(c.Xt); dfree(c.R); dfree(c.W); dfree(c.P); dfree(c.Q);
    dfree(c.Plo); dfree(c.part_a); dfree(c.part_b); dfree(c.part_r); dfree(c.part_c); dfree(c.qpart);
    const size_t bb = sizeof(double) * (size_t)c.n * S;
    DALLOC(c.U, bb); DALLOC(c.Y, bb); DALLOC(c.X0, bb); DALLOC(c.Xt, bb);
    DALLOC(c.R, bb); DALLOC(c.W, bb); DALLOC(c.P, bb); DALLOC(c.Q, bb);
    DALLOC(c.Plo, sizeof(float) * (size_t)lo_rows_padded(c.n) * S);
    int e = std::max(part_entries_update(S), part_entries_ls(S));
    e = std::max(e, 4);
    c.part_elems = (int64_t)NWG_MAX * e;
    DALLOC(c.part_a, sizeof(double) * c.part_elems);
    DALLOC(c.part_b, sizeof(double) * c.part_elems);
    DALLOC(c.part_r, sizeof(double) * PART_REDUCE_G * PART_REDUCE_EMAX);
    DALLOC(c.part_c, sizeof(double) * c.part_elems);
    if (c.dense) {
        c.qpart_elems = (int64_t)dense_ksplit(c.n) * c.n * S;
        DALLOC(c.qpart, sizeof(double) * c.qpart_elems);
    }
    c.Scap = S;
    return MBPCG_OK;
}

static mbpcg_status ensure_hist(Ctx& c, int64_t cap) {
    if (cap < 1) cap = 1;
    if (c.hist_cap >= cap) return MBPCG_OK;
    drop_graphs(c);
    dfree(c.hist);
    DALLOC(c.hist, sizeof(double) * cap);
    c.hist_cap = cap;
    return MBPCG_OK;
}

// ---------------------------------------------------------------------------
// launch plan of one solve
// ---------------------------------------------------------------------------
struct Plan {
    int s = 1, S = 1;
    int bs = 0;            // block-Jacobi block size (0: none)
    DenseKind kind = DENSE_F64;
    SpmmShape sp;          // sparse block-product tile shape
    int nwg_prod = 1;    // partials of the block product's Gram
    int nwg_spmm = 1;    // grid of the sparse product
    int nwg_upd = 1;     // update / gram_nu grid
    int nwg_dir = 1;
    int nwg_ls = 1;
    int nwg_e = 1;       // element-wise reductions
    int ksplit = 1;
    int nwg_dred = 1;    // dense reduce grid
};

static int round_grid(int64_t ntiles, int cap) {
    int64_t g = std::min<int64_t>(ntiles, cap);
    if (g >= 8) g = g / 8 * 8;
    return (int)std::max<int64_t>(g, 1);
}

static Plan make_plan(Ctx& c, int s, DenseKind kind) {
    Plan pl;
    pl.s = s;
    pl.S = padded_width(s);
    pl.kind = kind;
    const int S = pl.S;
    const int cap = S >= 16 ? 512 : 1024;
    auto it = c.tune.find(S);
    pl.sp = spmm_default_shape(S);
    if (it != c.tune.end() && it->second.sh.T) pl.sp = it->second.sh;
    const int64_t spmm_tiles = (c.n + pl.sp.T - 1) / pl.sp.T;
    pl.nwg_spmm = (it != c.tune.end() && it->second.nwg) ? std::min<int64_t>(it->second.nwg, NWG_MAX)
                                                         : round_grid(spmm_tiles, 2048);
    const int Tu = stream_tile(S);
    const int64_t upd_tiles = (c.n + Tu - 1) / Tu;
    pl.nwg_upd = round_grid(upd_tiles, cap);
    pl.nwg_dir = round_grid(upd_tiles, 1024);
    if (S <= 8 && c.cus > 0) {
        // widths whose partials stay small: fill every CU to the kernels'
        // occupancy (one wave of resident workgroups)
        const int ou = update_blocks_per_cu(S), od = dirupdate_blocks_per_cu(S);
        if (ou > 0) pl.nwg_upd = round_grid(upd_tiles, std::min(ou * c.cus, NWG_MAX));
        if (od > 0) pl.nwg_dir = round_grid(upd_tiles, std::min(od * c.cus, NWG_MAX));
    }
    pl.nwg_ls = round_grid((c.n + 63) / 64, cap);
    pl.nwg_e = round_grid((c.n + MB_BLOCK - 1) / MB_BLOCK, 1024);
    if (c.dense) {
        pl.ksplit = dense_ksplit(c.n);
        const int Tr = dense_reduce_rows(S);
        pl.nwg_dred = round_grid((c.n + Tr - 1) / Tr, cap);
        pl.nwg_prod = pl.nwg_dred;
    } else {
        pl.nwg_prod = pl.nwg_spmm;
    }
    return pl;
}

static CsrDev csr_of(const Ctx& c, bool scaled) {
    CsrDev a;
    a.n = c.n;
    a.nnz = c.nnz;
    a.rowptr = c.rowptr;
    a.colind = c.colind;
    a.vals = scaled ? c.vals_s : c.vals;
    return a;
}

// Q = A~ P (+ Gram partials in `part` unless null).  For the low-precision
// kinds P is read from c.Plo.
static hipError_t launch_product(Ctx& c, const Plan& pl, const double* P, double* Q, double* part,
                                 const DevState* st, int S_override = 0) {
    const int S = S_override ? S_override : pl.S;
    if (!c.dense) {
        const SpmmShape sh = S_override ? spmm_default_shape(S) : pl.sp;
        return launch_spmm(S, sh, pl.nwg_spmm, csr_of(c, true), P, Q, part, st, c.stream);
    }
    const void* A = pl.kind == DENSE_F64 ? (const void*)c.As : (const void*)c.Alo;
    hipError_t e = launch_dense_ap(S, pl.kind, c.n, A, c.n, c.Plo, P, c.qpart, pl.ksplit, st,
                                   c.stream);
    if (e != hipSuccess) return e;
    return launch_dense_reduce(S, pl.kind, c.n, pl.ksplit, c.qpart, P, Q, part, pl.nwg_dred, st,
                               c.stream);
}

// one iteration of Alg. 1's loop, from Xi to the new Sigma
// Partials of E entries from nwg workgroups, as the one-workgroup tails should
// read them: above 2 G partials they are first summed down to G by G
// workgroups (fixed order) into c.part_r.
static hipError_t staged_partials(Ctx& c, int nwg, int E, const double* part,
                                  const double** use, int* use_nwg) {
    // the tail's own threads per entry (a power of two, as in reduce_partials)
    int tpe = 1;
    while (tpe * 2 * E <= TAIL_THREADS) tpe *= 2;
    // one stage when each tail thread adds at most 32 partials
    if (nwg <= 2 * PART_REDUCE_G || nwg <= 32 * tpe) {
        *use = part;
        *use_nwg = nwg;
        return hipSuccess;
    }
    *use = c.part_r;
    *use_nwg = PART_REDUCE_G;
    return launch_part_reduce(nwg, E, part, c.part_r, PART_REDUCE_G, c.st, c.stream);
}

// block-Jacobi arguments of a plan: inverse rows in bjinv, M^-1 blocks in Y
static BjArgs bj_of(const Ctx& c, const Plan& pl) {
    BjArgs a;
    if (pl.bs) {
        a.bs = pl.bs;
        a.inv = c.bjinv;
        a.Y = c.Y;
    }
    return a;
}

// The block-Jacobi inverse of the scaled matrix (after setup_scaling).
static mbpcg_status setup_bjac(Ctx& c, const Plan& pl) {
    if (!pl.bs) return MBPCG_OK;
    if (!c.bjinv || c.bjinv_bs < pl.bs) {
        dfree(c.bjinv);
        c.bjinv = nullptr;
        c.bjinv_bs = 0;
        DALLOC(c.bjinv, sizeof(double) * (size_t)c.n * pl.bs);
        c.bjinv_bs = pl.bs;
        drop_graphs(c);
    }
    if (!c.dense) CK(launch_bjac_setup_csr(pl.bs, csr_of(c, true), c.bjinv, c.st, c.stream));
    else CK(launch_bjac_setup_dense(pl.bs, c.n, c.As, c.n, c.bjinv, c.st, c.stream));
    return MBPCG_OK;
}

// One iteration of Alg. 1's loop, from Xi to the new Sigma.  With ev (six
// events) the phase boundaries are recorded: ev[0] before the product, ev[1]
// after it, ev[2] after the Xi tail, ev[3] after the update, ev[4] after the
// QR tail, ev[5] after the direction update; at level 2 only ev[0] and ev[1].
static hipError_t launch_iteration(Ctx& c, const Plan& pl, double* hist,
                                   const hipEvent_t* ev = nullptr, int level = 1) {
    hipError_t e;
    const double* pr;
    int pn;
    auto mark = [&](int k) {
        return ev && (level == 1 || k <= 1) ? hipEventRecord(ev[k], c.stream) : hipSuccess;
    };
    if ((e = mark(0)) != hipSuccess) return e;
    if ((e = launch_product(c, pl, c.P, c.Q, c.part_a, c.st)) != hipSuccess) return e;
    if ((e = mark(1)) != hipSuccess) return e;
    if ((e = staged_partials(c, pl.nwg_prod, tri_count(pl.S), c.part_a, &pr, &pn)) != hipSuccess)
        return e;
    if ((e = launch_tail_xi(pl.S, pn, pr, c.st, c.stream)) != hipSuccess) return e;
    if ((e = mark(2)) != hipSuccess) return e;
    if ((e = launch_update(pl.S, pl.nwg_upd, c.n, c.P, c.Q, c.Xt, c.R, c.W, c.d, c.part_b, c.st,
                           c.stream, bj_of(c, pl))) != hipSuccess)
        return e;
    if ((e = mark(3)) != hipSuccess) return e;
    if ((e = staged_partials(c, pl.nwg_upd, tri_count(pl.S) + pl.S, c.part_b, &pr, &pn)) !=
        hipSuccess)
        return e;
    if ((e = launch_tail_qr(pl.S, pn, pr, c.st, hist, 0, c.stream)) != hipSuccess) return e;
    if ((e = mark(4)) != hipSuccess) return e;
    if ((e = launch_dirupdate(pl.S, pl.nwg_dir, c.n, c.W, c.P, c.Plo, pl.kind, 0, c.st,
                              c.stream, pl.bs ? c.Y : nullptr, c.Xt)) != hipSuccess)
        return e;
    return mark(5);
}

// One CG-CG step.  With ev: ev[0] before the vector update, ev[1] after it,
// ev[2] after the SpMV, ev[3..5] after the tail; at level 2 only ev[1] and
// ev[2].
static hipError_t launch_cg_iteration(Ctx& c, const Plan& pl, double* hist,
                                      const hipEvent_t* ev = nullptr, int level = 1) {
    hipError_t e;
    auto mark = [&](int k) {
        return ev && (level == 1 || k == 1 || k == 2) ? hipEventRecord(ev[k], c.stream)
                                                      : hipSuccess;
    };
    if ((e = mark(0)) != hipSuccess) return e;
    if ((e = launch_cg_update(pl.nwg_e, c.n, c.P, c.W, c.Xt, c.R, c.Q, c.d, c.part_c, c.st,
                              c.stream, bj_of(c, pl))) != hipSuccess)
        return e;
    if ((e = mark(1)) != hipSuccess) return e;
    // the product of the (preconditioned) residual: u = M^-1 r lives in Y
    if ((e = launch_product(c, pl, pl.bs ? c.Y : c.R, c.Q, c.part_a, c.st)) != hipSuccess) return e;
    if ((e = mark(2)) != hipSuccess) return e;
    if ((e = launch_tail_cg(pl.nwg_e, c.part_c, pl.nwg_prod, c.part_a, c.st, hist, c.stream)) !=
        hipSuccess)
        return e;
    for (int k = 3; k < 6; ++k)
        if ((e = mark(k)) != hipSuccess) return e;
    return hipSuccess;
}

static mbpcg_status get_graph(Ctx& c, const Plan& pl, int m, int cg, hipGraphExec_t* out) {
    auto key = std::make_tuple((cg * 2 + c.dense) * 64 + pl.bs, pl.S, m,
                               pl.sp.T * 10000 + pl.sp.SL * 1000 + pl.sp.V * 100 + pl.sp.U * 10 + pl.sp.W,
                               pl.nwg_spmm, (int)pl.kind);
    auto it = c.graphs.find(key);
    if (it != c.graphs.end()) {
        *out = it->second;
        return MBPCG_OK;
    }
    hipGraph_t g = nullptr;
    CK(hipStreamBeginCapture(c.stream, hipStreamCaptureModeThreadLocal));
    hipError_t le = hipSuccess;
    for (int i = 0; i < m && le == hipSuccess; ++i)
        le = cg ? launch_cg_iteration(c, pl, c.hist) : launch_iteration(c, pl, c.hist);
    hipError_t ce = hipStreamEndCapture(c.stream, &g);
    if (le != hipSuccess || ce != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        c.err = std::string("graph capture failed: ") +
                hipGetErrorString(le != hipSuccess ? le : ce);
        return MBPCG_ERR_HIP;
    }
    hipGraphExec_t ex = nullptr;
    hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) {
        c.err = std::string("graph instantiate failed: ") + hipGetErrorString(ie);
        return MBPCG_ERR_HIP;
    }
    c.graphs[key] = ex;
    *out = ex;
    return MBPCG_OK;
}

static int auto_poll(const Ctx& c, int cg) {
    // iterations per graph launch: enough to hide the host check, few enough
    // that the no-op tail after convergence stays short
    if (c.n * (cg ? 1 : 4) < (1 << 18)) return 32;
    return 16;
}

static mbpcg_status read_state(Ctx& c) {
    CK(hipMemcpyAsync(c.st_host, c.st, sizeof(DevState), hipMemcpyDeviceToHost, c.stream));
    CK(hipStreamSynchronize(c.stream));
    return MBPCG_OK;
}

// Run batches of m iterations until the device sets `done`.
static mbpcg_status run_loop(Ctx& c, const Plan& pl, const mbpcg_params& p, int cg, double* ms_loop,
                            double* prof_ms, double* prof_n) {
    const int m = p.poll_every > 0 ? p.poll_every : auto_poll(c, cg);
    const double t0 = now_ms();
    // iterations done before this call (a loop resumed after a least squares)
    const int64_t it0 = c.st_host->iter;
    if (p.profile) {
        // The iterations are launched directly, with HIP events between the
        // kernels of every iteration (the per-step timing of Sec. 3, Table 2;
        // events recorded inside graphs do not carry timestamps here), and
        // polled like the graph path so the host never waits inside an
        // iteration.  Level 2 records only the two events around the block
        // product.
        constexpr int EV = 6;
        const int level = p.profile == 2 ? 2 : 1;
        const int64_t max_it = p.max_iter + 2 * (int64_t)m + 2;
        int64_t issued = 0;
        auto issue_batch = [&](int slot) -> mbpcg_status {
            for (int i = 0; i < m && issued < max_it; ++i, ++issued) {
                while ((int64_t)c.pev.size() < (issued + 1) * EV) {
                    hipEvent_t e;
                    CK(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
                    c.pev.push_back(e);
                }
                const hipEvent_t* ev = &c.pev[issued * EV];
                CK(cg ? launch_cg_iteration(c, pl, c.hist, ev, level)
                      : launch_iteration(c, pl, c.hist, ev, level));
            }
            CK(hipMemcpyAsync(c.pinned + 2 * slot, c.st, 8, hipMemcpyDeviceToHost, c.stream));
            CK(hipEventRecord(c.ev_poll[slot], c.stream));
            return MBPCG_OK;
        };
        CKS(issue_batch(0));
        CKS(issue_batch(1));
        for (int64_t k = 0;; ++k) {
            const int slot = (int)(k & 1);
            CK(hipEventSynchronize(c.ev_poll[slot]));
            if (c.pinned[2 * slot]) break;
            if (issued >= max_it) break;
            CKS(issue_batch(slot));
        }
        CK(hipStreamSynchronize(c.stream));
        *ms_loop = now_ms() - t0;
        CKS(read_state(c));
        const int64_t ran = std::min<int64_t>(c.st_host->iter - it0, issued);
        for (int64_t i = 0; i < ran; ++i) {
            const hipEvent_t* ev = &c.pev[i * EV];
            for (int k = 0; k + 1 < EV; ++k) {
                if (level == 2 && k != (cg ? 1 : 0)) continue;
                float ms = 0.f;
                CK(hipEventElapsedTime(&ms, ev[k], ev[k + 1]));
                const int q = cg ? (k == 1 ? 0 : (k == 0 ? 2 : 7)) : k;
                c.phase_ms[q] += ms;
                if (k == (cg ? 1 : 0)) {
                    *prof_ms += ms;
                    *prof_n += 1.0;
                }
            }
        }
        return MBPCG_OK;
    }
    hipGraphExec_t g = nullptr;
    CKS(get_graph(c, pl, m, cg, &g));
    const int64_t max_launch = p.max_iter / m + 4;
    int64_t launched = 0;
    for (int k = 0; k < 2; ++k) {
        CK(hipGraphLaunch(g, c.stream));
        CK(hipMemcpyAsync(c.pinned + 2 * k, c.st, 8, hipMemcpyDeviceToHost, c.stream));
        CK(hipEventRecord(c.ev_poll[k], c.stream));
        ++launched;
    }
    for (int64_t k = 0;; ++k) {
        const int slot = (int)(k & 1);
        CK(hipEventSynchronize(c.ev_poll[slot]));
        if (c.pinned[2 * slot]) break;
        if (launched >= max_launch) break;
        CK(hipGraphLaunch(g, c.stream));
        CK(hipMemcpyAsync(c.pinned + 2 * slot, c.st, 8, hipMemcpyDeviceToHost, c.stream));
        CK(hipEventRecord(c.ev_poll[slot], c.stream));
        ++launched;
    }
    CK(hipStreamSynchronize(c.stream));
    *ms_loop = now_ms() - t0;
    return MBPCG_OK;
}


static mbpcg_status status_of(int done) {
    switch (done) {
        case DONE_CONVERGED: return MBPCG_OK;
        case DONE_ZERO_RHS: return MBPCG_OK;
        case DONE_MAXITER: return MBPCG_NOT_CONVERGED;
        case DONE_BREAKDOWN: return MBPCG_ERR_BREAKDOWN;
        case DONE_NOTSPD: return MBPCG_ERR_NOT_SPD;
        case DONE_NONFINITE: return MBPCG_ERR_NONFINITE;
    }
    return MBPCG_NOT_CONVERGED;
}

// diag, scaling (Sec. 1), b~ and ||b|| partials
static mbpcg_status setup_scaling(Ctx& c, const Plan& pl, const double* b, int jacobi) {
    if (!c.dense) {
        CK(launch_diag_csr(csr_of(c, false), jacobi, c.d, c.st, c.stream));
        if (jacobi) {
            if (!c.vals_s) DALLOC(c.vals_s, sizeof(double) * (size_t)std::max<int64_t>(c.nnz, 1));
            CK(launch_scale_csr(csr_of(c, false), c.d, c.vals_s, c.stream));
        } else {
            if (!c.vals_s) DALLOC(c.vals_s, sizeof(double) * (size_t)std::max<int64_t>(c.nnz, 1));
            CK(hipMemcpyAsync(c.vals_s, c.vals, sizeof(double) * c.nnz, hipMemcpyDeviceToDevice,
                              c.stream));
        }
    } else {
        CK(launch_diag_dense(c.n, c.A, c.n, jacobi, c.d, c.st, c.stream));
        if (jacobi) {
            if (!c.As || c.As == c.A) {
                c.As = nullptr;
                DALLOC(c.As, sizeof(double) * (size_t)c.n * c.n);
                drop_graphs(c);
            }
            CK(launch_scale_dense(c.n, c.A, c.n, c.d, c.As, c.stream));
        } else {
            if (c.As && c.As != c.A) {
                dfree(c.As);
                drop_graphs(c);
            }
            if (c.As != c.A) drop_graphs(c);
            c.As = c.A;
        }
    }
    CK(launch_rhs(pl.nwg_e, c.n, b, c.d, c.bbar, c.part_c, c.stream));
    return MBPCG_OK;
}

// ---------------------------------------------------------------------------
// Algorithm 1 on device-resident b and x.
// ---------------------------------------------------------------------------
static mbpcg_status run_mbpcg(Ctx& c, const double* b, double* x, const double* Udev,
                              const mbpcg_params& p, DenseKind kind, bool true_resid,
                              mbpcg_info& info) {
    const int s = p.s;
    Plan pl = make_plan(c, s, kind);
    pl.bs = p.precond == MBPCG_PRECOND_BLOCK_JACOBI ? p.block_size : 0;
    const int S = pl.S;
    CKS(ensure_blocks(c, S));
    CKS(ensure_hist(c, p.history ? p.max_iter : 1));
    const int jac = p.precond != MBPCG_PRECOND_NONE;
    const double tol0 = p.tol_initial > 0 ? p.tol_initial : p.tol;
    const double tau = p.tau > 0 ? p.tau : 1e-12;
    const double t0 = now_ms();
    memset(c.st_host, 0, sizeof(DevState));

    CK(launch_state_init(c.st, s, (int)std::min<int64_t>(p.max_iter, INT32_MAX), p.tol, tol0, tau,
                         p.history ? (int)std::min<int64_t>(p.max_iter, INT32_MAX) : 0, c.stream));
    CKS(setup_scaling(c, pl, b, jac));
    CKS(setup_bjac(c, pl));
    // random block U
    if (Udev) CK(launch_pad_block(S, c.n, s, Udev, c.U, c.stream));
    else CK(launch_uniform(S, c.n, s, p.seed, c.U, c.stream));
    // initial guess: Y = A~ U, ||Y||_F
    if (kind != DENSE_F64) CK(launch_block_to_lo(kind, c.n, S, c.U, c.Plo, c.stream));
    CK(launch_product(c, pl, c.U, c.Y, nullptr, c.st));
    CK(launch_ynorm(S, pl.nwg_e, c.n, c.Y, c.part_a, c.stream));
    CK(launch_tail_gamma(pl.nwg_e, c.part_c, pl.nwg_e, c.part_a, c.st, c.stream));
    // scaled right-hand sides, R0, first Cholesky QR, P0
    CK(launch_init(S, c.n, s, c.U, c.Y, c.bbar, c.X0, c.Xt, c.R, c.st, c.stream));
    // (preconditioned: Y = M^-1 R0, Gram R0^T Y, P0 = M^-1 W0 = Y M)
    CK(launch_gram_nu(S, pl.nwg_upd, c.n, c.R, c.d, c.part_b, c.stream, bj_of(c, pl)));
    CK(launch_tail_qr(S, pl.nwg_upd, c.part_b, c.st, nullptr, 1, c.stream));
    CK(hipMemcpyAsync(c.W, c.R, sizeof(double) * (size_t)c.n * S, hipMemcpyDeviceToDevice,
                      c.stream));
    CK(launch_dirupdate(S, pl.nwg_dir, c.n, c.W, c.P, c.Plo, kind, 1, c.st, c.stream,
                        pl.bs ? c.Y : nullptr, c.Xt));
    const double t_setup = now_ms();

    double ms_loop = 0.0, prof_ms = 0.0, prof_n = 0.0;
    for (double& v : c.phase_ms) v = 0.0;
    // least squares of the termination: c^, x = D^-1 (X~ + X0) c^ and the
    // accept test (its partials avoid part_b, which a resumed Cholesky QR
    // still reads)
    auto least_squares = [&]() -> mbpcg_status {
        CK(launch_ls_gram(S, pl.nwg_ls, c.n, b, c.R, c.d, c.part_a, c.st, c.stream));
        CK(launch_tail_ls(S, pl.nwg_ls, c.n, c.part_a, c.st, c.stream));
        CK(launch_ls_apply(S, pl.nwg_e, c.n, c.Xt, c.X0, c.R, b, c.d, x, c.part_c, c.st,
                           c.stream));
        CK(launch_tail_accept(pl.nwg_e, c.part_c, c.st, c.stream));
        return MBPCG_OK;
    };
    bool ls_done = false;
    for (;;) {
        double ms = 0.0;
        CKS(run_loop(c, pl, p, 0, &ms, &prof_ms, &prof_n));
        ms_loop += ms;
        CKS(read_state(c));
        if (c.st_host->done != DONE_LS) break;
        // tol_initial > tol (Alg. 1's two tests): the best column met
        // tol_initial, so this iteration's combination is tried; the solve
        // ends if it meets tol or the best column does, else the loop goes on
        // from this iteration's Cholesky QR and direction update
        CKS(least_squares());
        CKS(read_state(c));
        ls_done = c.st_host->done != DONE_RUNNING;
        if (ls_done) break;
        const double* pr;
        int pn;
        CK(staged_partials(c, pl.nwg_upd, tri_count(S) + S, c.part_b, &pr, &pn));
        CK(launch_tail_qr(S, pn, pr, c.st, nullptr, 2, c.stream));
        CK(launch_dirupdate(S, pl.nwg_dir, c.n, c.W, c.P, c.Plo, kind, 0, c.st, c.stream,
                            pl.bs ? c.Y : nullptr, c.Xt));
    }
    const int done = c.st_host->done;

    if (done == DONE_ZERO_RHS) {
        CK(hipMemsetAsync(x, 0, sizeof(double) * c.n, c.stream));
    } else {
        if (done == DONE_CONVERGED && !ls_done) CKS(least_squares());
        CK(launch_select(S, c.n, c.Xt, c.X0, c.d, x, c.st, 0, c.stream));
        if (true_resid) {
            // partial sums of ||b - A v||^2 (original A) into part_a
            auto residual = [&](const double* v) -> hipError_t {
                if (!c.dense) return launch_resid_csr(pl.nwg_e, csr_of(c, false), b, v, c.part_a,
                                                      c.stream);
                hipError_t e = launch_dense_ap(1, DENSE_F64, c.n, c.A, c.n, nullptr, v, c.qpart,
                                               pl.ksplit, nullptr, c.stream);
                if (e != hipSuccess) return e;
                return launch_dense_resid_reduce(c.n, pl.ksplit, c.qpart, b, nullptr, c.part_a,
                                                 pl.nwg_e, c.stream);
            };
            CK(residual(x));
            CK(launch_tail_true(pl.nwg_e, c.part_a, c.st, c.stream));
            if (done == DONE_CONVERGED) {
                CKS(read_state(c));
                const DevState& h0 = *c.st_host;
                // an accepted combination that misses the tolerance on its true
                // residual gives way to the best column when that one is lower
                if (h0.accepted && !(h0.rel_true < h0.tol)) {
                    double* xh = c.W;  // idle after the loop: n x S >= n doubles
                    CK(launch_select(S, c.n, c.Xt, c.X0, c.d, xh, c.st, 1, c.stream));
                    CK(residual(xh));
                    CK(launch_tail_pick(pl.nwg_e, c.part_a, c.st, c.stream));
                    CK(launch_select(S, c.n, c.Xt, c.X0, c.d, x, c.st, 0, c.stream));
                }
            }
        }
    }
    CKS(read_state(c));
    const double t1 = now_ms();
    const DevState& h = *c.st_host;
    info.iterations += h.iter;
    info.best_column = h.h;
    info.final_width = h.width;
    info.deflations += h.deflations;
    info.used_fallback = (done == DONE_ZERO_RHS) ? 0 : (h.accepted ? 0 : 1);
    info.rel_res_best_basis = h.nu_h;
    info.rel_res_ls = (done == DONE_CONVERGED) ? h.rel_ls : NAN;
    info.rel_res_true = (done == DONE_ZERO_RHS) ? 0.0 : h.rel_true;
    info.ms_total += t1 - t0;
    info.ms_per_iter = h.iter > 0 ? ms_loop / h.iter : 0.0;
    info.ms_spmm += prof_ms;
    info.spmm_launches += (int64_t)prof_n;
    for (int k = 0; k < 8; ++k) info.ms_phase[k] += c.phase_ms[k];
    (void)t_setup;
    if (p.history && h.iter > 0) {
        const int64_t k = std::min<int64_t>(h.iter, p.max_iter);
        CK(hipMemcpy(p.history, c.hist, sizeof(double) * k, hipMemcpyDeviceToHost));
    }
    return status_of(done);
}

// ---------------------------------------------------------------------------
// Chronopoulos-Gear CG (x0 = 0) on the same scaled system and stop rule.
// ---------------------------------------------------------------------------
static mbpcg_status run_cg(Ctx& c, const double* b, double* x, const mbpcg_params& p,
                           mbpcg_info& info) {
    Plan pl = make_plan(c, 1, DENSE_F64);
    pl.bs = p.precond == MBPCG_PRECOND_BLOCK_JACOBI ? p.block_size : 0;
    CKS(ensure_blocks(c, 1));
    CKS(ensure_hist(c, p.history ? p.max_iter : 1));
    const int jac = p.precond != MBPCG_PRECOND_NONE;
    const double t0 = now_ms();
    memset(c.st_host, 0, sizeof(DevState));
    CK(launch_state_init(c.st, 1, (int)std::min<int64_t>(p.max_iter, INT32_MAX), p.tol, p.tol, 1e-12,
                         p.history ? (int)std::min<int64_t>(p.max_iter, INT32_MAX) : 0, c.stream));
    CKS(setup_scaling(c, pl, b, jac));
    CKS(setup_bjac(c, pl));
    CK(launch_cg_init(c.n, c.bbar, c.Xt, c.R, c.P, c.W, c.stream));
    if (pl.bs) {
        // u = M^-1 r0 and (||b||^2, r0^T u) in place of the right-hand side sums
        CK(launch_cg_prec(pl.nwg_e, c.n, c.R, c.d, c.part_c, bj_of(c, pl), c.stream));
        CK(launch_product(c, pl, c.Y, c.Q, c.part_a, c.st));
    } else {
        CK(launch_product(c, pl, c.R, c.Q, c.part_a, c.st));
    }
    CK(launch_tail_cg0(pl.nwg_e, c.part_c, pl.nwg_prod, c.part_a, c.st, c.stream));
    double ms_loop = 0.0, prof_ms = 0.0, prof_n = 0.0;
    for (double& v : c.phase_ms) v = 0.0;
    CKS(run_loop(c, pl, p, 1, &ms_loop, &prof_ms, &prof_n));
    CKS(read_state(c));
    const int done = c.st_host->done;
    if (done == DONE_ZERO_RHS) {
        CK(hipMemsetAsync(x, 0, sizeof(double) * c.n, c.stream));
    } else {
        CK(launch_unscale(c.n, c.Xt, c.d, x, c.stream));
        if (!c.dense) {
            CK(launch_resid_csr(pl.nwg_e, csr_of(c, false), b, x, c.part_a, c.stream));
        } else {
            CK(launch_dense_ap(1, DENSE_F64, c.n, c.A, c.n, nullptr, x, c.qpart, pl.ksplit, nullptr,
                               c.stream));
            CK(launch_dense_resid_reduce(c.n, pl.ksplit, c.qpart, b, nullptr, c.part_a, pl.nwg_e,
                                         c.stream));
        }
        CK(launch_tail_true(pl.nwg_e, c.part_a, c.st, c.stream));
    }
    CKS(read_state(c));
    const double t1 = now_ms();
    const DevState& h = *c.st_host;
    info.iterations = h.iter;
    info.best_column = 0;
    info.final_width = 1;
    info.rel_res_best_basis = h.cg_rel;
    info.rel_res_ls = NAN;
    info.rel_res_true = (done == DONE_ZERO_RHS) ? 0.0 : h.rel_true;
    info.ms_total = t1 - t0;
    info.ms_per_iter = h.iter > 0 ? ms_loop / h.iter : 0.0;
    info.ms_spmm = prof_ms;
    info.spmm_launches = (int64_t)prof_n;
    for (int k = 0; k < 8; ++k) info.ms_phase[k] = c.phase_ms[k];
    if (p.history && h.iter > 0) {
        const int64_t k = std::min<int64_t>(h.iter, p.max_iter);
        CK(hipMemcpy(p.history, c.hist, sizeof(double) * k, hipMemcpyDeviceToHost));
    }
    return status_of(done);
}

// ---------------------------------------------------------------------------
// FP64 iterative refinement around a low-precision inner MBPCG (dense A).
// ---------------------------------------------------------------------------
static mbpcg_status run_ir(Ctx& c, const double* b, double* x, const double* Udev,
                           const mbpcg_params& p, mbpcg_info& info) {
    const DenseKind kind = p.precision == MBPCG_FP32_IR ? DENSE_F32 : DENSE_BF16;
    const double t0 = now_ms();
    if (!c.rvec) DALLOC(c.rvec, sizeof(double) * c.n);
    if (!c.xacc) DALLOC(c.xacc, sizeof(double) * c.n);
    // scaling and the low-precision copy of A are made once per solve
    Plan pl = make_plan(c, p.s, kind);
    CKS(ensure_blocks(c, pl.S));
    const int jac = p.precond == MBPCG_PRECOND_JACOBI;
    CK(launch_state_init(c.st, p.s, 1, p.tol, p.tol, 1e-12, 0, c.stream));
    CKS(setup_scaling(c, pl, b, jac));
    if (!c.Alo || c.alo_kind != kind) {
        dfree(c.Alo);
        DALLOC(c.Alo, dense_lo_bytes(kind, c.n));
        c.alo_kind = kind;
        drop_graphs(c);
    }
    CK(launch_cast_dense(kind, c.n, c.As, c.n, c.Alo, c.stream));
    CK(hipMemsetAsync(c.xacc, 0, sizeof(double) * c.n, c.stream));
    CK(hipMemcpyAsync(c.rvec, b, sizeof(double) * c.n, hipMemcpyDeviceToDevice, c.stream));
    // ||b|| in FP64 (the k-split partials of A * 0 are the zeros in xacc)
    CK(launch_dense_resid_reduce(c.n, 1, c.xacc, b, nullptr, c.part_c, pl.nwg_e, c.stream));
    CK(launch_tail_norm(pl.nwg_e, c.part_c, c.st, c.stream));
    CKS(read_state(c));
    const double bnorm = c.st_host->res_norm;
    if (!std::isfinite(bnorm)) return MBPCG_ERR_NONFINITE;
    if (bnorm == 0.0) {
        if (x) CK(hipMemsetAsync(x, 0, sizeof(double) * c.n, c.stream));
        CK(hipStreamSynchronize(c.stream));
        info.rel_res_true = 0.0;
        info.ms_total = now_ms() - t0;
        return MBPCG_OK;
    }
    mbpcg_params inner = p;
    inner.tol_initial = 0.0;
    inner.history = nullptr;
    mbpcg_status last = MBPCG_OK;
    double rel = 1.0;
    bool stalled = false;
    int outer = 0;
    const int max_outer = p.max_outer > 0 ? p.max_outer : 50;
    const double floor_tol = p.inner_tol > 0 ? p.inner_tol : 5e-6;
    // the FP64 residual of the new x, into rvec and rel
    auto fp64_residual = [&]() -> mbpcg_status {
        CK(launch_dense_ap(1, DENSE_F64, c.n, c.A, c.n, nullptr, c.xacc, c.qpart, pl.ksplit, nullptr,
                           c.stream));
        CK(launch_dense_resid_reduce(c.n, pl.ksplit, c.qpart, b, c.rvec, c.part_a, pl.nwg_e,
                                     c.stream));
        CK(launch_tail_norm(pl.nwg_e, c.part_a, c.st, c.stream));
        CKS(read_state(c));
        rel = c.st_host->res_norm / bnorm;
        return MBPCG_OK;
    };
    for (outer = 1; outer <= max_outer; ++outer) {
        // an inner solve needs to reduce r only as far as this outer step can
        // finish the job: ir_tol / rel with a factor 2 of margin, never looser
        // than 0.1 and never tighter than inner_tol
        inner.tol = std::min(0.1, std::max(floor_tol, 0.5 * p.ir_tol / rel));
        inner.seed = p.seed + (uint64_t)(outer - 1) * 7919u;
        mbpcg_info ii;
        memset(&ii, 0, sizeof(ii));
        // inner solve A_lo d = r; d lands in c.xdev
        last = run_mbpcg(c, c.rvec, c.xdev, outer == 1 ? Udev : nullptr, inner, kind, false, ii);
        info.iterations += ii.iterations;
        info.deflations += ii.deflations;
        info.ms_spmm += ii.ms_spmm;
        info.spmm_launches += ii.spmm_launches;
        for (int k = 0; k < 8; ++k) info.ms_phase[k] += ii.ms_phase[k];
        info.best_column = ii.best_column;
        info.final_width = ii.final_width;
        info.used_fallback = ii.used_fallback;
        info.rel_res_best_basis = ii.rel_res_best_basis;
        info.rel_res_ls = ii.rel_res_ls;
        if (last == MBPCG_ERR_HIP || last == MBPCG_ERR_OOM) return last;
        if (last == MBPCG_ERR_NOT_SPD || last == MBPCG_ERR_NONFINITE) break;
        // x += d;  r = b - A x with the FP64 A
        const double rel_before = rel;
        CK(launch_axpy_ir(c.n, c.xacc, c.xdev, 1.0, c.stream));
        CKS(fp64_residual());
        if (!(rel < rel_before)) {
            // no progress (the low-precision operator is too far from A for
            // this system): take the step back and stop with the best x
            CK(launch_axpy_ir(c.n, c.xacc, c.xdev, -1.0, c.stream));
            CKS(fp64_residual());
            stalled = true;
            break;
        }
        if (!(rel > p.ir_tol)) break;
    }
    info.rel_res_true = rel;
    if (stalled && last == MBPCG_OK) last = MBPCG_NOT_CONVERGED;
    if (x) CK(hipMemcpyAsync(x, c.xacc, sizeof(double) * c.n, hipMemcpyDeviceToDevice, c.stream));
    CK(hipStreamSynchronize(c.stream));
    info.outer_iterations = std::min(outer, max_outer);
    info.ms_total = now_ms() - t0;
    info.ms_per_iter = info.iterations > 0 ? info.ms_total / info.iterations : 0.0;
    if (!std::isfinite(rel)) return MBPCG_ERR_NONFINITE;
    if (rel <= p.ir_tol) return MBPCG_OK;
    return last < 0 ? last : MBPCG_NOT_CONVERGED;
}

// ---------------------------------------------------------------------------
// entry points used by the C ABI
// ---------------------------------------------------------------------------
mbpcg_status solve_entry(Ctx& c, const double* b, double* x, mbpcg_mem mem,
                         const mbpcg_params& p, mbpcg_info& info, int cg) {
    CK(hipSetDevice(c.device));
    // order after the caller's stream
    CK(hipEventRecord(c.ev_user, c.user_stream));
    CK(hipStreamWaitEvent(c.stream, c.ev_user, 0));
    const double* bd = b;
    double* xd = x;
    const double* Ud = nullptr;
    if (mem == MBPCG_MEM_HOST) {
        CK(hipMemcpyAsync(c.bdev, b, sizeof(double) * c.n, hipMemcpyHostToDevice, c.stream));
        bd = c.bdev;
        xd = c.xdev;
    }
    if (p.U && !cg) {
        if (mem == MBPCG_MEM_HOST) {
            CKS(ensure_blocks(c, padded_width(p.s)));
            CK(hipMemcpyAsync(c.Y, p.U, sizeof(double) * c.n * p.s, hipMemcpyHostToDevice,
                              c.stream));
            Ud = c.Y;
        } else {
            Ud = p.U;
        }
    }
    mbpcg_status st;
    if (cg) st = run_cg(c, bd, xd, p, info);
    else if (p.precision == MBPCG_FP64) st = run_mbpcg(c, bd, xd, Ud, p, DENSE_F64, true, info);
    else st = run_ir(c, bd, mem == MBPCG_MEM_HOST ? nullptr : xd, Ud, p, info);
    if (st == MBPCG_ERR_HIP || st == MBPCG_ERR_OOM) return st;
    if (!cg && p.precision == MBPCG_FP64 && p.X_out) {
        // block iterate at exit (zero when the setup did not finish, e.g. b = 0)
        const size_t bytes = sizeof(double) * (size_t)c.n * p.s;
        double* dst = mem == MBPCG_MEM_HOST ? c.W : p.X_out;
        if (c.st_host->ready)
            CK(launch_export_x(padded_width(p.s), c.n, p.s, c.Xt, c.X0, dst, c.stream));
        else
            CK(hipMemsetAsync(dst, 0, bytes, c.stream));
        if (mem == MBPCG_MEM_HOST)
            CK(hipMemcpyAsync(p.X_out, c.W, bytes, hipMemcpyDeviceToHost, c.stream));
    }
    if (mem == MBPCG_MEM_HOST) {
        const double* src = (!cg && p.precision != MBPCG_FP64) ? c.xacc : c.xdev;
        CK(hipMemcpyAsync(x, src, sizeof(double) * c.n, hipMemcpyDeviceToHost, c.stream));
    }
    CK(hipStreamSynchronize(c.stream));
    return st;
}

mbpcg_status block_product_entry(Ctx& c, int s, int jacobi, const double* P, double* Q, double* C) {
    CK(hipSetDevice(c.device));
    CK(hipEventRecord(c.ev_user, c.user_stream));
    CK(hipStreamWaitEvent(c.stream, c.ev_user, 0));
    Plan pl = make_plan(c, s, DENSE_F64);
    CKS(ensure_blocks(c, pl.S));
    CK(launch_state_init(c.st, s, 1, 1.0, 1.0, 1e-12, 0, c.stream));
    CKS(setup_scaling(c, pl, c.bdev, jacobi));
    CK(launch_state_init(c.st, s, 1, 1.0, 1.0, 1e-12, 0, c.stream));
    CK(launch_product(c, pl, P, Q, c.part_a, c.st));
    hipError_t launch_gram_out(int S, int nwg, const double* part, double* C, hipStream_t s);
    CK(launch_gram_out(pl.S, pl.nwg_prod, c.part_a, C, c.stream));
    CK(hipStreamSynchronize(c.stream));
    return MBPCG_OK;
}

// ---------------------------------------------------------------------------
// The block product without any allocation, for callers that cannot allocate
// (code under graph capture, serving loops).  Its Gram partial sums go to a
// fixed device array instead of the context's buffers; each GPU holds its
// own copy until the process ends, and every call on that GPU shares it, so
// calls that overlap on one GPU race.  The product's grid is capped so that
// its partials fit; every slot a call reads is written by that call first.
// ---------------------------------------------------------------------------
constexpr int64_t NOALLOC_SCRATCH_DOUBLES = 1 << 19;   // 4 MiB of partial sums
static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_DOUBLES];

static std::mutex g_scratch_mu;
static double* g_scratch_ptr[256] = {};

// device address of this GPU's scratch array (the device must be current)
static mbpcg_status scratch_address(Ctx& c, double** out) {
    int dev = 0;
    CK(hipGetDevice(&dev));
    if (dev < 0 || dev >= 256) {
        c.err = "device index out of range for the fixed scratch array";
        return MBPCG_ERR_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        CK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[dev];
    return MBPCG_OK;
}

mbpcg_status block_product_noalloc_entry(Ctx& c, int s, int jacobi, const double* P, double* Q,
                                         double* C) {
    if (c.dense) {
        c.err = "the allocation-free block product takes CSR matrices only (the dense product's "
                "split-K partials exceed the fixed scratch array)";
        return MBPCG_ERR_UNSUPPORTED;
    }
    if (!c.vals_s) {
        c.err = "context has no scaled-value buffer";
        return MBPCG_ERR_UNSUPPORTED;
    }
    CK(hipSetDevice(c.device));
    double* part = nullptr;
    CKS(scratch_address(c, &part));
    CK(hipEventRecord(c.ev_user, c.user_stream));
    CK(hipStreamWaitEvent(c.stream, c.ev_user, 0));
    // the launch plan of the allocating entry (tuned shape and grid); the
    // grid is lowered to the largest multiple of 8 (the XCD-aware tile order)
    // whose partials fit when it would not fit
    const Plan pl = make_plan(c, s, DENSE_F64);
    const int S = pl.S;
    const int E = tri_count(S);
    const SpmmShape sh = pl.sp;
    int64_t nwg = pl.nwg_spmm;
    const int64_t cap = NOALLOC_SCRATCH_DOUBLES / E / 8 * 8;
    if (cap < 1) {
        c.err = "block width too large for the fixed scratch array";
        return MBPCG_ERR_UNSUPPORTED;
    }
    nwg = std::max<int64_t>(1, std::min(nwg, cap));
    if (nwg * E > NOALLOC_SCRATCH_DOUBLES) {
        c.err = "Gram partial sums exceed the fixed scratch array";
        return MBPCG_ERR_UNSUPPORTED;
    }
    // scaling of the matrix (Sec. 1) into the context's buffers, as the
    // allocating entry does
    CK(launch_state_init(c.st, s, 1, 1.0, 1.0, 1e-12, 0, c.stream));
    CK(launch_diag_csr(csr_of(c, false), jacobi, c.d, c.st, c.stream));
    if (jacobi) {
        CK(launch_scale_csr(csr_of(c, false), c.d, c.vals_s, c.stream));
    } else {
        CK(hipMemcpyAsync(c.vals_s, c.vals, sizeof(double) * c.nnz, hipMemcpyDeviceToDevice,
                          c.stream));
    }
    CK(launch_state_init(c.st, s, 1, 1.0, 1.0, 1e-12, 0, c.stream));
    CK(launch_spmm(S, sh, (int)nwg, csr_of(c, true), P, Q, part, c.st, c.stream));
    CK(launch_gram_out(S, (int)nwg, part, C, c.stream));
    CK(hipStreamSynchronize(c.stream));
    return MBPCG_OK;
}

mbpcg_status time_block_product_entry(Ctx& c, int s, int reps, const double* P, double* Q,
                                      double* ms_avg) {
    CK(hipSetDevice(c.device));
    Plan pl = make_plan(c, s, DENSE_F64);
    CKS(ensure_blocks(c, pl.S));
    if (!c.vals_s && !c.dense) CKS(setup_scaling(c, pl, c.bdev, 0));
    if (c.dense && !c.As) c.As = c.A;
    CK(launch_state_init(c.st, s, 1, 1.0, 1.0, 1e-12, 0, c.stream));
    CK(launch_product(c, pl, P, Q, c.part_a, c.st));  // warm-up
    CK(hipEventRecord(c.ev_a, c.stream));
    for (int i = 0; i < reps; ++i) {
        if (!c.dense) {
            CK(launch_spmm(pl.S, pl.sp, pl.nwg_spmm, csr_of(c, true), P, Q, c.part_a, c.st,
                           c.stream));
        } else {
            CK(launch_dense_ap(pl.S, DENSE_F64, c.n, c.As, c.n, nullptr, P, c.qpart, pl.ksplit, c.st,
                               c.stream));
        }
    }
    CK(hipEventRecord(c.ev_b, c.stream));
    CK(hipEventSynchronize(c.ev_b));
    float ms = 0.f;
    CK(hipEventElapsedTime(&ms, c.ev_a, c.ev_b));
    *ms_avg = (double)ms / reps;
    return MBPCG_OK;
}

mbpcg_status tune_entry(Ctx& c, int s, mbpcg_tile_shape* out) {
    CK(hipSetDevice(c.device));
    Plan pl = make_plan(c, s, DENSE_F64);
    const int S = pl.S;
    CKS(ensure_blocks(c, S));
    if (c.dense) {
        if (out) {
            *out = mbpcg_tile_shape{};
            out->tile_rows = 256;
            out->workgroups = pl.nwg_dred;
        }
        return MBPCG_OK;
    }
    if (!c.vals_s) CKS(setup_scaling(c, pl, c.bdev, 1));
    CK(hipMemsetAsync(c.P, 0, sizeof(double) * (size_t)c.n * S, c.stream));
    CK(launch_state_init(c.st, s, 1, 1.0, 1.0, 1e-12, 0, c.stream));
    Tuning best_t{pl.sp, pl.nwg_spmm};
    double best = 1e30;
    const int64_t flush_bytes = 640ll << 20;
    char* flush = nullptr;
    if (hipMalloc(&flush, flush_bytes) != hipSuccess) {
        (void)hipGetLastError();
        c.err = "autotune: no memory for the cache-flush buffer";
        return MBPCG_ERR_OOM;
    }
    struct FlushFree {
        char* p;
        ~FlushFree() { if (p) (void)hipFree(p); }
    } flush_guard{flush};
    CK(hipMemsetAsync(flush, 0, flush_bytes, c.stream));
    SpmmShape shapes[64];
    const int nsh = spmm_shape_list(S, shapes, 64);
    int dev = 0, cus = 0;
    CK(hipGetDevice(&dev));
    CK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    for (int k = 0; k < nsh; ++k) {
        const SpmmShape sh = shapes[k];
        const int64_t tiles = (c.n + sh.T - 1) / sh.T;
        // fixed grids, and the one that fills every CU to the shape's occupancy
        const int resident = spmm_blocks_per_cu(S, sh) * cus;
        for (int w : {512, 1024, 2048, 4096, resident}) {
            if (w <= 0) continue;
            const int nwg = round_grid(std::min<int64_t>(tiles, w), NWG_MAX);
            if (w > 1024 && nwg < w) continue;  // already capped by the tile count
            CK(launch_spmm(S, sh, nwg, csr_of(c, true), c.P, c.Q, c.part_a, c.st, c.stream));
            // In a solve the product follows kernels that stream far more
            // than the 256 MB last-level cache through it, the last of which
            // has just written P; so each timed launch is preceded by a copy
            // of 2 x 320 MB and by a write of the whole P block, and timed
            // alone; the median of 9 such launches counts.
            float t[9];
            for (int r = 0; r < 9; ++r) {
                CK(launch_stream_copy(flush + flush_bytes / 2, flush, flush_bytes / 2, c.stream));
                CK(launch_stream_copy(c.P, c.W, (int64_t)sizeof(double) * c.n * S, c.stream));
                CK(hipEventRecord(c.ev_a, c.stream));
                CK(launch_spmm(S, sh, nwg, csr_of(c, true), c.P, c.Q, c.part_a, c.st, c.stream));
                CK(hipEventRecord(c.ev_b, c.stream));
                CK(hipEventSynchronize(c.ev_b));
                CK(hipEventElapsedTime(&t[r], c.ev_a, c.ev_b));
            }
            std::sort(t, t + 9);
            const double avg = t[4];
            if (avg < best) {
                best = avg;
                best_t = Tuning{sh, nwg};
            }
        }
    }
    c.tune[S] = best_t;
    if (out) {
        *out = mbpcg_tile_shape{};
        out->tile_rows = best_t.sh.T;
        out->lanes_per_row = spmm_lanes_per_row(S, best_t.sh);
        out->cols_per_lane = best_t.sh.V;
        out->loads_in_flight = best_t.sh.U;
        out->waves_per_simd = best_t.sh.W;
        out->workgroups = best_t.nwg;
        out->ms = best;
    }
    return MBPCG_OK;
}

mbpcg_status set_shape_entry(Ctx& c, int s, const mbpcg_tile_shape& t) {
    const int S = padded_width(s);
    if (t.cols_per_lane <= 0 || t.lanes_per_row <= 0) return MBPCG_ERR_UNSUPPORTED;
    SpmmShape sh;
    sh.T = t.tile_rows;
    sh.V = t.cols_per_lane;
    sh.U = t.loads_in_flight;
    sh.W = t.waves_per_simd;
    sh.SL = t.lanes_per_row * t.cols_per_lane / S;
    if (sh.SL * S != t.lanes_per_row * t.cols_per_lane || !spmm_valid_shape(S, sh))
        return MBPCG_ERR_UNSUPPORTED;
    int nwg = 0;
    if (t.workgroups > 0) nwg = std::min(t.workgroups, NWG_MAX);
    c.tune[S] = Tuning{sh, nwg};
    return MBPCG_OK;
}

}  // namespace mb

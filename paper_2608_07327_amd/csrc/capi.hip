// C ABI of the library (include/mbpcg.h).  Arguments are checked here before
// any HIP call; nothing throws across the boundary.
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "runtime.hpp"

namespace mb {
mbpcg_status ctx_init_common(Ctx& c, hipStream_t user_stream);
mbpcg_status solve_entry(Ctx& c, const double* b, double* x, mbpcg_mem mem, const mbpcg_params& p,
                         mbpcg_info& info, int cg);
mbpcg_status block_product_entry(Ctx& c, int s, int jacobi, const double* P, double* Q, double* C);
mbpcg_status block_product_noalloc_entry(Ctx& c, int s, int jacobi, const double* P, double* Q,
                                         double* C);
mbpcg_status time_block_product_entry(Ctx& c, int s, int reps, const double* P, double* Q,
                                      double* ms_avg);
mbpcg_status tune_entry(Ctx& c, int s, mbpcg_tile_shape* out);
mbpcg_status set_shape_entry(Ctx& c, int s, const mbpcg_tile_shape& t);
struct BatchCtx;
BatchCtx* batch_new();
void batch_delete(BatchCtx* c);
const char* batch_error(const BatchCtx* c);
mbpcg_status batch_create(BatchCtx& c, int32_t nsys, const mbpcg_system* systems, mbpcg_mem mem,
                          hipStream_t user_stream);
mbpcg_status batch_solve(BatchCtx& c, const mbpcg_params& p, mbpcg_info* per_system,
                         hipStream_t user_stream, double* kernel_ms);
mbpcg_status batch_tune(BatchCtx& c, const mbpcg_params& p, mbpcg_batch_tuning* out);
mbpcg_status batch_entry(int32_t nsys, const mbpcg_system* systems, const mbpcg_params& common,
                         mbpcg_info* per_system, mbpcg_mem mem, hipStream_t stream,
                         std::string& err);
}  // namespace mb

static thread_local std::string g_create_error;

static mbpcg_status fail_create(const char* msg) {
    g_create_error = msg;
    return MBPCG_ERR_INVALID_ARG;
}

extern "C" {

void mbpcg_default_params(mbpcg_params* p) {
    if (!p) return;
    memset(p, 0, sizeof(*p));
    p->s = 4;
    p->tol = 1e-8;
    p->tol_initial = 0.0;
    p->max_iter = 100000;
    p->precond = MBPCG_PRECOND_JACOBI;
    p->seed = 0;
    p->U = nullptr;
    p->tau = 1e-12;
    p->precision = MBPCG_FP64;
    p->ir_tol = 1e-10;
    p->inner_tol = 5e-6;
    p->max_outer = 50;
    p->history = nullptr;
    p->poll_every = 0;
    p->profile = 0;
    p->block_size = 8;
}

const char* mbpcg_status_str(mbpcg_status st) {
    switch (st) {
        case MBPCG_OK: return "ok";
        case MBPCG_NOT_CONVERGED: return "not converged (iteration cap reached)";
        case MBPCG_ERR_INVALID_ARG: return "invalid argument";
        case MBPCG_ERR_NOT_SPD: return "matrix not symmetric positive definite";
        case MBPCG_ERR_BREAKDOWN: return "block breakdown (all columns dropped)";
        case MBPCG_ERR_NONFINITE: return "non-finite value";
        case MBPCG_ERR_HIP: return "HIP runtime error";
        case MBPCG_ERR_OOM: return "out of device memory";
        case MBPCG_ERR_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char* mbpcg_last_error(mbpcg_ctx ctx) {
    if (!ctx) return g_create_error.c_str();
    return ctx->c.err.c_str();
}

mbpcg_status mbpcg_create_csr(mbpcg_ctx* out, int64_t n, int64_t nnz, const int32_t* rowptr,
                              const int32_t* colind, const double* vals, mbpcg_mem mem,
                              void* hip_stream) {
    if (!out) return fail_create("ctx pointer is NULL");
    *out = nullptr;
    if (n < 1 || n >= (int64_t)INT32_MAX) return fail_create("n must be in [1, 2^31-1)");
    if (nnz < 0 || nnz >= (int64_t)INT32_MAX) return fail_create("nnz must be in [0, 2^31-1)");
    if (!rowptr) return fail_create("rowptr is NULL");
    if (nnz > 0 && (!colind || !vals)) return fail_create("colind/vals are NULL");
    if (mem != MBPCG_MEM_HOST && mem != MBPCG_MEM_DEVICE) return fail_create("bad mem kind");
    if (mem == MBPCG_MEM_HOST) {
        if (rowptr[0] != 0) return fail_create("rowptr[0] must be 0");
        if ((int64_t)rowptr[n] != nnz) return fail_create("rowptr[n] must equal nnz");
        for (int64_t r = 0; r < n; ++r)
            if (rowptr[r + 1] < rowptr[r]) return fail_create("rowptr must be non-decreasing");
        for (int64_t k = 0; k < nnz; ++k) {
            if (colind[k] < 0 || (int64_t)colind[k] >= n) return fail_create("colind out of range");
            if (!std::isfinite(vals[k])) return fail_create("non-finite matrix value");
        }
    }
    mbpcg_ctx h = new (std::nothrow) mbpcg_ctx_s;
    if (!h) return MBPCG_ERR_OOM;
    mb::Ctx& c = h->c;
    c.dense = 0;
    c.n = n;
    c.nnz = nnz;
    mbpcg_status st = mb::ctx_init_common(c, (hipStream_t)hip_stream);
    auto alloc = [&](void** p, size_t bytes) -> mbpcg_status {
        hipError_t e = hipMalloc(p, bytes ? bytes : 16);
        if (e == hipErrorOutOfMemory) return MBPCG_ERR_OOM;
        return e == hipSuccess ? MBPCG_OK : MBPCG_ERR_HIP;
    };
    if (st == MBPCG_OK) st = alloc((void**)&c.rowptr, sizeof(int32_t) * (n + 1));
    if (st == MBPCG_OK) st = alloc((void**)&c.colind, sizeof(int32_t) * nnz);
    if (st == MBPCG_OK) st = alloc((void**)&c.vals, sizeof(double) * nnz);
    // the scaled copy of the values, here rather than at the first solve, so
    // that the allocation-free block product finds it
    if (st == MBPCG_OK) st = alloc((void**)&c.vals_s, sizeof(double) * nnz);
    const hipMemcpyKind kind = mem == MBPCG_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    if (st == MBPCG_OK && hipMemcpy(c.rowptr, rowptr, sizeof(int32_t) * (n + 1), kind) != hipSuccess)
        st = MBPCG_ERR_HIP;
    if (st == MBPCG_OK && nnz > 0 && hipMemcpy(c.colind, colind, sizeof(int32_t) * nnz, kind) != hipSuccess)
        st = MBPCG_ERR_HIP;
    if (st == MBPCG_OK && nnz > 0 && hipMemcpy(c.vals, vals, sizeof(double) * nnz, kind) != hipSuccess)
        st = MBPCG_ERR_HIP;
    if (st != MBPCG_OK) {
        g_create_error = c.err.empty() ? "device allocation or copy failed" : c.err;
        delete h;
        return st;
    }
    *out = h;
    return MBPCG_OK;
}

mbpcg_status mbpcg_create_dense(mbpcg_ctx* out, int64_t n, const double* A, int64_t lda,
                                mbpcg_mem mem, void* hip_stream) {
    if (!out) return fail_create("ctx pointer is NULL");
    *out = nullptr;
    if (n < 1 || n > (int64_t)1 << 20) return fail_create("n must be in [1, 2^20]");
    if (lda < n) return fail_create("lda must be >= n");
    if (!A) return fail_create("A is NULL");
    if (mem != MBPCG_MEM_HOST && mem != MBPCG_MEM_DEVICE) return fail_create("bad mem kind");
    mbpcg_ctx h = new (std::nothrow) mbpcg_ctx_s;
    if (!h) return MBPCG_ERR_OOM;
    mb::Ctx& c = h->c;
    c.dense = 1;
    c.n = n;
    c.nnz = n * n;
    mbpcg_status st = mb::ctx_init_common(c, (hipStream_t)hip_stream);
    if (st == MBPCG_OK) {
        hipError_t e = hipMalloc((void**)&c.A, sizeof(double) * (size_t)n * n);
        if (e != hipSuccess) st = e == hipErrorOutOfMemory ? MBPCG_ERR_OOM : MBPCG_ERR_HIP;
    }
    if (st == MBPCG_OK) {
        const hipMemcpyKind kind =
            mem == MBPCG_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
        if (hipMemcpy2D(c.A, sizeof(double) * n, A, sizeof(double) * lda, sizeof(double) * n, n,
                        kind) != hipSuccess)
            st = MBPCG_ERR_HIP;
    }
    if (st != MBPCG_OK) {
        g_create_error = c.err.empty() ? "device allocation or copy failed" : c.err;
        delete h;
        return st;
    }
    c.As = c.A;
    *out = h;
    return MBPCG_OK;
}

static mbpcg_status check_params(mbpcg_ctx ctx, const double* b, double* x, mbpcg_mem mem,
                                 const mbpcg_params* p, int cg) {
    if (!ctx || !b || !x || !p) return MBPCG_ERR_INVALID_ARG;
    if (mem != MBPCG_MEM_HOST && mem != MBPCG_MEM_DEVICE) return MBPCG_ERR_INVALID_ARG;
    if (!(p->tol > 0.0) || !std::isfinite(p->tol)) return MBPCG_ERR_INVALID_ARG;
    if (p->max_iter < 1 || p->max_iter > (int64_t)INT32_MAX) return MBPCG_ERR_INVALID_ARG;
    if (p->precond != MBPCG_PRECOND_NONE && p->precond != MBPCG_PRECOND_JACOBI &&
        p->precond != MBPCG_PRECOND_BLOCK_JACOBI)
        return MBPCG_ERR_INVALID_ARG;
    if (p->precond == MBPCG_PRECOND_BLOCK_JACOBI && !mb::bjac_supported(p->block_size))
        return MBPCG_ERR_INVALID_ARG;
    if (p->poll_every < 0 || p->poll_every > 4096) return MBPCG_ERR_INVALID_ARG;
    if (cg) return MBPCG_OK;
    if (p->s < 1) return MBPCG_ERR_INVALID_ARG;
    if (p->s > 32) return MBPCG_ERR_UNSUPPORTED;
    if (!std::isfinite(p->tol_initial) || !std::isfinite(p->tau)) return MBPCG_ERR_INVALID_ARG;
    if (p->precision != MBPCG_FP64 && p->precision != MBPCG_FP32_IR &&
        p->precision != MBPCG_BF16_IR)
        return MBPCG_ERR_INVALID_ARG;
    if (p->precision != MBPCG_FP64) {
        if (!ctx->c.dense) return MBPCG_ERR_UNSUPPORTED;
        if (p->precond == MBPCG_PRECOND_BLOCK_JACOBI) return MBPCG_ERR_UNSUPPORTED;
        if (!(p->ir_tol > 0.0) || !(p->inner_tol > 0.0) || p->max_outer < 0)
            return MBPCG_ERR_INVALID_ARG;
    }
    return MBPCG_OK;
}

static void zero_info(mbpcg_info* info) {
    if (info) memset(info, 0, sizeof(*info));
}

mbpcg_status mbpcg_solve(mbpcg_ctx ctx, const double* b, double* x, mbpcg_mem mem,
                         const mbpcg_params* params, mbpcg_info* info) {
    mbpcg_status v = check_params(ctx, b, x, mem, params, 0);
    if (v != MBPCG_OK) {
        if (ctx) ctx->c.err = "invalid or unsupported parameters";
        return v;
    }
    mbpcg_info local;
    zero_info(&local);
    mbpcg_status st = mb::solve_entry(ctx->c, b, x, mem, *params, local, 0);
    local.status = st;
    if (info) *info = local;
    return st;
}

mbpcg_status mbpcg_cg_solve(mbpcg_ctx ctx, const double* b, double* x, mbpcg_mem mem,
                            const mbpcg_params* params, mbpcg_info* info) {
    mbpcg_status v = check_params(ctx, b, x, mem, params, 1);
    if (v != MBPCG_OK) {
        if (ctx) ctx->c.err = "invalid parameters";
        return v;
    }
    mbpcg_info local;
    zero_info(&local);
    mbpcg_status st = mb::solve_entry(ctx->c, b, x, mem, *params, local, 1);
    local.status = st;
    if (info) *info = local;
    return st;
}

static bool pow2_width(int s) { return s == 1 || s == 2 || s == 4 || s == 8 || s == 16 || s == 32; }

mbpcg_status mbpcg_block_product(mbpcg_ctx ctx, int32_t s, mbpcg_precond precond, const double* P,
                                 double* Q, double* C) {
    if (!ctx || !P || !Q || !C) return MBPCG_ERR_INVALID_ARG;
    if (!pow2_width(s)) return MBPCG_ERR_UNSUPPORTED;
    if (precond != MBPCG_PRECOND_NONE && precond != MBPCG_PRECOND_JACOBI) return MBPCG_ERR_INVALID_ARG;
    return mb::block_product_entry(ctx->c, s, precond == MBPCG_PRECOND_JACOBI, P, Q, C);
}

mbpcg_status mbpcg_block_product_noalloc(mbpcg_ctx ctx, int32_t s, mbpcg_precond precond,
                                         const double* P, double* Q, double* C) {
    if (!ctx || !P || !Q || !C) return MBPCG_ERR_INVALID_ARG;
    if (!pow2_width(s)) return MBPCG_ERR_UNSUPPORTED;
    if (precond != MBPCG_PRECOND_NONE && precond != MBPCG_PRECOND_JACOBI) return MBPCG_ERR_INVALID_ARG;
    return mb::block_product_noalloc_entry(ctx->c, s, precond == MBPCG_PRECOND_JACOBI, P, Q, C);
}

mbpcg_status mbpcg_time_block_product(mbpcg_ctx ctx, int32_t s, int32_t reps, const double* P,
                                      double* Q, double* ms_avg) {
    if (!ctx || !P || !Q || !ms_avg || reps < 1) return MBPCG_ERR_INVALID_ARG;
    if (!pow2_width(s)) return MBPCG_ERR_UNSUPPORTED;
    return mb::time_block_product_entry(ctx->c, s, reps, P, Q, ms_avg);
}

mbpcg_status mbpcg_autotune(mbpcg_ctx ctx, int32_t s, mbpcg_tile_shape* best) {
    if (!ctx) return MBPCG_ERR_INVALID_ARG;
    if (!pow2_width(s)) return MBPCG_ERR_UNSUPPORTED;
    mbpcg_tile_shape t{};
    mbpcg_status st = mb::tune_entry(ctx->c, s, &t);
    if (st != MBPCG_OK) return st;
    if (best) *best = t;
    return MBPCG_OK;
}

mbpcg_status mbpcg_tile_shapes(int32_t s, mbpcg_tile_shape* out, int32_t cap, int32_t* count) {
    if (!pow2_width(s) || cap < 0 || (cap > 0 && !out)) return s < 1 ? MBPCG_ERR_INVALID_ARG
                                                                    : MBPCG_ERR_UNSUPPORTED;
    mb::SpmmShape sh[64];
    const int k = mb::spmm_shape_list(s, sh, 64);
    for (int i = 0; i < k && i < cap; ++i) {
        out[i] = mbpcg_tile_shape{};
        out[i].tile_rows = sh[i].T;
        out[i].lanes_per_row = mb::spmm_lanes_per_row(s, sh[i]);
        out[i].cols_per_lane = sh[i].V;
        out[i].loads_in_flight = sh[i].U;
        out[i].waves_per_simd = sh[i].W;
    }
    if (count) *count = k;
    return MBPCG_OK;
}

mbpcg_status mbpcg_set_tile_shape(mbpcg_ctx ctx, int32_t s, const mbpcg_tile_shape* shape) {
    if (!ctx || !shape) return MBPCG_ERR_INVALID_ARG;
    if (!pow2_width(s)) return MBPCG_ERR_UNSUPPORTED;
    return mb::set_shape_entry(ctx->c, s, *shape);
}

static mbpcg_status check_batch_params(const mbpcg_params* common) {
    if (!common) return MBPCG_ERR_INVALID_ARG;
    if (!(common->tol > 0.0) || !std::isfinite(common->tol) || common->max_iter < 1 ||
        common->max_iter > (int64_t)INT32_MAX)
        return MBPCG_ERR_INVALID_ARG;
    if (common->precond != MBPCG_PRECOND_NONE && common->precond != MBPCG_PRECOND_JACOBI &&
        common->precond != MBPCG_PRECOND_BLOCK_JACOBI)
        return MBPCG_ERR_INVALID_ARG;
    if (!std::isfinite(common->tol_initial) || !std::isfinite(common->tau))
        return MBPCG_ERR_INVALID_ARG;
    if (common->precision != MBPCG_FP64 && common->precision != MBPCG_FP32_IR &&
        common->precision != MBPCG_BF16_IR)
        return MBPCG_ERR_INVALID_ARG;
    // the batched kernel runs the FP64 method with diagonal scaling or none,
    // and the paper's setting of equal tolerances
    if (common->precond == MBPCG_PRECOND_BLOCK_JACOBI) return MBPCG_ERR_UNSUPPORTED;
    if (common->precision != MBPCG_FP64) return MBPCG_ERR_UNSUPPORTED;
    if (common->tol_initial > 0.0 && common->tol_initial != common->tol)
        return MBPCG_ERR_UNSUPPORTED;
    return MBPCG_OK;
}

static mbpcg_status check_batch_systems(int32_t nsys, const mbpcg_system* systems,
                                        mbpcg_mem mem) {
    if (nsys < 1 || !systems) return MBPCG_ERR_INVALID_ARG;
    if (mem != MBPCG_MEM_HOST && mem != MBPCG_MEM_DEVICE) return MBPCG_ERR_INVALID_ARG;
    for (int32_t i = 0; i < nsys; ++i) {
        const mbpcg_system& y = systems[i];
        if (y.n < 1 || y.n >= (int64_t)INT32_MAX || y.nnz < 0 || y.nnz >= (int64_t)INT32_MAX)
            return MBPCG_ERR_INVALID_ARG;
        if (!y.rowptr || !y.b || !y.x || (y.nnz > 0 && (!y.colind || !y.vals)))
            return MBPCG_ERR_INVALID_ARG;
        if (y.s < 1) return MBPCG_ERR_INVALID_ARG;
        if (y.s > 8) return MBPCG_ERR_UNSUPPORTED;
        if (mem == MBPCG_MEM_HOST) {
            if (y.rowptr[0] != 0 || (int64_t)y.rowptr[y.n] != y.nnz) return MBPCG_ERR_INVALID_ARG;
            for (int64_t r = 0; r < y.n; ++r)
                if (y.rowptr[r + 1] < y.rowptr[r]) return MBPCG_ERR_INVALID_ARG;
            for (int64_t k = 0; k < y.nnz; ++k)
                if (y.colind[k] < 0 || (int64_t)y.colind[k] >= y.n) return MBPCG_ERR_INVALID_ARG;
        }
    }
    return MBPCG_OK;
}

mbpcg_status mbpcg_solve_batch(int32_t nsys, const mbpcg_system* systems,
                               const mbpcg_params* common, mbpcg_info* per_system, mbpcg_mem mem,
                               void* hip_stream) {
    if (nsys < 1 || !systems || !common) return MBPCG_ERR_INVALID_ARG;
    if (mem != MBPCG_MEM_HOST && mem != MBPCG_MEM_DEVICE) return MBPCG_ERR_INVALID_ARG;
    mbpcg_status v = check_batch_params(common);
    if (v == MBPCG_OK) v = check_batch_systems(nsys, systems, mem);
    if (v != MBPCG_OK) return v;
    std::string err;
    mbpcg_status st = mb::batch_entry(nsys, systems, *common, per_system, mem,
                                      (hipStream_t)hip_stream, err);
    if (st != MBPCG_OK) g_create_error = err;
    return st;
}

struct mbpcg_batch_s {
    mb::BatchCtx* c = nullptr;
    ~mbpcg_batch_s() { mb::batch_delete(c); }
};

mbpcg_status mbpcg_batch_create(mbpcg_batch* out, int32_t nsys, const mbpcg_system* systems,
                                mbpcg_mem mem, void* hip_stream) {
    if (!out) return MBPCG_ERR_INVALID_ARG;
    *out = nullptr;
    mbpcg_status v = check_batch_systems(nsys, systems, mem);
    if (v != MBPCG_OK) return v;
    mbpcg_batch h = new (std::nothrow) mbpcg_batch_s;
    if (!h) return MBPCG_ERR_OOM;
    h->c = mb::batch_new();
    if (!h->c) {
        delete h;
        return MBPCG_ERR_OOM;
    }
    const mbpcg_status st = mb::batch_create(*h->c, nsys, systems, mem, (hipStream_t)hip_stream);
    if (st != MBPCG_OK) {
        g_create_error = mb::batch_error(h->c);
        delete h;
        return st;
    }
    *out = h;
    return MBPCG_OK;
}

mbpcg_status mbpcg_batch_solve(mbpcg_batch batch, const mbpcg_params* common,
                               mbpcg_info* per_system, void* hip_stream) {
    if (!batch || !common) return MBPCG_ERR_INVALID_ARG;
    mbpcg_status v = check_batch_params(common);
    if (v != MBPCG_OK) return v;
    const mbpcg_status st = mb::batch_solve(*batch->c, *common, per_system,
                                            (hipStream_t)hip_stream, nullptr);
    if (st != MBPCG_OK) g_create_error = mb::batch_error(batch->c);
    return st;
}

mbpcg_status mbpcg_batch_autotune(mbpcg_batch batch, const mbpcg_params* common,
                                  mbpcg_batch_tuning* out) {
    if (!batch || !common) return MBPCG_ERR_INVALID_ARG;
    mbpcg_status v = check_batch_params(common);
    if (v != MBPCG_OK) return v;
    const mbpcg_status st = mb::batch_tune(*batch->c, *common, out);
    if (st != MBPCG_OK) g_create_error = mb::batch_error(batch->c);
    return st;
}

void mbpcg_batch_destroy(mbpcg_batch batch) { delete batch; }

mbpcg_status mbpcg_stream_copy(void* dst, const void* src, int64_t bytes, void* hip_stream) {
    if (!dst || !src || bytes < 0) return MBPCG_ERR_INVALID_ARG;
    if (bytes == 0) return MBPCG_OK;
    hipError_t e = mb::launch_stream_copy(dst, src, bytes, (hipStream_t)hip_stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)hip_stream);
    return e == hipSuccess ? MBPCG_OK : MBPCG_ERR_HIP;
}

void mbpcg_destroy(mbpcg_ctx ctx) { delete ctx; }

}  // extern "C"

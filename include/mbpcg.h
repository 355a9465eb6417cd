/*
 * mbpcg — Multi-Basis Parallel Conjugate Gradient on AMD Instinct MI355X (gfx950).
 *
 * The method (Xu & Regev, arXiv 2608.07327, Sec. 2, Algorithm 1) solves one
 * symmetric positive definite system A x = b by running Dubrulle-R block CG
 * on s duplicate copies of it, B = [b ... b], each copy started from its own
 * random initial guess, and returns the least-squares combination of the s
 * iterates (Proposition 1 gives A X = B - R, so no extra product is needed).
 *
 * Conventions of this interface
 *   - Every function returns an mbpcg_status; nothing throws across it.
 *   - Matrices are FP64.  Sparse A is CSR with int32 indices (Sec. 3: CSR for
 *     sparse, column-major for dense).  Dense A is column-major with leading
 *     dimension lda >= n.
 *   - Vectors b and x have length n.  `mem` says whether a pointer is host or
 *     device memory of the current HIP device.
 *   - A context copies A into memory it owns; the caller keeps ownership of
 *     every pointer it passes.  x is written in place.
 *   - A context is bound to one HIP stream and is not thread safe.  Work is
 *     queued on that stream; solve calls return after the result is in x.
 *   - Argument checks (sizes, CSR structure when A is on the host, finite
 *     parameters) run before any HIP call: INVALID_ARG never touches the GPU.
 *   - After any status other than INVALID_ARG, *info is filled and x holds the
 *     best iterate available.
 */
#ifndef MBPCG_H
#define MBPCG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mbpcg_ctx_s* mbpcg_ctx;

typedef enum {
    MBPCG_OK = 0,
    MBPCG_NOT_CONVERGED = 1,     /* max_iter reached; x = best column X_h       */
    MBPCG_ERR_INVALID_ARG = -1,
    MBPCG_ERR_NOT_SPD = -2,      /* a_jj <= 0 under Jacobi, or P^T A P not SPD */
    MBPCG_ERR_BREAKDOWN = -3,    /* every column dropped before convergence     */
    MBPCG_ERR_NONFINITE = -4,    /* NaN/Inf in the input or the iteration       */
    MBPCG_ERR_HIP = -5,          /* a HIP runtime call failed (see last_error)  */
    MBPCG_ERR_OOM = -6,
    MBPCG_ERR_UNSUPPORTED = -7   /* e.g. s > 32, or a mode the library lacks    */
} mbpcg_status;

/* NONE: A as given.  JACOBI: the symmetric diagonal scaling of Sec. 1.
 * BLOCK_JACOBI: that scaling, then the block-Jacobi preconditioner M (the
 * diagonal blocks of block_size consecutive rows of the scaled matrix, the
 * last block shorter when block_size does not divide n) in the
 * preconditioned form of the method that Sec. 2 says it admits: the residual
 * basis is orthonormal in the M^-1 inner product (Cholesky QR of V^T M^-1 V)
 * and the directions are built from M^-1 W.  FP64 single-system solves and
 * the CG baseline only. */
typedef enum {
    MBPCG_PRECOND_NONE = 0,
    MBPCG_PRECOND_JACOBI = 1,
    MBPCG_PRECOND_BLOCK_JACOBI = 2
} mbpcg_precond;

/* Arithmetic of the block product A P.  FP64 everywhere is the paper's
 * (Sec. 3).  The two IR modes round a copy of dense A to FP32 or BF16, run the
 * inner block CG with that copy on the matrix cores (FP32 accumulation) and
 * correct in an FP64 iterative-refinement loop with FP64 residuals; the s x s
 * Cholesky, deflation and all other work stay FP64. */
typedef enum { MBPCG_FP64 = 0, MBPCG_FP32_IR = 1, MBPCG_BF16_IR = 2 } mbpcg_precision;

typedef enum { MBPCG_MEM_HOST = 0, MBPCG_MEM_DEVICE = 1 } mbpcg_mem;

typedef struct {
    int32_t s;              /* copies (block width), 1..32                               */
    double tol;             /* convergence tolerance on ||b - A x|| / ||b|| (Alg. 1)     */
    double tol_initial;     /* best-column tolerance of Alg. 1's first stop test; <= 0   */
                            /* means tol (the paper's setting).  Once the best column's  */
                            /* residual is below it, the least-squares combination is   */
                            /* tried every iteration and the solve ends when that meets  */
                            /* tol or the best column does (Alg. 1's second test).       */
                            /* Single-system FP64 solves; IR inner solves and batches    */
                            /* use tol (a batch with tol_initial != tol: UNSUPPORTED)    */
    int64_t max_iter;       /* iteration cap (inner cap in IR mode)                      */
    mbpcg_precond precond;  /* NONE, JACOBI (Sec. 1 scaling) or BLOCK_JACOBI (above)     */
    uint64_t seed;          /* SplitMix64 seed of the Uniform(-1,1) initial block         */
    const double* U;        /* optional n x s row-major initial block, same mem as b     */
    double tau;             /* deflation threshold of Cholesky QR; <= 0 means 1e-12      */
    mbpcg_precision precision;
    double ir_tol;          /* IR: outer tolerance (FP64 residual)                       */
    double inner_tol;       /* IR: tightest relative tolerance of an inner solve; each   */
                            /* inner solve asks only for 0.5 ir_tol / (current outer     */
                            /* residual), clamped to [inner_tol, 0.1]                    */
    int32_t max_outer;      /* IR: outer iteration cap                                   */
    double* history;        /* optional host array [max_iter]: ||R_h|| / ||b|| per step  */
    int32_t poll_every;     /* iterations per graph launch between host checks; 0 = auto */
    int32_t profile;        /* 1: time each phase with HIP events (no graphs); 2: time
                               only the block product (two events per iteration)       */
    int32_t block_size;     /* BLOCK_JACOBI: rows per diagonal block, 4, 8, 16 or 32     */
    double* X_out;          /* optional n x s row-major, same memory kind as b: the block */
                            /* iterate X = X~ + X0 at exit in the scaled space (Sec. 1), */
                            /* for parity checks; FP64 solves only (ignored in IR mode)  */
} mbpcg_params;

typedef struct {
    int64_t iterations;        /* inner block steps (summed over IR outer steps)       */
    int64_t outer_iterations;  /* IR outer steps (0 in FP64 mode)                      */
    int32_t best_column;       /* h of Alg. 1 at exit                                  */
    int32_t final_width;       /* columns left after deflation                         */
    int32_t deflations;        /* columns dropped by Cholesky QR                       */
    int32_t used_fallback;     /* 1: x is the best column, not the LS combination:     */
                               /* the combination was not finite, missed the tolerance */
                               /* on B^ c, or (FP64 solves) missed it on its true       */
                               /* residual while the best column's true residual was    */
                               /* lower (its coefficients can amplify the rounding      */
                               /* drift between A X and B - R of Proposition 1)         */
    double rel_res_best_basis; /* ||R_h|| / ||b|| at exit                              */
    double rel_res_ls;         /* ||b - B^ c|| / ||b|| of the LS combination           */
    double rel_res_true;       /* ||b - A x|| / ||b|| recomputed in FP64 on A          */
    double ms_total;           /* wall time of the solve (scaling included, Sec. 4)    */
    double ms_per_iter;        /* loop time / iterations                               */
    double ms_spmm;            /* profile mode: summed time of the block product       */
    int64_t spmm_launches;     /* profile mode: number of block-product launches       */
    double ms_phase[8];        /* profile mode: product, Xi, updates, QR, P, LS, setup, other;
                                  a batch reports the whole batch's phases (other =
                                  kernel time outside them, or the kernel time when
                                  not profiling) */
    int32_t status;            /* mbpcg_status of this solve (per system in a batch)   */
    int32_t reserved;
} mbpcg_info;

/* Fill *p with defaults: s=4, tol=1e-8, tol_initial=0, max_iter=100000,
 * JACOBI, seed=0, tau=1e-12, FP64, ir_tol=1e-10, inner_tol=5e-6, max_outer=50. */
void mbpcg_default_params(mbpcg_params* p);

/* Create a context for sparse A (CSR, FP64 values, int32 rowptr[n+1] and
 * colind[nnz], columns in any order inside a row).  A is copied. */
mbpcg_status mbpcg_create_csr(mbpcg_ctx* ctx, int64_t n, int64_t nnz,
                              const int32_t* rowptr, const int32_t* colind,
                              const double* vals, mbpcg_mem mem, void* hip_stream);

/* Create a context for dense A (column-major n x n, leading dimension lda).
 * A is copied.  Sec. 3 stores dense A column-major. */
mbpcg_status mbpcg_create_dense(mbpcg_ctx* ctx, int64_t n, const double* A, int64_t lda,
                                mbpcg_mem mem, void* hip_stream);

/* Solve A x = b with Algorithm 1 (MBPCG). */
mbpcg_status mbpcg_solve(mbpcg_ctx ctx, const double* b, double* x, mbpcg_mem mem,
                         const mbpcg_params* params, mbpcg_info* info);

/* Solve A x = b with Chronopoulos-Gear CG from x0 = 0, on the same scaled
 * system and with the same stop rule: the paper's CG baseline (Sec. 1, Sec. 4). */
mbpcg_status mbpcg_cg_solve(mbpcg_ctx ctx, const double* b, double* x, mbpcg_mem mem,
                            const mbpcg_params* params, mbpcg_info* info);

/* One block product of the solver's hot loop, exposed for testing and
 * measurement: Q = A~ P and C = P^T Q for the scaled matrix A~ = D^-1 A D^-1
 * (D = I with precond NONE), P and Q row-major n x s on the device, C row-major
 * s x s on the device (lower triangle i >= j written; upper left untouched).
 * This is the A P and P^T A P of Alg. 1. */
mbpcg_status mbpcg_block_product(mbpcg_ctx ctx, int32_t s, mbpcg_precond precond,
                                 const double* P, double* Q, double* C);

/* mbpcg_block_product without any allocation, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, arithmetic and results
 * (Q bitwise; C bitwise when the grid below is not lowered).  CSR contexts
 * only (MBPCG_ERR_UNSUPPORTED for dense ones).  The Gram's per-workgroup
 * partial sums go to a fixed 4 MiB device array, one per GPU, held until the
 * process ends; the product's grid is lowered where needed so that they fit
 * (at most 992 workgroups at s = 32), and a call whose partials would not fit
 * returns MBPCG_ERR_UNSUPPORTED with mbpcg_last_error set.  Every call on a
 * GPU shares that GPU's array: calls that overlap on one GPU race (serialise
 * them).  The context's own buffers (scaling, state) are allocated by
 * mbpcg_create_csr. */
mbpcg_status mbpcg_block_product_noalloc(mbpcg_ctx ctx, int32_t s, mbpcg_precond precond,
                                         const double* P, double* Q, double* C);

/* Time `reps` launches of the block-product kernel of mbpcg_block_product with
 * HIP events on the context's stream; *ms_avg receives the mean duration. */
mbpcg_status mbpcg_time_block_product(mbpcg_ctx ctx, int32_t s, int32_t reps,
                                      const double* P, double* Q, double* ms_avg);

/* Tile shape of the sparse block product, as chosen by mbpcg_autotune. */
typedef struct {
    int32_t tile_rows;       /* rows of A per tile; the tile's CSR slice is staged in LDS */
    int32_t lanes_per_row;   /* lanes sharing one row of A */
    int32_t cols_per_lane;   /* adjacent columns of P one lane gathers per nonzero (1, 2, 4) */
    int32_t loads_in_flight; /* gathers a lane issues before it consumes the first */
    int32_t workgroups;      /* grid of the block-product kernel */
    int32_t waves_per_simd;  /* occupancy the kernel was compiled for (0: compiler's choice) */
    double ms;               /* mean duration of one block product with this shape */
} mbpcg_tile_shape;

/* Autotune the block product Q = A~ P, C = P^T Q of this context (the A P of
 * Alg. 1) for block width s (1, 2, 4, 8, 16 or 32): every compiled tile shape
 * and grid size is timed with HIP events on the context's stream and the
 * fastest is kept for later solves of this width.  Dense contexts keep their
 * fixed tiling (tile_rows = 256, other fields 0).  best may be NULL. */
mbpcg_status mbpcg_autotune(mbpcg_ctx ctx, int32_t s, mbpcg_tile_shape* best);

/* The compiled tile shapes of the sparse block product for width s: writes
 * up to cap of them (workgroups = 0, ms = 0) and their total number to
 * *count.  Needs no GPU. */
mbpcg_status mbpcg_tile_shapes(int32_t s, mbpcg_tile_shape* out, int32_t cap, int32_t* count);

/* Fix the block-product tile shape of this context for width s, as if
 * mbpcg_autotune had chosen it: tile_rows, lanes_per_row, cols_per_lane and
 * loads_in_flight must name a compiled shape (MBPCG_ERR_UNSUPPORTED
 * otherwise); workgroups <= 0 selects the default grid.  Ignored by dense
 * contexts. */
mbpcg_status mbpcg_set_tile_shape(mbpcg_ctx ctx, int32_t s, const mbpcg_tile_shape* shape);

/* One independent system of a batch; pointers as given by `mem`. */
typedef struct {
    int64_t n, nnz;
    const int32_t* rowptr;
    const int32_t* colind;
    const double* vals;
    const double* b;
    double* x;
    int32_t s;   /* block width of this system, 1..8 */
} mbpcg_system;

/* Solve nsys independent sparse systems (uneven n and s) together in one
 * persistent launch per graph replay.  common->s is ignored; each system uses
 * its own s.  per_system[nsys] receives each system's info.  The call returns
 * when the batch has finished; concurrent calls from several threads of one
 * process run one after the other (the kernel's arguments live in one
 * device symbol). */
mbpcg_status mbpcg_solve_batch(int32_t nsys, const mbpcg_system* systems,
                               const mbpcg_params* common, mbpcg_info* per_system,
                               mbpcg_mem mem, void* hip_stream);

/* A batch context: the systems of mbpcg_solve_batch uploaded once (CSR and b
 * copied into library-owned device memory; the caller's x pointers receive
 * each solve's results), with the persistent kernel captured in a HIP graph
 * that every solve replays.  mbpcg_solve_batch is create + solve + destroy.
 * Validation as in mbpcg_solve_batch; errors: mbpcg_last_error(NULL). */
typedef struct mbpcg_batch_s* mbpcg_batch;

mbpcg_status mbpcg_batch_create(mbpcg_batch* batch, int32_t nsys, const mbpcg_system* systems,
                                mbpcg_mem mem, void* hip_stream);

/* Solve every system of the batch with parameters `common` (as in
 * mbpcg_solve_batch), writing x through the pointers given at create and
 * per_system[nsys] (may be NULL).  Returns when the batch has finished.
 * The persistent kernel's grid barrier waits at most 2^24 polls (the
 * environment variable MBPCG_BATCH_SPIN_LIMIT, a positive integer, lowers
 * the bound; tests use it to reach this path): a longer wait makes every
 * workgroup exit and the call return MBPCG_ERR_HIP with mbpcg_last_error
 * set, and the next solve starts afresh. */
mbpcg_status mbpcg_batch_solve(mbpcg_batch batch, const mbpcg_params* common,
                               mbpcg_info* per_system, void* hip_stream);

/* Result of mbpcg_batch_autotune. */
typedef struct {
    int32_t workgroups;        /* grid of the persistent kernel chosen                   */
    int32_t classes;           /* (block width, row-length class) pairs in the batch     */
    int32_t two_slot_classes;  /* classes given two lane groups per row                  */
    int32_t trials;            /* timed trial solves run                                 */
    double ms;                 /* kernel time of the best trial (capped at 12 iterations) */
} mbpcg_batch_tuning;

/* Choose the batched kernel's free parameters by timed trials (solves capped
 * at 12 iterations, which overwrite x): lane groups per CSR row for each
 * (padded width, row-length class) of the batch -- [0, 16), [16, 48), 48 or
 * more nonzeros per row -- and the grid (all co-resident workgroups, 3/4,
 * 1/2).  The per-class choice is kept for the process: a later batch whose
 * classes are all known skips those trials.  Later solves of this batch use
 * the choice. */
mbpcg_status mbpcg_batch_autotune(mbpcg_batch batch, const mbpcg_params* common,
                                  mbpcg_batch_tuning* out);

void mbpcg_batch_destroy(mbpcg_batch batch);

/* Copy `bytes` bytes device-to-device with the library's plain streaming copy
 * kernel on `hip_stream`; used to calibrate hardware byte counters. */
mbpcg_status mbpcg_stream_copy(void* dst, const void* src, int64_t bytes, void* hip_stream);

void mbpcg_destroy(mbpcg_ctx ctx);
const char* mbpcg_status_str(mbpcg_status st);
/* Message of the last failure on ctx (ctx may be NULL for create failures). */
const char* mbpcg_last_error(mbpcg_ctx ctx);

#ifdef __cplusplus
}
#endif
#endif

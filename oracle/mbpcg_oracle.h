/*
 * CPU oracle of Multi-Basis Parallel CG (Xu & Regev, arXiv 2608.07327).
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, single-threaded, FP64 C with sequential
 * sums (or, on request, a blocked-pairwise order used to measure the
 * rounding-order noise floor).  It shares no code, header or constant with
 * the GPU library; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark may call it.
 *
 * Blocks (n x k) are row-major: element (r, j) at X[r*k + j].
 * Dense matrices are column-major: element (r, c) at a[c*lda + r].
 * Small k x k matrices are row-major.
 */
#ifndef MBPCG_ORACLE_H
#define MBPCG_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int64_t n;
    int dense;                 /* 0: CSR, 1: dense column-major */
    const int32_t* rowptr;     /* CSR */
    const int32_t* colind;
    const double* vals;
    const double* a;           /* dense */
    int64_t lda;
    int lo;                    /* dense products in low precision (mixed-precision
                                  extension): 0 FP64, 1 FP32, 2 BF16 -- A and X
                                  rounded to nearest even, products accumulated
                                  in FP32 in column order.  CSR ignores it. */
} or_matrix;

enum {
    OR_OK = 0, OR_NOT_CONVERGED = 1, OR_ERR_NOT_SPD = -2, OR_ERR_BREAKDOWN = -3,
    OR_ERR_NONFINITE = -4
};

typedef struct {
    int s;                /* number of duplicate copies (block width) */
    double tol;           /* convergence tolerance on ||b - A x|| / ||b|| */
    double tol_initial;   /* tolerance of the best column; <= 0 means = tol */
    int64_t max_iter;
    int jacobi;           /* 1: symmetric diagonal scaling D = diag(sqrt(a_jj)) */
    uint64_t seed;        /* SplitMix64 seed of the random initial block */
    const double* U;      /* optional explicit n x s initial block (overrides seed) */
    double tau;           /* Cholesky-QR deflation threshold (relative) */
    int ls_scaled;        /* 1: stop test and least squares in the scaled space */
    double* history;      /* optional [max_iter]: ||R_h|| / ||b|| after each iteration */
    double* X_out;        /* optional n x s: X = X~ + X0 at exit (scaled space) */
    double* R_out;        /* optional n x s: R at exit (scaled space) */
    double* prop1_gap;    /* optional [max_iter]: ||A X - (B - R)||_F / ||B||_F (scaled) */
    int check_true;       /* 1: an accepted combination whose true residual is not below
                             tol gives way to the best column when that column's true
                             residual is lower (the fallback after Proposition 1) */
    int bj_block;         /* >= 2: block-Jacobi preconditioner with blocks of bj_block
                             consecutive rows of the (scaled) matrix, in the
                             preconditioned Dubrulle-R form; < 2: none */
} or_params;

typedef struct {
    int status;
    int64_t iterations;
    int best_column;
    int final_width;
    int deflations;
    int used_fallback;
    double rel_res_best;  /* ||R_h|| / ||b|| at exit */
    double rel_res_ls;    /* ||b - B^ c|| / ||b|| of the least-squares combination */
    double rel_res_true;  /* ||b - A x|| / ||b|| recomputed on the original A */
    double seconds;       /* wall time of scaling + setup + loop + termination */
    double seconds_setup; /* scaling + random block + first QR */
    int ls_kept;          /* columns the least squares kept (s when none was left out) */
} or_info;

/* summation order of every reduction over n: 0 sequential, 1 blocked pairwise */
void or_set_summation(int mode);

/* SplitMix64 output number k (k = 0, 1, ...) of the stream seeded with seed */
uint64_t or_splitmix64(uint64_t seed, uint64_t k);
/* U[r*s + j] = 2 * u - 1, u = (splitmix64(seed, j*n + r) >> 11) * 2^-53 */
void or_uniform_block(uint64_t seed, int64_t n, int s, double* U);

/* x rounded to the nearest BF16 value (ties to even), returned as a double */
double or_round_bf16(double x);

/* Y = A X for an n x k block */
void or_matmul_block(const or_matrix* A, int k, const double* X, double* Y);
/* C (k1 x k2) = X^T Y for blocks X (n x k1), Y (n x k2) */
void or_gram(int64_t n, int k1, const double* X, int k2, const double* Y, double* C);
/* lower Cholesky C = L L^T from the lower triangle of C (m x m); 0 ok, -1 fail */
int or_cholesky(int m, const double* C, double* L);
/* Xi = (L L^T)^{-1} by solving against the identity */
void or_spd_inverse(int m, const double* L, double* Xi);
/* Cholesky QR with column dropping.  V is n x m.  On return W (n x m_out,
 * row-major with row stride m_out), Z (m_out x m), keep[m] (1 kept), and the
 * width m_out.  W and Z must hold n*m and m*m doubles. */
int or_cholqr_deflate(int64_t n, int m, const double* V, double tau,
                      double* W, double* Z, int* keep);
/* Cholesky QR in the M^-1 inner product: Gram V^T Y (Y = M^-1 V; entry
 * (i > j) taken as V_i^T Y_j), W = V_J U_JJ^-1, MW = Y_J U_JJ^-1 */
int or_cholqr_deflate_prec(int64_t n, int m, const double* V, const double* Y, double tau,
                           double* W, double* MW, double* Z, int* keep);
/* Y = M^-1 X (n x m) for the block-Jacobi preconditioner of block size bs on
 * the matrix scaled as a solve with this jacobi flag would scale it */
void or_block_jacobi_apply(const or_matrix* A, int jacobi, int bs, int m, const double* X,
                           double* Y, int* status);
/* min_c ||b - B c||_2 for B n x m (row-major) by Householder QR.
 * Writes c[m]; returns 0, or -1 when R has a zero diagonal. */
int or_lstsq(int64_t n, int m, const double* B, const double* b, double* c);
/* the same, with the number of columns kept written to *kept (when not NULL) */
int or_lstsq_kept(int64_t n, int m, const double* B, const double* b, double* c, int* kept);

/* Algorithm 1 (MBPCG).  x receives the solution in the original space. */
int or_mbpcg_solve(const or_matrix* A, const double* b, const or_params* p,
                   double* x, or_info* info);
/* textbook Hestenes-Stiefel CG on the scaled system from x0 (original space,
 * may be NULL for zero); stop test ||D r|| / ||b|| < tol */
int or_hs_cg(const or_matrix* A, const double* b, const double* x0, double tol,
             int64_t max_iter, int jacobi, int bj_block, double* x, double* history, or_info* info);
/* Chronopoulos-Gear CG (x0 = 0 in the paper's baseline) */
int or_cg_cg(const or_matrix* A, const double* b, const double* x0, double tol,
             int64_t max_iter, int jacobi, int bj_block, double* x, double* history, or_info* info);

#ifdef __cplusplus
}
#endif
#endif

/*
 * CPU oracle of Multi-Basis Parallel CG (Xu & Regev, arXiv 2608.07327).
 *
 * TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline
 * leg of the benchmark call it; the GPU library never does.  Plain C99,
 * one thread, FP64, no BLAS.  Each function names the passage of the paper
 * it follows.  Where the paper is silent the reading taken is stated at the
 * function.
 */
#define _POSIX_C_SOURCE 199309L
#include "mbpcg_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

static int g_sum_mode = 0;

void or_set_summation(int mode) { g_sum_mode = mode; }

static double now_s(void)
{
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

static void* xcalloc(size_t count, size_t size)
{
    void* p = calloc(count ? count : 1, size ? size : 1);
    if (!p) abort();
    return p;
}

/* ---------------------------------------------------------------------------
 * Reductions over the n rows.  Mode 0 adds the row terms left to right.
 * Mode 1 adds them in blocks of 64 rows and combines the block sums as a
 * binary counter (pairwise tree); it exists only to measure how much the
 * result moves when the summation order changes.
 * ------------------------------------------------------------------------- */
#define OR_BLOCK 64
#define OR_LEVELS 64

typedef struct {
    int E;
    int64_t in_block;
    double* blk;
    double* lvl;     /* OR_LEVELS x E */
    int used[OR_LEVELS];
    double* out;     /* E: mode-0 running sums */
} reducer;

static void red_init(reducer* R, int E)
{
    memset(R, 0, sizeof(*R));
    R->E = E;
    R->out = (double*)xcalloc((size_t)E, sizeof(double));
    if (g_sum_mode == 1) {
        R->blk = (double*)xcalloc((size_t)E, sizeof(double));
        R->lvl = (double*)xcalloc((size_t)E * OR_LEVELS, sizeof(double));
    }
}

/* target for this row's terms */
static double* red_row(reducer* R) { return g_sum_mode == 1 ? R->blk : R->out; }

static void red_push_block(reducer* R)
{
    int E = R->E, l = 0;
    while (l < OR_LEVELS && R->used[l]) {
        for (int e = 0; e < E; ++e) R->blk[e] = R->lvl[(size_t)l * E + e] + R->blk[e];
        R->used[l] = 0;
        ++l;
    }
    for (int e = 0; e < E; ++e) R->lvl[(size_t)l * E + e] = R->blk[e];
    R->used[l] = 1;
    memset(R->blk, 0, sizeof(double) * (size_t)E);
    R->in_block = 0;
}

static void red_end_row(reducer* R)
{
    if (g_sum_mode == 1 && ++R->in_block == OR_BLOCK) red_push_block(R);
}

static void red_finish(reducer* R, double* result)
{
    if (g_sum_mode == 1) {
        if (R->in_block) red_push_block(R);
        for (int e = 0; e < R->E; ++e) R->out[e] = 0.0;
        for (int l = 0; l < OR_LEVELS; ++l)
            if (R->used[l])
                for (int e = 0; e < R->E; ++e) R->out[e] += R->lvl[(size_t)l * R->E + e];
        free(R->blk);
        free(R->lvl);
    }
    memcpy(result, R->out, sizeof(double) * (size_t)R->E);
    free(R->out);
}

/* sum_r x[r*incx] * y[r*incy] */
static double dot_strided(int64_t n, const double* x, int64_t incx, const double* y, int64_t incy)
{
    reducer R;
    red_init(&R, 1);
    for (int64_t r = 0; r < n; ++r) {
        red_row(&R)[0] += x[r * incx] * y[r * incy];
        red_end_row(&R);
    }
    double v;
    red_finish(&R, &v);
    return v;
}

/* ---------------------------------------------------------------------------
 * Random initial block (Alg. 1, the random block U; Sec. 2 states only that the entries
 * are iid Uniform(-1, 1)).  Reading taken: SplitMix64 (Steele, Lea & Flood,
 * "Fast splittable pseudorandom number generators", OOPSLA 2014) used as a
 * counter-based generator: output k of the stream seeded with `seed`.
 * ------------------------------------------------------------------------- */
uint64_t or_splitmix64(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + (k + 1u) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

void or_uniform_block(uint64_t seed, int64_t n, int s, double* U)
{
    for (int64_t r = 0; r < n; ++r)
        for (int j = 0; j < s; ++j) {
            uint64_t z = or_splitmix64(seed, (uint64_t)j * (uint64_t)n + (uint64_t)r);
            double u = (double)(z >> 11) * (1.0 / 9007199254740992.0);
            U[r * s + j] = 2.0 * u - 1.0;
        }
}

/* ---------------------------------------------------------------------------
 * Nearest BF16 (8 significant bits) with ties to even, straight from the
 * double: the significand scaled to 8 integer bits and rounded by rint
 * (round-half-even in the default rounding mode).  Normal range only, which
 * covers every matrix and block this oracle rounds.
 * ------------------------------------------------------------------------- */
double or_round_bf16(double x)
{
    if (x == 0.0 || !isfinite(x)) return x;
    int e;
    double m = frexp(x, &e);          /* x = m 2^e, 0.5 <= |m| < 1 */
    return ldexp(rint(ldexp(m, 8)), e - 8);
}

static double round_lo(int lo, double x)
{
    return lo == 1 ? (double)(float)x : or_round_bf16(x);
}

/* ---------------------------------------------------------------------------
 * Block product Y = A X (Alg. 1: A U for the initial block and A P in every iteration).  CSR rows
 * are summed in stored order; a dense product sums over columns in order.
 * With A->lo set (dense only), A and X are rounded to FP32 or BF16 and each
 * product is rounded to FP32 and added in FP32, as the mixed-precision
 * extension's inner products accumulate.
 * ------------------------------------------------------------------------- */
void or_matmul_block(const or_matrix* A, int k, const double* X, double* Y)
{
    int64_t n = A->n;
    if (A->dense && A->lo) {
        /* FP32 sums over the columns: sequential in mode 0; in mode 1 blocks
         * of OR_BLOCK columns are summed and the block sums combined as a
         * binary counter, all in FP32 */
        const size_t E = (size_t)(n * k);
        float* acc = (float*)calloc(E, sizeof(float));
        float* xr = (float*)malloc(sizeof(float) * (size_t)k);
        float* lvl = NULL;
        int used[OR_LEVELS];
        memset(used, 0, sizeof(used));
        int in_block = 0;
        if (g_sum_mode == 1) lvl = (float*)calloc(E * OR_LEVELS, sizeof(float));
        for (int64_t c = 0; c < n; ++c) {
            const double* col = A->a + c * A->lda;
            for (int j = 0; j < k; ++j) xr[j] = (float)round_lo(A->lo, X[c * k + j]);
            for (int64_t r = 0; r < n; ++r) {
                const float a = (float)round_lo(A->lo, col[r]);
                float* yr = acc + r * k;
                for (int j = 0; j < k; ++j) yr[j] = yr[j] + a * xr[j];
            }
            if (g_sum_mode == 1 && (++in_block == OR_BLOCK || c == n - 1)) {
                int l = 0;   /* acc holds a block sum: carry it up the counter */
                while (l < OR_LEVELS && used[l]) {
                    for (size_t e = 0; e < E; ++e) acc[e] = lvl[(size_t)l * E + e] + acc[e];
                    used[l] = 0;
                    ++l;
                }
                memcpy(lvl + (size_t)l * E, acc, sizeof(float) * E);
                used[l] = 1;
                memset(acc, 0, sizeof(float) * E);
                in_block = 0;
            }
        }
        if (g_sum_mode == 1) {
            for (int l = 0; l < OR_LEVELS; ++l)
                if (used[l])
                    for (size_t e = 0; e < E; ++e) acc[e] = acc[e] + lvl[(size_t)l * E + e];
            free(lvl);
        }
        for (size_t e = 0; e < E; ++e) Y[e] = (double)acc[e];
        free(xr);
        free(acc);
        return;
    }
    if (!A->dense) {
        for (int64_t r = 0; r < n; ++r)
            for (int j = 0; j < k; ++j) {
                double acc = 0.0;
                for (int32_t q = A->rowptr[r]; q < A->rowptr[r + 1]; ++q)
                    acc += A->vals[q] * X[(int64_t)A->colind[q] * k + j];
                Y[r * k + j] = acc;
            }
    } else {
        /* the sum over the columns is a reduction over n terms: sequential in
         * mode 0, blocked pairwise in mode 1 */
        reducer Rd;
        red_init(&Rd, (int)(n * k));
        for (int64_t c = 0; c < n; ++c) {
            const double* col = A->a + c * A->lda;
            const double* xr = X + c * k;
            double* acc = red_row(&Rd);
            for (int64_t r = 0; r < n; ++r) {
                double a = col[r];
                double* yr = acc + r * k;
                for (int j = 0; j < k; ++j) yr[j] += a * xr[j];
            }
            red_end_row(&Rd);
        }
        red_finish(&Rd, Y);
    }
}

/* C = X^T Y (Alg. 1: P^T A P of the step matrix Xi; the Cholesky QR Grams) */
void or_gram(int64_t n, int k1, const double* X, int k2, const double* Y, double* C)
{
    reducer R;
    red_init(&R, k1 * k2);
    for (int64_t r = 0; r < n; ++r) {
        double* acc = red_row(&R);
        const double* xr = X + r * k1;
        const double* yr = Y + r * k2;
        for (int i = 0; i < k1; ++i)
            for (int j = 0; j < k2; ++j) acc[i * k2 + j] += xr[i] * yr[j];
        red_end_row(&R);
    }
    red_finish(&R, C);
}

/* Textbook lower Cholesky by columns, reading the lower triangle of C
 * (Sec. 3: Xi is applied through a Cholesky factor of P^T A P). */
int or_cholesky(int m, const double* C, double* L)
{
    memset(L, 0, sizeof(double) * (size_t)(m * m));
    for (int j = 0; j < m; ++j) {
        double d = C[j * m + j];
        for (int k = 0; k < j; ++k) d -= L[j * m + k] * L[j * m + k];
        if (!(d > 0.0) || !isfinite(d)) return -1;
        double ljj = sqrt(d);
        L[j * m + j] = ljj;
        for (int i = j + 1; i < m; ++i) {
            double v = C[i * m + j];
            for (int k = 0; k < j; ++k) v -= L[i * m + k] * L[j * m + k];
            L[i * m + j] = v / ljj;
        }
    }
    return 0;
}

/* Xi = (L L^T)^{-1}: forward then backward substitution for each unit vector */
void or_spd_inverse(int m, const double* L, double* Xi)
{
    double* y = (double*)xcalloc((size_t)m, sizeof(double));
    for (int c = 0; c < m; ++c) {
        for (int i = 0; i < m; ++i) {
            double v = (i == c) ? 1.0 : 0.0;
            for (int k = 0; k < i; ++k) v -= L[i * m + k] * y[k];
            y[i] = v / L[i * m + i];
        }
        for (int i = m - 1; i >= 0; --i) {
            double v = y[i];
            for (int k = i + 1; k < m; ++k) v -= L[k * m + i] * Xi[k * m + c];
            Xi[i * m + c] = v / L[i * m + i];
        }
    }
    free(y);
}

/* ---------------------------------------------------------------------------
 * Cholesky QR (Sec. 3: the single-pass Cholesky QR of Fukaya et al.) with
 * column dropping.  The paper only needs the new basis to keep independent
 * columns; it does not say what to do when a column loses independence.
 * Reading taken: factor G = V^T V = U^T U column by column and drop column
 * j when its independent part is too small, delta_j <= tau * G_jj, where
 * delta_j = G_jj - sum over kept l < j of U_lj^2.  Kept set J:
 *   W = V_J U_JJ^{-1},  Z = U_{J, :}  (|J| x m, upper trapezoidal),
 * so V = W Z up to the dropped parts and the recurrences of Alg. 1 keep
 * their form with a rectangular Z.
 * ------------------------------------------------------------------------- */
/* The factorisation half: from the Gram G (m x m; the entries G[l][j], l < j,
 * and the diagonal are read) to the kept set J (nk columns, keep[] flags),
 * Z = rows J of U and Mi = U_JJ^{-1} (nk x nk, upper triangular). */
static int cholqr_factor(int m, const double* G, double tau, double* Z, int* keep, int* J,
                         double* Mi)
{
    double* U = (double*)xcalloc((size_t)(m * m), sizeof(double));
    int nk = 0;
    for (int j = 0; j < m; ++j) {
        for (int a = 0; a < nk; ++a) {
            int l = J[a];
            double v = G[l * m + j];
            for (int b = 0; b < a; ++b) v -= U[J[b] * m + l] * U[J[b] * m + j];
            U[l * m + j] = v / U[l * m + l];
        }
        double g = G[j * m + j];
        double d = g;
        for (int a = 0; a < nk; ++a) d -= U[J[a] * m + j] * U[J[a] * m + j];
        if (g > 0.0 && isfinite(d) && d > tau * g) {
            U[j * m + j] = sqrt(d);
            J[nk++] = j;
            keep[j] = 1;
        } else {
            keep[j] = 0;
        }
    }
    /* Z = rows J of U, upper trapezoidal */
    for (int a = 0; a < nk; ++a)
        for (int j = 0; j < m; ++j) Z[a * m + j] = (j >= J[a]) ? U[J[a] * m + j] : 0.0;
    /* Minv = U_JJ^{-1} by back substitution, column by column */
    for (int c = 0; c < nk; ++c)
        for (int a = c; a >= 0; --a) {
            double v = (a == c) ? 1.0 : 0.0;
            for (int b = a + 1; b <= c; ++b) v -= U[J[a] * m + J[b]] * Mi[b * nk + c];
            Mi[a * nk + c] = v / U[J[a] * m + J[a]];
        }
    free(U);
    return nk;
}

/* W = V_J Mi (n x nk) for the kept set J of an n x m block V */
static void apply_kept_inverse(int64_t n, int m, int nk, const int* J, const double* Mi,
                               const double* V, double* W)
{
    for (int64_t r = 0; r < n; ++r)
        for (int c = 0; c < nk; ++c) {
            double acc = 0.0;
            for (int a = 0; a <= c; ++a) acc += V[r * m + J[a]] * Mi[a * nk + c];
            W[r * nk + c] = acc;
        }
}

int or_cholqr_deflate(int64_t n, int m, const double* V, double tau,
                      double* W, double* Z, int* keep)
{
    double* G = (double*)xcalloc((size_t)(m * m), sizeof(double));
    double* Mi = (double*)xcalloc((size_t)(m * m + 1), sizeof(double));
    int* J = (int*)xcalloc((size_t)m, sizeof(int));
    or_gram(n, m, V, m, V, G);
    int nk = cholqr_factor(m, G, tau, Z, keep, J, Mi);
    apply_kept_inverse(n, m, nk, J, Mi, V, W);
    free(J);
    free(Mi);
    free(G);
    return nk;
}

/* ---------------------------------------------------------------------------
 * Preconditioned Cholesky QR (the preconditioned form of Dubrulle-R that the
 * paper says its method admits, Sec. 2).  With an SPD preconditioner M the
 * residual basis W is orthonormal in the M^-1 inner product, W^T M^-1 W = I,
 * and the directions are built from M^-1 W.  Given V and Y = M^-1 V, factor
 * the Gram V^T Y = U^T U (with the dropping rule of or_cholqr_deflate) and
 * return W = V_J U_JJ^{-1} and MW = Y_J U_JJ^{-1} (= M^-1 W).  V^T Y is
 * symmetric in exact arithmetic; the entry used for the pair (i > j) is
 * V_i^T Y_j.
 * ------------------------------------------------------------------------- */
int or_cholqr_deflate_prec(int64_t n, int m, const double* V, const double* Y, double tau,
                           double* W, double* MW, double* Z, int* keep)
{
    double* H = (double*)xcalloc((size_t)(m * m), sizeof(double));
    double* G = (double*)xcalloc((size_t)(m * m), sizeof(double));
    double* Mi = (double*)xcalloc((size_t)(m * m + 1), sizeof(double));
    int* J = (int*)xcalloc((size_t)m, sizeof(int));
    or_gram(n, m, V, m, Y, H);                 /* H[i][j] = V_i^T Y_j */
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) G[i * m + j] = (i >= j) ? H[i * m + j] : H[j * m + i];
    int nk = cholqr_factor(m, G, tau, Z, keep, J, Mi);
    apply_kept_inverse(n, m, nk, J, Mi, V, W);
    apply_kept_inverse(n, m, nk, J, Mi, Y, MW);
    free(J);
    free(Mi);
    free(G);
    free(H);
    return nk;
}


/* ---------------------------------------------------------------------------
 * Least squares min_c ||b - B c|| (Alg. 1, the combination c^ of the termination).  The paper writes
 * the normal equations and reports that forming B^T B overflows or loses
 * accuracy; the oracle computes the same minimiser by Householder QR.  A
 * column whose part orthogonal to the columns already taken is not above
 * 1e-12 of its norm (numerically dependent, or beyond the n-th independent
 * column when B has more columns than rows) is left out with coefficient 0;
 * the residual is the same minimum.
 * ------------------------------------------------------------------------- */
int or_lstsq(int64_t n, int m, const double* B, const double* b, double* c)
{
    return or_lstsq_kept(n, m, B, b, c, NULL);
}

int or_lstsq_kept(int64_t n, int m, const double* B, const double* b, double* c, int* kept)
{
    const double tau_ls = 1e-12;
    double* Bc = (double*)xcalloc((size_t)(n * m), sizeof(double)); /* column-major */
    double* bb = (double*)xcalloc((size_t)n, sizeof(double));
    double* rdiag = (double*)xcalloc((size_t)m + 1, sizeof(double));
    int* kc = (int*)xcalloc((size_t)m + 1, sizeof(int)); /* kept column of reflection q */
    int rc = 0;
    for (int64_t r = 0; r < n; ++r) {
        for (int j = 0; j < m; ++j) Bc[(int64_t)j * n + r] = B[r * m + j];
        bb[r] = b[r];
    }
    int p = 0; /* reflections done = kept columns */
    for (int k = 0; k < m; ++k) {
        c[k] = 0.0;
        double* v = Bc + (int64_t)k * n;
        double n0 = sqrt(dot_strided(n, v, 1, v, 1));
        if (!isfinite(n0)) { rc = -1; break; }
        if (p >= n) continue;
        double nrm = sqrt(dot_strided(n - p, v + p, 1, v + p, 1));
        if (!(nrm > tau_ls * n0)) continue; /* dependent (or zero) column: left out */
        double alpha = (v[p] > 0.0) ? -nrm : nrm;
        v[p] -= alpha; /* Householder vector in rows p.. of column k */
        double vtv = dot_strided(n - p, v + p, 1, v + p, 1);
        for (int j = k + 1; j < m; ++j) {
            double* col = Bc + (int64_t)j * n;
            double t = 2.0 * dot_strided(n - p, v + p, 1, col + p, 1) / vtv;
            for (int64_t r = p; r < n; ++r) col[r] -= t * v[r];
        }
        double t = 2.0 * dot_strided(n - p, v + p, 1, bb + p, 1) / vtv;
        for (int64_t r = p; r < n; ++r) bb[r] -= t * v[r];
        rdiag[p] = alpha;
        kc[p] = k;
        ++p;
    }
    if (rc == 0) {
        if (p == 0) rc = -1;
        /* back substitution over the kept columns; row q of R holds
         * Bc[col][q] for the kept columns after column kc[q] */
        for (int q = p - 1; q >= 0 && rc == 0; --q) {
            double v = bb[q];
            for (int q2 = q + 1; q2 < p; ++q2) v -= Bc[(int64_t)kc[q2] * n + q] * c[kc[q2]];
            c[kc[q]] = v / rdiag[q];
        }
    }
    if (kept) *kept = p;
    free(kc);
    free(rdiag);
    free(bb);
    free(Bc);
    return rc;
}

/* ---------------------------------------------------------------------------
 * Diagonal scaling (Sec. 1): D_jj = sqrt(A_jj), A~ = D^{-1} A D^{-1},
 * entry by entry a_rc / (d_r * d_c).
 * ------------------------------------------------------------------------- */
typedef struct {
    or_matrix As;
    double* vals;
    double* a;
    double* d;
} scaled_t;

static int make_scaled(const or_matrix* A, int jacobi, scaled_t* S)
{
    int64_t n = A->n;
    memset(S, 0, sizeof(*S));
    S->d = (double*)xcalloc((size_t)n, sizeof(double));
    S->As = *A;
    for (int64_t r = 0; r < n; ++r) {
        double arr = 0.0;
        if (!A->dense) {
            for (int32_t q = A->rowptr[r]; q < A->rowptr[r + 1]; ++q)
                if (A->colind[q] == r) arr += A->vals[q];
        } else {
            arr = A->a[r * A->lda + r];
        }
        if (jacobi) {
            if (!(arr > 0.0) || !isfinite(arr)) return OR_ERR_NOT_SPD;
            S->d[r] = sqrt(arr);
        } else {
            S->d[r] = 1.0;
        }
    }
    if (!jacobi) return OR_OK;
    if (!A->dense) {
        int64_t nnz = A->rowptr[n];
        S->vals = (double*)xcalloc((size_t)nnz, sizeof(double));
        for (int64_t r = 0; r < n; ++r)
            for (int32_t q = A->rowptr[r]; q < A->rowptr[r + 1]; ++q)
                S->vals[q] = A->vals[q] / (S->d[r] * S->d[A->colind[q]]);
        S->As.vals = S->vals;
    } else {
        S->a = (double*)xcalloc((size_t)(n * n), sizeof(double));
        for (int64_t c = 0; c < n; ++c)
            for (int64_t r = 0; r < n; ++r)
                S->a[c * n + r] = A->a[c * A->lda + r] / (S->d[r] * S->d[c]);
        S->As.a = S->a;
        S->As.lda = n;
    }
    return OR_OK;
}

static void free_scaled(scaled_t* S)
{
    free(S->vals);
    free(S->a);
    free(S->d);
}

/* ---------------------------------------------------------------------------
 * Block-Jacobi preconditioner: M = the block diagonal of the (scaled) matrix
 * with blocks of bs consecutive rows (the last one shorter when bs does not
 * divide n).  Each block is factored by the textbook Cholesky; M^-1 X is
 * formed block by block by forward and back substitution.
 * ------------------------------------------------------------------------- */
typedef struct {
    int bs;
    int64_t n, nblk;
    double* L; /* nblk blocks of bs x bs, lower factor, row-major */
} bjac_t;

static int bjac_setup(const or_matrix* A, int bs, bjac_t* M)
{
    int64_t n = A->n;
    M->bs = bs;
    M->n = n;
    M->nblk = (n + bs - 1) / bs;
    M->L = (double*)xcalloc((size_t)(M->nblk * bs * bs), sizeof(double));
    double* B = (double*)xcalloc((size_t)(bs * bs), sizeof(double));
    int rc = OR_OK;
    for (int64_t k = 0; k < M->nblk && rc == OR_OK; ++k) {
        int64_t lo = k * bs, hi = lo + bs < n ? lo + bs : n;
        int nb = (int)(hi - lo);
        memset(B, 0, sizeof(double) * (size_t)(bs * bs));
        for (int64_t r = lo; r < hi; ++r) {
            if (A->dense) {
                for (int64_t c = lo; c < hi; ++c) B[(r - lo) * nb + (c - lo)] = A->a[c * A->lda + r];
            } else {
                for (int32_t e = A->rowptr[r]; e < A->rowptr[r + 1]; ++e) {
                    int64_t c = A->colind[e];
                    if (c >= lo && c < hi) B[(r - lo) * nb + (c - lo)] += A->vals[e];
                }
            }
        }
        if (or_cholesky(nb, B, M->L + k * bs * bs) != 0) rc = OR_ERR_NOT_SPD;
    }
    free(B);
    return rc;
}

/* Y = M^-1 X for an n x m row-major block */
static void bjac_apply(const bjac_t* M, int m, const double* X, double* Y)
{
    int bs = M->bs;
    double* z = (double*)xcalloc((size_t)bs, sizeof(double));
    for (int64_t k = 0; k < M->nblk; ++k) {
        int64_t lo = k * bs, hi = lo + bs < M->n ? lo + bs : M->n;
        int nb = (int)(hi - lo);
        const double* L = M->L + k * bs * bs;
        for (int j = 0; j < m; ++j) {
            for (int i = 0; i < nb; ++i) {      /* L z = x */
                double v = X[(lo + i) * m + j];
                for (int c = 0; c < i; ++c) v -= L[i * nb + c] * z[c];
                z[i] = v / L[i * nb + i];
            }
            for (int i = nb - 1; i >= 0; --i) { /* L^T y = z */
                double v = z[i];
                for (int c = i + 1; c < nb; ++c) v -= L[c * nb + i] * Y[(lo + c) * m + j];
                Y[(lo + i) * m + j] = v / L[i * nb + i];
            }
        }
    }
    free(z);
}

static void bjac_free(bjac_t* M)
{
    free(M->L);
    M->L = NULL;
}

/* y = M^-1 x for the preconditioner of a solve; identity when bs < 2 */
void or_block_jacobi_apply(const or_matrix* A, int jacobi, int bs, int m, const double* X,
                           double* Y, int* status)
{
    scaled_t S;
    int rc = make_scaled(A, jacobi, &S);
    bjac_t M;
    memset(&M, 0, sizeof(M));
    if (rc == OR_OK) rc = bjac_setup(&S.As, bs, &M);
    if (rc == OR_OK) bjac_apply(&M, m, X, Y);
    bjac_free(&M);
    free_scaled(&S);
    if (status) *status = rc;
}

static double true_rel_residual(const or_matrix* A, const double* b, const double* x, double bnorm)
{
    int64_t n = A->n;
    double* ax = (double*)xcalloc((size_t)n, sizeof(double));
    or_matmul_block(A, 1, x, ax);
    for (int64_t r = 0; r < n; ++r) ax[r] = b[r] - ax[r];
    double v = sqrt(dot_strided(n, ax, 1, ax, 1)) / bnorm;
    free(ax);
    return v;
}

/* column norms of D R (original residuals, Sec. 1: R = D R~), j < s */
static void residual_norms(int64_t n, int s, const double* R, const double* d, int scaled, double* nu)
{
    reducer Rd;
    red_init(&Rd, s);
    for (int64_t r = 0; r < n; ++r) {
        double* acc = red_row(&Rd);
        double dr = scaled ? 1.0 : d[r];
        for (int j = 0; j < s; ++j) {
            double v = dr * R[r * s + j];
            acc[j] += v * v;
        }
        red_end_row(&Rd);
    }
    red_finish(&Rd, nu);
    for (int j = 0; j < s; ++j) nu[j] = sqrt(nu[j]);
}

/* ---------------------------------------------------------------------------
 * Algorithm 1 (Multi-Basis Parallel CG), with the initial-residual system of
 * Sec. 2, Proposition 1 for B^ = B - R, and the two-tolerance termination
 * with fallback to the best column described after Proposition 1.
 * ------------------------------------------------------------------------- */
int or_mbpcg_solve(const or_matrix* A, const double* b, const or_params* p,
                   double* x, or_info* info)
{
    const int64_t n = A->n;
    const int s = p->s;
    const double tol = p->tol;
    const double tol0 = (p->tol_initial > 0.0) ? p->tol_initial : p->tol;
    const double tau = (p->tau > 0.0) ? p->tau : 1e-12;
    or_info inf;
    memset(&inf, 0, sizeof(inf));
    double t0 = now_s();

    double bnorm = sqrt(dot_strided(n, b, 1, b, 1));
    if (!isfinite(bnorm)) {
        inf.status = OR_ERR_NONFINITE;
        if (info) *info = inf;
        return inf.status;
    }
    if (bnorm == 0.0) {
        memset(x, 0, sizeof(double) * (size_t)n);
        inf.final_width = s;
        if (info) *info = inf;
        return OR_OK;
    }

    scaled_t S;
    bjac_t BJ;
    memset(&BJ, 0, sizeof(BJ));
    const int prec = p->bj_block >= 2;
    int rc = make_scaled(A, p->jacobi, &S);
    if (rc == OR_OK && prec) rc = bjac_setup(&S.As, p->bj_block, &BJ);
    if (rc != OR_OK) {
        bjac_free(&BJ);
        free_scaled(&S);
        inf.status = rc;
        if (info) *info = inf;
        return rc;
    }
    const double* d = S.d;
    const or_matrix* As = &S.As;

    size_t blk = (size_t)(n * s);
    double* bbar = (double*)xcalloc((size_t)n, sizeof(double));
    double* U = (double*)xcalloc(blk, sizeof(double));
    double* Y = (double*)xcalloc(blk, sizeof(double));
    double* X0 = (double*)xcalloc(blk, sizeof(double));
    double* Xt = (double*)xcalloc(blk, sizeof(double));
    double* R = (double*)xcalloc(blk, sizeof(double));
    double* W = (double*)xcalloc(blk, sizeof(double));
    double* P = (double*)xcalloc(blk, sizeof(double));
    double* Q = (double*)xcalloc(blk, sizeof(double));
    double* V = (double*)xcalloc(blk, sizeof(double));
    double* Pn = (double*)xcalloc(blk, sizeof(double));
    double* Yp = (double*)xcalloc(blk, sizeof(double)); /* M^-1 V (preconditioned) */
    double* MW = (double*)xcalloc(blk, sizeof(double)); /* M^-1 W (preconditioned) */
    double* Sig = (double*)xcalloc((size_t)(s * s), sizeof(double));
    double* Sn = (double*)xcalloc((size_t)(s * s), sizeof(double));
    double* Z = (double*)xcalloc((size_t)(s * s), sizeof(double));
    double* C = (double*)xcalloc((size_t)(s * s), sizeof(double));
    double* L = (double*)xcalloc((size_t)(s * s), sizeof(double));
    double* Xi = (double*)xcalloc((size_t)(s * s), sizeof(double));
    double* al = (double*)xcalloc((size_t)(s * s), sizeof(double));
    double* nu = (double*)xcalloc((size_t)s, sizeof(double));
    double* chat = (double*)xcalloc((size_t)s, sizeof(double));
    int* keep = (int*)xcalloc((size_t)s, sizeof(int));

    for (int64_t r = 0; r < n; ++r) bbar[r] = b[r] / d[r];

    /* random block and initial guess: X0 = (||B||_F / ||A U||_F) U with B = [b ... b] */
    if (p->U) memcpy(U, p->U, sizeof(double) * blk);
    else or_uniform_block(p->seed, n, s, U);
    or_matmul_block(As, s, U, Y);
    double nb2 = dot_strided(n, bbar, 1, bbar, 1);
    double ny2;
    {
        reducer Rf;
        red_init(&Rf, 1);
        for (int64_t r = 0; r < n; ++r) {
            double acc = 0.0;
            for (int j = 0; j < s; ++j) acc += Y[r * s + j] * Y[r * s + j];
            red_row(&Rf)[0] += acc;
            red_end_row(&Rf);
        }
        red_finish(&Rf, &ny2);
    }
    double gamma = sqrt((double)s * nb2) / sqrt(ny2);
    /* scaled right-hand sides, X~0 = 0 and R0: A X0 is taken as gamma * (A U) */
    for (size_t e = 0; e < blk; ++e) {
        X0[e] = gamma * U[e];
        R[e] = bbar[e / (size_t)s] - gamma * Y[e];
    }
    if (!isfinite(gamma)) { rc = OR_ERR_NONFINITE; goto fallback_none; }

    /* first Cholesky QR (W0, Sigma0) and P0 = W0 (preconditioned: the QR in
     * the M^-1 inner product and P0 = M^-1 W0) */
    int m;
    if (prec) {
        bjac_apply(&BJ, s, R, Yp);
        m = or_cholqr_deflate_prec(n, s, R, Yp, tau, W, MW, Z, keep);
    } else {
        m = or_cholqr_deflate(n, s, R, tau, W, Z, keep);
    }
    inf.deflations = s - m;
    memcpy(Sig, Z, sizeof(double) * (size_t)(m * s));
    for (int64_t r = 0; r < n; ++r)
        for (int c = 0; c < m; ++c) P[r * m + c] = prec ? MW[r * m + c] : W[r * m + c];
    inf.seconds_setup = now_s() - t0;

    int64_t it = 0;
    int h = 0;
    double nu_h;
    residual_norms(n, s, R, d, p->ls_scaled, nu);
    {
        double bref = p->ls_scaled ? sqrt(nb2) : bnorm;
        h = 0;
        for (int j = 1; j < s; ++j) if (nu[j] < nu[h]) h = j;
        nu_h = nu[h] / bref;
    }
    int converged = 0, accepted = 0;
    double rel_ls = NAN;
    if (m == 0) {
        converged = 1;
    }
    /* no iteration when the first Cholesky QR already dropped every column
     * (R0 = 0): the count stays 0 */
    if (!converged)
    for (it = 1; !converged && it <= p->max_iter; ++it) {
        /* step matrix Xi = (P^T A P)^-1 */
        or_matmul_block(As, m, P, Q);
        or_gram(n, m, P, m, Q, C);
        if (or_cholesky(m, C, L) != 0) { rc = OR_ERR_NOT_SPD; it -= 1; break; }
        or_spd_inverse(m, L, Xi);
        for (int a = 0; a < m; ++a)
            for (int j = 0; j < s; ++j) {
                double acc = 0.0;
                for (int c = 0; c < m; ++c) acc += Xi[a * m + c] * Sig[c * s + j];
                al[a * s + j] = acc;
            }
        /* X~ += P alpha, R -= (A P) alpha */
        for (int64_t r = 0; r < n; ++r)
            for (int j = 0; j < s; ++j) {
                double tx = 0.0, tr = 0.0;
                for (int a = 0; a < m; ++a) {
                    tx += P[r * m + a] * al[a * s + j];
                    tr += Q[r * m + a] * al[a * s + j];
                }
                Xt[r * s + j] = Xt[r * s + j] + tx;
                R[r * s + j] = R[r * s + j] - tr;
            }
        /* best column h in the original residual norm */
        residual_norms(n, s, R, d, p->ls_scaled, nu);
        double bref = p->ls_scaled ? sqrt(nb2) : bnorm;
        h = 0;
        for (int j = 1; j < s; ++j) if (nu[j] < nu[h]) h = j;
        nu_h = nu[h] / bref;
        if (p->history) p->history[it - 1] = nu_h;
        if (p->prop1_gap) {
            /* Proposition 1 (scaled system): A X = B - R with X = X~ + X0 */
            double* T = Pn;
            for (size_t e = 0; e < blk; ++e) V[e] = Xt[e] + X0[e];
            or_matmul_block(As, s, V, T);
            double g2 = 0.0;
            for (int64_t r = 0; r < n; ++r)
                for (int j = 0; j < s; ++j) {
                    double e = T[r * s + j] - (bbar[r] - R[r * s + j]);
                    g2 += e * e;
                }
            p->prop1_gap[it - 1] = sqrt(g2) / sqrt((double)s * nb2);
        }
        if (!isfinite(nu_h)) { rc = OR_ERR_NONFINITE; break; }
        /* stop test and least-squares termination */
        if (nu_h < tol0) {
            /* B^ = B - R in the original space, c^ and its residual */
            double* Bh = V;
            for (int64_t r = 0; r < n; ++r)
                for (int j = 0; j < s; ++j) {
                    double ro = p->ls_scaled ? R[r * s + j] : d[r] * R[r * s + j];
                    double br = p->ls_scaled ? bbar[r] : b[r];
                    Bh[r * s + j] = br - ro;
                }
            const double* bref_v = p->ls_scaled ? bbar : b;
            int lsr = or_lstsq_kept(n, s, Bh, bref_v, chat, &inf.ls_kept);
            int finite = (lsr == 0);
            for (int j = 0; j < s && finite; ++j) finite = isfinite(chat[j]);
            if (finite) {
                double r2;
                reducer Rr;
                red_init(&Rr, 1);
                for (int64_t r = 0; r < n; ++r) {
                    double acc = 0.0;
                    for (int j = 0; j < s; ++j) acc += Bh[r * s + j] * chat[j];
                    double e = bref_v[r] - acc;
                    red_row(&Rr)[0] += e * e;
                    red_end_row(&Rr);
                }
                red_finish(&Rr, &r2);
                rel_ls = sqrt(r2) / bref;
            }
            if (finite && rel_ls < tol) { converged = 1; accepted = 1; break; }
            if (nu_h < tol) { converged = 1; accepted = 0; break; }
        }
        /* V = W - (A P) Xi, then Cholesky QR with column dropping */
        for (int64_t r = 0; r < n; ++r)
            for (int c = 0; c < m; ++c) {
                double acc = 0.0;
                for (int a = 0; a < m; ++a) acc += Q[r * m + a] * Xi[a * m + c];
                V[r * m + c] = W[r * m + c] - acc;
            }
        int mn;
        if (prec) {
            bjac_apply(&BJ, m, V, Yp);
            mn = or_cholqr_deflate_prec(n, m, V, Yp, tau, W, MW, Z, keep);
        } else {
            mn = or_cholqr_deflate(n, m, V, tau, W, Z, keep);
        }
        inf.deflations += m - mn;
        /* P = W + P Z^T (preconditioned: M^-1 W + P Z^T), Sigma = Z Sigma */
        const double* Wd = prec ? MW : W;
        for (int64_t r = 0; r < n; ++r)
            for (int c = 0; c < mn; ++c) {
                double acc = 0.0;
                for (int a = 0; a < m; ++a) acc += P[r * m + a] * Z[c * m + a];
                Pn[r * mn + c] = Wd[r * mn + c] + acc;
            }
        memcpy(P, Pn, sizeof(double) * (size_t)(n * mn));
        for (int c = 0; c < mn; ++c)
            for (int j = 0; j < s; ++j) {
                double acc = 0.0;
                for (int a = 0; a < m; ++a) acc += Z[c * m + a] * Sig[a * s + j];
                Sn[c * s + j] = acc;
            }
        memcpy(Sig, Sn, sizeof(double) * (size_t)(mn * s));
        m = mn;
        if (m == 0) { rc = OR_ERR_BREAKDOWN; break; }
    }
    if (it > p->max_iter) it = p->max_iter;
    inf.iterations = it;
    inf.final_width = m;
    inf.best_column = h;
    inf.rel_res_best = nu_h;
    inf.rel_res_ls = rel_ls;

    /* X = X~ + X0, x = X c^ (or the best column) in the original space */
    if (converged && accepted) {
        for (int64_t r = 0; r < n; ++r) {
            double acc = 0.0;
            for (int j = 0; j < s; ++j) acc += (Xt[r * s + j] + X0[r * s + j]) * chat[j];
            x[r] = acc / d[r];
        }
        inf.status = OR_OK;
    } else {
        for (int64_t r = 0; r < n; ++r) x[r] = (Xt[r * s + h] + X0[r * s + h]) / d[r];
        inf.used_fallback = 1;
        inf.status = converged ? OR_OK : (rc != OR_OK ? rc : OR_NOT_CONVERGED);
    }
    if (p->X_out)
        for (size_t e = 0; e < blk; ++e) p->X_out[e] = Xt[e] + X0[e];
    if (p->R_out) memcpy(p->R_out, R, sizeof(double) * blk);
    inf.rel_res_true = true_rel_residual(A, b, x, bnorm);
    /* Prop. 1 holds in exact arithmetic only: A X and B - R drift apart by
     * rounding, and coefficients c^ of large magnitude (the columns of X
     * approach the same x) amplify that drift in X c^.  The combination is
     * kept when its true residual meets the tolerance; otherwise the best
     * column is returned when its own true residual is lower. */
    if (p->check_true && converged && accepted && !(inf.rel_res_true < tol)) {
        double* xh = (double*)xcalloc((size_t)n, sizeof(double));
        for (int64_t r = 0; r < n; ++r) xh[r] = (Xt[r * s + h] + X0[r * s + h]) / d[r];
        double th = true_rel_residual(A, b, xh, bnorm);
        if (th < inf.rel_res_true) {
            memcpy(x, xh, sizeof(double) * (size_t)n);
            inf.rel_res_true = th;
            inf.used_fallback = 1;
        }
        free(xh);
    }
    inf.seconds = now_s() - t0;
    rc = inf.status;
    goto done;

fallback_none:
    inf.status = rc;
    memset(x, 0, sizeof(double) * (size_t)n);
    inf.seconds = now_s() - t0;
done:
    free(keep); free(chat); free(nu); free(al); free(Xi); free(L); free(C); free(Z);
    free(Sn); free(Sig); free(Pn); free(V); free(Q); free(P); free(W); free(R);
    free(Xt); free(X0); free(Y); free(U); free(bbar); free(Yp); free(MW);
    bjac_free(&BJ);
    free_scaled(&S);
    if (info) *info = inf;
    return rc;
}

/* ---------------------------------------------------------------------------
 * Textbook CG (Hestenes & Stiefel) on the diagonally scaled system; the
 * s = 1 special case of Alg. 1 reduces to it in exact arithmetic.
 * ------------------------------------------------------------------------- */
int or_hs_cg(const or_matrix* A, const double* b, const double* x0, double tol,
             int64_t max_iter, int jacobi, int bj_block, double* x, double* history,
             or_info* info)
{
    int64_t n = A->n;
    or_info inf;
    memset(&inf, 0, sizeof(inf));
    double t0 = now_s();
    double bnorm = sqrt(dot_strided(n, b, 1, b, 1));
    if (bnorm == 0.0) {
        memset(x, 0, sizeof(double) * (size_t)n);
        if (info) *info = inf;
        return OR_OK;
    }
    scaled_t S;
    bjac_t BJ;
    memset(&BJ, 0, sizeof(BJ));
    const int prec = bj_block >= 2;
    int rc = make_scaled(A, jacobi, &S);
    if (rc == OR_OK && prec) rc = bjac_setup(&S.As, bj_block, &BJ);
    if (rc != OR_OK) {
        bjac_free(&BJ);
        free_scaled(&S);
        inf.status = rc;
        if (info) *info = inf;
        return rc;
    }
    double* xs = (double*)xcalloc((size_t)n, sizeof(double));
    double* r = (double*)xcalloc((size_t)n, sizeof(double));
    double* z = (double*)xcalloc((size_t)n, sizeof(double));
    double* pv = (double*)xcalloc((size_t)n, sizeof(double));
    double* q = (double*)xcalloc((size_t)n, sizeof(double));
    for (int64_t i = 0; i < n; ++i) xs[i] = x0 ? x0[i] * S.d[i] : 0.0;
    or_matmul_block(&S.As, 1, xs, q);
    for (int64_t i = 0; i < n; ++i) r[i] = b[i] / S.d[i] - q[i];
    /* preconditioned residual z = M^-1 r (z = r without a preconditioner) */
    if (prec) bjac_apply(&BJ, 1, r, z);
    else memcpy(z, r, sizeof(double) * (size_t)n);
    memcpy(pv, z, sizeof(double) * (size_t)n);
    double gam = dot_strided(n, r, 1, z, 1);
    int64_t it;
    double rel = NAN;
    int conv = 0;
    for (it = 1; it <= max_iter; ++it) {
        or_matmul_block(&S.As, 1, pv, q);
        double alpha = gam / dot_strided(n, pv, 1, q, 1);
        for (int64_t i = 0; i < n; ++i) { xs[i] += alpha * pv[i]; r[i] -= alpha * q[i]; }
        double e2 = 0.0;
        for (int64_t i = 0; i < n; ++i) { double v = S.d[i] * r[i]; e2 += v * v; }
        rel = sqrt(e2) / bnorm;
        if (history) history[it - 1] = rel;
        if (rel < tol) { conv = 1; break; }
        if (prec) bjac_apply(&BJ, 1, r, z);
        else memcpy(z, r, sizeof(double) * (size_t)n);
        double gn = dot_strided(n, r, 1, z, 1);
        double beta = gn / gam;
        gam = gn;
        for (int64_t i = 0; i < n; ++i) pv[i] = z[i] + beta * pv[i];
    }
    inf.iterations = conv ? it : max_iter;
    inf.status = conv ? OR_OK : OR_NOT_CONVERGED;
    inf.rel_res_best = rel;
    inf.final_width = 1;
    for (int64_t i = 0; i < n; ++i) x[i] = xs[i] / S.d[i];
    inf.seconds = now_s() - t0;
    inf.rel_res_true = true_rel_residual(A, b, x, bnorm);
    free(q); free(pv); free(z); free(r); free(xs);
    bjac_free(&BJ);
    free_scaled(&S);
    if (info) *info = inf;
    return inf.status;
}

/* ---------------------------------------------------------------------------
 * Chronopoulos-Gear CG (the paper's CG baseline, Sec. 1 and Sec. 4): both
 * inner products of an iteration are formed after the one SpMV, and
 * alpha_{i} = gamma_i / (delta_i - beta_i gamma_i / alpha_{i-1}), which
 * equals CG's p^T A p in exact arithmetic.
 * ------------------------------------------------------------------------- */
int or_cg_cg(const or_matrix* A, const double* b, const double* x0, double tol,
             int64_t max_iter, int jacobi, int bj_block, double* x, double* history,
             or_info* info)
{
    int64_t n = A->n;
    or_info inf;
    memset(&inf, 0, sizeof(inf));
    double t0 = now_s();
    double bnorm = sqrt(dot_strided(n, b, 1, b, 1));
    if (bnorm == 0.0) {
        memset(x, 0, sizeof(double) * (size_t)n);
        if (info) *info = inf;
        return OR_OK;
    }
    scaled_t S;
    bjac_t BJ;
    memset(&BJ, 0, sizeof(BJ));
    const int prec = bj_block >= 2;
    int rc = make_scaled(A, jacobi, &S);
    if (rc == OR_OK && prec) rc = bjac_setup(&S.As, bj_block, &BJ);
    if (rc != OR_OK) {
        bjac_free(&BJ);
        free_scaled(&S);
        inf.status = rc;
        if (info) *info = inf;
        return rc;
    }
    double* xs = (double*)xcalloc((size_t)n, sizeof(double));
    double* r = (double*)xcalloc((size_t)n, sizeof(double));
    double* u = (double*)xcalloc((size_t)n, sizeof(double));
    double* w = (double*)xcalloc((size_t)n, sizeof(double));
    double* pv = (double*)xcalloc((size_t)n, sizeof(double));
    double* sv = (double*)xcalloc((size_t)n, sizeof(double));
    for (int64_t i = 0; i < n; ++i) xs[i] = x0 ? x0[i] * S.d[i] : 0.0;
    or_matmul_block(&S.As, 1, xs, w);
    for (int64_t i = 0; i < n; ++i) r[i] = b[i] / S.d[i] - w[i];
    /* u = M^-1 r (u = r without a preconditioner), w = A u */
    if (prec) bjac_apply(&BJ, 1, r, u);
    else memcpy(u, r, sizeof(double) * (size_t)n);
    or_matmul_block(&S.As, 1, u, w);
    double gam = dot_strided(n, r, 1, u, 1);
    double del = dot_strided(n, w, 1, u, 1);
    double alpha = gam / del, beta = 0.0;
    int64_t it;
    double rel = NAN;
    int conv = 0;
    for (it = 1; it <= max_iter; ++it) {
        for (int64_t i = 0; i < n; ++i) {
            pv[i] = u[i] + beta * pv[i];
            sv[i] = w[i] + beta * sv[i];
            xs[i] += alpha * pv[i];
            r[i] -= alpha * sv[i];
        }
        double e2 = 0.0;
        for (int64_t i = 0; i < n; ++i) { double v = S.d[i] * r[i]; e2 += v * v; }
        rel = sqrt(e2) / bnorm;
        if (history) history[it - 1] = rel;
        if (rel < tol) { conv = 1; break; }
        if (prec) bjac_apply(&BJ, 1, r, u);
        else memcpy(u, r, sizeof(double) * (size_t)n);
        or_matmul_block(&S.As, 1, u, w);
        double gn = dot_strided(n, r, 1, u, 1);
        del = dot_strided(n, w, 1, u, 1);
        beta = gn / gam;
        alpha = gn / (del - beta * gn / alpha);
        gam = gn;
    }
    inf.iterations = conv ? it : max_iter;
    inf.status = conv ? OR_OK : OR_NOT_CONVERGED;
    inf.rel_res_best = rel;
    inf.final_width = 1;
    for (int64_t i = 0; i < n; ++i) x[i] = xs[i] / S.d[i];
    inf.seconds = now_s() - t0;
    inf.rel_res_true = true_rel_residual(A, b, x, bnorm);
    free(sv); free(pv); free(w); free(u); free(r); free(xs);
    bjac_free(&BJ);
    free_scaled(&S);
    if (info) *info = inf;
    return inf.status;
}

// Host-side launch interface of the MBPCG kernels (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dev_common.hpp"

namespace mb {

struct CsrDev {
    int64_t n, nnz;
    const int32_t* rowptr;
    const int32_t* colind;
    const double* vals;
};

// widths compiled into the library
inline bool width_supported(int S) { return S == 1 || S == 2 || S == 4 || S == 8 || S == 16 || S == 32; }
inline int padded_width(int s) {
    int S = 1;
    while (S < s) S *= 2;
    return S;
}
// entries of one workgroup's partial for each reduction
inline int part_entries_gram(int S) { return tri_count(S); }
inline int part_entries_update(int S) { return tri_count(S) + S; }
// double-double Gram of the termination least squares: hi and lo per entry
inline int part_entries_ls(int S) { return 2 * tri_count(S + 1); }

// tile rows of the streaming n x S kernels: 4 rows per thread
__host__ __device__ constexpr int stream_tile(int S) { return 1024 / S; }
// rows per tile of the dense reduce/Gram kernel (more workgroups for wide blocks)
__host__ __device__ constexpr int dense_reduce_rows(int S) { return S >= 16 ? 32 : 64; }

// ---- block product Q = A P (+ lower triangle of P^T Q per workgroup).
// Shape: T rows per tile, SL slots per row, V adjacent columns per lane, U
// gathers in flight per lane, W requested wavefronts per SIMD (0: the
// compiler's choice); only the compiled combinations are valid.
struct SpmmShape {
    int T = 0, SL = 0, V = 0, U = 0, W = 0;
};
hipError_t launch_spmm(int S, const SpmmShape& sh, int nwg, const CsrDev& A, const double* P,
                       double* Q, double* part, const DevState* st, hipStream_t stream);
bool spmm_valid_shape(int S, const SpmmShape& sh);
int spmm_shape_list(int S, SpmmShape* out, int cap);
SpmmShape spmm_default_shape(int S);
int spmm_lanes_per_row(int S, const SpmmShape& sh);
// workgroups of the shape's block-product kernel that fit on one CU (0 on error)
int spmm_blocks_per_cu(int S, const SpmmShape& sh);

// ---- dense product: Q partials over KSPLIT column ranges, then reduce + Gram
enum DenseKind { DENSE_F64 = 0, DENSE_F32 = 1, DENSE_BF16 = 2 };
hipError_t launch_dense_ap(int S, DenseKind kind, int64_t n, const void* A, int64_t lda,
                           const void* Plo, const double* P, double* qpart, int ksplit,
                           const DevState* st, hipStream_t stream);
int dense_ksplit(int64_t n);
int dense_nwg_rows(int64_t n);
// qpart holds FP64 partials for DENSE_F64 and FP32 partials (the matrix
// cores' FP32 accumulators) for the low-precision kinds
hipError_t launch_dense_reduce(int S, DenseKind kind, int64_t n, int ksplit, const double* qpart,
                               const double* P, double* Q, double* part, int nwg,
                               const DevState* st, hipStream_t stream);
// Low-precision operands of the dense product, stored in the matrix cores'
// operand order so that every wavefront load is one contiguous 1 KiB run:
//  A: 16-row x KS-column tiles (KS = 16 for FP32, 32 for BF16), tile (rt, kc)
//     at ((rt * ceil(n/KS) + kc) * 64 + lane) * VL elements, lane = 16 lk + li
//     holding A[16 rt + li][KS kc + VL lk + u], u < VL (VL = 4 FP32, 8 BF16);
//     rows and columns beyond n are zero.
//  P: groups of VL consecutive rows, element (k, j) at
//     (k / VL) * S * VL + j * VL + k % VL; rows are padded to a multiple of 32
//     with zeros.
__host__ __device__ constexpr int lo_vec(int kind) { return kind == DENSE_F32 ? 4 : 8; }
__host__ __device__ constexpr int lo_kstep(int kind) { return kind == DENSE_F32 ? 16 : 32; }
__host__ __device__ inline int64_t lo_pindex(int kind, int64_t k, int j, int S) {
    const int vl = lo_vec(kind);
    return (k / vl) * S * vl + (int64_t)j * vl + k % vl;
}
__host__ __device__ inline int64_t lo_rows_padded(int64_t n) { return (n + 31) / 32 * 32; }
size_t dense_lo_bytes(DenseKind kind, int64_t n);
// FP64 column-major A -> the tiled low-precision layout, round to nearest even
hipError_t launch_cast_dense(DenseKind kind, int64_t n, const double* A, int64_t lda, void* out,
                             hipStream_t stream);
// r = b - (sum of the ksplit partials of A x) and partial sums of r^2 (S = 1)
hipError_t launch_dense_resid_reduce(int64_t n, int ksplit, const double* qpart, const double* b,
                                     double* r_out, double* part, int nwg, hipStream_t stream);

// ---- block-Jacobi preconditioner (the preconditioned form of Sec. 2)
// M = diagonal blocks of bs consecutive rows of the scaled matrix; inv holds
// M^-1 row by row: inv[r * bs + c] = (block inverse)[r - lo][c], lo = r / bs * bs,
// zero for columns beyond n.  bs = 0 means no preconditioner.
inline bool bjac_supported(int bs) { return bs == 4 || bs == 8 || bs == 16 || bs == 32; }
struct BjArgs {
    int bs = 0;               // 0: none
    const double* inv = nullptr;
    double* Y = nullptr;      // n x S output M^-1 V (or M^-1 r for CG)
};
// inv from the CSR (A.vals = scaled values) or dense column-major matrix;
// a block that is not SPD sets st->done = DONE_NOTSPD
hipError_t launch_bjac_setup_csr(int bs, const CsrDev& A, double* inv, DevState* st,
                                 hipStream_t s);
hipError_t launch_bjac_setup_dense(int bs, int64_t n, const double* A, int64_t lda, double* inv,
                                   DevState* st, hipStream_t s);

// ---- fused updates of one iteration
// With bj.bs: also Y = M^-1 V into bj.Y and the Gram V^T Y (entry (i >= j) =
// V_i^T Y_j) instead of V^T V.
hipError_t launch_update(int S, int nwg, int64_t n, const double* P, const double* Q, double* Xt,
                         double* R, double* W, const double* d, double* part, const DevState* st,
                         hipStream_t stream, const BjArgs& bj = BjArgs());
// With Yp (the preconditioned path, FP64 only): W = V M and P = Yp M + P Z^T.
// Xt: X~, which the non-first direction update advances by P alpha for
// S <= 16 (the update kernel does it at S = 32).
hipError_t launch_dirupdate(int S, int nwg, int64_t n, double* W, double* P, void* Plo,
                            DenseKind lo_kind, int first, const DevState* st, hipStream_t stream,
                            const double* Yp, double* Xt);

// workgroups of k_update<S, 0> / k_dirupdate<S, 0, DENSE_F64, 0> per CU (0 on error)
int update_blocks_per_cu(int S);
int dirupdate_blocks_per_cu(int S);

// ---- setup
hipError_t launch_diag_csr(const CsrDev& A, int jacobi, double* d, DevState* st, hipStream_t s);
hipError_t launch_diag_dense(int64_t n, const double* A, int64_t lda, int jacobi, double* d,
                             DevState* st, hipStream_t s);
hipError_t launch_scale_csr(const CsrDev& A, const double* d, double* vals_s, hipStream_t s);
hipError_t launch_scale_dense(int64_t n, const double* A, int64_t lda, const double* d, double* As,
                              hipStream_t s);
hipError_t launch_rhs(int nwg, int64_t n, const double* b, const double* d, double* bbar,
                      double* part, hipStream_t s);
hipError_t launch_uniform(int S, int64_t n, int s, uint64_t seed, double* U, hipStream_t st);
hipError_t launch_pad_block(int S, int64_t n, int s, const double* Uin, double* U, hipStream_t st);
hipError_t launch_ynorm(int S, int nwg, int64_t n, const double* Y, double* part, hipStream_t s);
hipError_t launch_init(int S, int64_t n, int s, const double* U, const double* Y,
                       const double* bbar, double* X0, double* Xt, double* R, const DevState* st,
                       hipStream_t stream);
hipError_t launch_gram_nu(int S, int nwg, int64_t n, const double* X, const double* d, double* part,
                          hipStream_t stream, const BjArgs& bj = BjArgs());

// ---- termination
hipError_t launch_ls_gram(int S, int nwg, int64_t n, const double* b, const double* R,
                          const double* d, double* part, const DevState* st, hipStream_t s);
hipError_t launch_ls_apply(int S, int nwg, int64_t n, const double* Xt, const double* X0,
                           const double* R, const double* b, const double* d, double* x,
                           double* part, const DevState* st, hipStream_t s);
hipError_t launch_select(int S, int64_t n, const double* Xt, const double* X0, const double* d,
                         double* x, const DevState* st, int force, hipStream_t s);
hipError_t launch_resid_csr(int nwg, const CsrDev& A, const double* b, const double* x,
                            double* part, hipStream_t s);

// ---- Chronopoulos-Gear CG
hipError_t launch_cg_init(int64_t n, const double* bbar, double* x, double* r, double* p,
                          double* sv, hipStream_t s);
// With bj.bs: p = u + beta p with u = M^-1 r (bj.Y), then the new u from the new
// r; partials (||D r||^2, r^T u) instead of (||D r||^2, r^T r)
hipError_t launch_cg_update(int nwg, int64_t n, double* p, double* sv, double* x, double* r,
                            const double* w, const double* d, double* part, const DevState* st,
                            hipStream_t s, const BjArgs& bj = BjArgs());
// u = M^-1 r into bj.Y and partials (||D r||^2, r^T u) (the preconditioned CG start)
hipError_t launch_cg_prec(int nwg, int64_t n, const double* r, const double* d, double* part,
                          const BjArgs& bj, hipStream_t s);
hipError_t launch_unscale(int64_t n, const double* xs, const double* d, double* x, hipStream_t s);
// out (n x s row-major) = X~ + X0 (n x S blocks), the block iterate at exit
hipError_t launch_export_x(int S, int64_t n, int s, const double* Xt, const double* X0, double* out,
                           hipStream_t st);

// ---- tails (one workgroup): reductions of partials + s x s FP64 work
hipError_t launch_tail_gamma(int nwg_b, const double* part_b, int nwg_y, const double* part_y,
                             DevState* st, hipStream_t s);
// first stage of a two-stage partial sum: nwg partials of E entries (stride E)
// -> G partials in out (stride E); E <= PART_REDUCE_EMAX
constexpr int PART_REDUCE_EMAX = 1024;
constexpr int PART_REDUCE_G = 32;
hipError_t launch_part_reduce(int nwg, int E, const double* part, double* out, int G,
                              const DevState* st, hipStream_t s);
hipError_t launch_tail_xi(int S, int nwg, const double* part, DevState* st, hipStream_t s);
hipError_t launch_tail_qr(int S, int nwg, const double* part, DevState* st, double* hist,
                          int setup, hipStream_t s);
hipError_t launch_tail_ls(int S, int nwg, int64_t n, const double* part, DevState* st,
                          hipStream_t s);
hipError_t launch_tail_accept(int nwg, const double* part, DevState* st, hipStream_t s);
hipError_t launch_tail_true(int nwg, const double* part, DevState* st, hipStream_t s);
hipError_t launch_tail_pick(int nwg, const double* part, DevState* st, hipStream_t s);
hipError_t launch_tail_cg0(int nwg_b, const double* part_b, int nwg_s, const double* part_s,
                           DevState* st, hipStream_t s);
hipError_t launch_tail_cg(int nwg_u, const double* part_u, int nwg_s, const double* part_s,
                          DevState* st, double* hist, hipStream_t s);
hipError_t launch_state_init(DevState* st, int s, int max_iter, double tol, double tol0,
                             double tau, int n_hist, hipStream_t stream);

// n x S block -> the low-precision P layout (padding rows zero)
hipError_t launch_block_to_lo(DenseKind kind, int64_t n, int S, const double* src, void* dst,
                             hipStream_t s);
hipError_t launch_axpy_ir(int64_t n, double* x, const double* d, double alpha, hipStream_t s);
// sqrt of a reduced sum of squares into st->res_norm
hipError_t launch_tail_norm(int nwg, const double* part, DevState* st, hipStream_t s);
// reduce Gram partials (lower triangle) into C (S x S row-major, i >= j)
hipError_t launch_gram_out(int S, int nwg, const double* part, double* C, hipStream_t s);

// plain streaming copy (byte-counter calibration)
hipError_t launch_stream_copy(void* dst, const void* src, int64_t bytes, hipStream_t s);

}  // namespace mb

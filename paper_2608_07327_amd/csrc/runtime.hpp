// Host runtime of the MBPCG library: the context, its device buffers and the
// drivers of Algorithm 1, of the CG baseline and of the FP64 iterative
// refinement around a low-precision inner solve.
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/mbpcg.h"
#include "kernels.hpp"

namespace mb {

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

struct Tuning {
    SpmmShape sh;  // tile shape of the sparse block product (T = 0: not tuned)
    int nwg = 0;   // workgroups of the block product
};

struct Ctx {
    // problem
    int dense = 0;
    int64_t n = 0, nnz = 0;
    int device = 0;
    int cus = 0;                   // compute units of the device
    hipStream_t user_stream = nullptr;
    hipStream_t stream = nullptr;  // private, non-blocking
    std::string err;

    // matrix (device)
    int32_t* rowptr = nullptr;
    int32_t* colind = nullptr;
    double* vals = nullptr;     // original values (true residual)
    double* vals_s = nullptr;   // scaled values
    double* A = nullptr;        // dense original, column-major, lda = n
    double* As = nullptr;       // dense scaled (== A when no scaling)
    void* Alo = nullptr;        // dense low-precision copy in the tiled operand layout
    DenseKind alo_kind = DENSE_F64;
    int scaled_jacobi = -1;     // which scaling vals_s / As hold

    // vectors
    double* d = nullptr;
    double* bbar = nullptr;
    double* bdev = nullptr;
    double* xdev = nullptr;
    double* rvec = nullptr;     // IR residual
    double* xacc = nullptr;     // IR accumulated solution
    double* bjinv = nullptr;    // block-Jacobi inverse rows, n x bjinv_bs
    int bjinv_bs = 0;

    // blocks, capacity Scap columns
    int Scap = 0;
    double *U = nullptr, *Y = nullptr, *X0 = nullptr, *Xt = nullptr, *R = nullptr, *W = nullptr,
           *P = nullptr, *Q = nullptr;
    void* Plo = nullptr;
    double* qpart = nullptr;    // dense split-K partials
    int64_t qpart_elems = 0;

    // reductions
    double* part_a = nullptr;
    double* part_b = nullptr;
    double* part_r = nullptr;   // first stage of a two-stage partial sum
    double* part_c = nullptr;
    int64_t part_elems = 0;
    DevState* st = nullptr;
    double* hist = nullptr;
    int64_t hist_cap = 0;
    int32_t* pinned = nullptr;  // 2 x {done, iter}
    DevState* st_host = nullptr;
    hipEvent_t ev_poll[2] = {nullptr, nullptr};
    hipEvent_t ev_a = nullptr, ev_b = nullptr, ev_user = nullptr;
    std::vector<hipEvent_t> pev;  // profile mode: 6 events per iteration
    double phase_ms[8] = {0, 0, 0, 0, 0, 0, 0, 0};

    // graphs keyed by (kind, S, m, tile shape, nwg, precision)
    std::map<std::tuple<int, int, int, int, int, int>, hipGraphExec_t> graphs;
    std::map<int, Tuning> tune;  // per S

    ~Ctx();
};

}  // namespace mb

struct mbpcg_ctx_s {
    mb::Ctx c;
};

// Batched solves of independent densities of different sizes (gfx950).
//
// Each member of a batch is a complete solve with its own plan tables (shared
// between members of equal parameters) and its own workspace.  Instead of five
// launches per member, every stage is one launch over a work table that lists
// the blocks of all members, largest members first: a block reads its entry,
// its member's device plan, and runs the same body as the single-solve kernel
// at that member's transform length.  All blocks have 256 threads, so a length
// F = 2^LOG transform (F/16 threads) takes 4096/F rows or columns per block.
//
// Stage order (as in a single solve, the node side runs on the plan's second
// stream beside the I1 columns):
//   rows_forward   every member's rows                       (DIR)
//   cols_type2     every member's type-2 window columns      (DIR)
//   side stream:   nodes (every member's subproblems: interp, q_j h^2, spread),
//                  then cols_type1 (every member's window columns, -DIR)
//   cols           I1 spectrum columns (g1 multiplier and inverse), then those
//                  of the members with the mixed multiplier
//   after both:    rows_inverse, every member's rows         (-DIR)
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "solver_device.hpp"

namespace phi {

namespace {

// LDS of a batched FFT block: the largest G x padded transform over the lengths
constexpr int batch_lds_entries() {
    int m = 0;
    for (int lg = kBatchMinLogFine; lg <= kBatchMaxLogFine; ++lg) {
        const int e = batch_lines(lg) * lds_group_stride(1 << lg);
        m = e > m ? e : m;
    }
    return m;
}
constexpr int kBatchLds = batch_lds_entries();

static_assert(FftShape<kBatchMaxLogFine>::NT * batch_lines(kBatchMaxLogFine) == kBatchThreads,
              "batched blocks hold whole transforms");
static_assert(FftShape<kBatchMinLogFine>::NT * batch_lines(kBatchMinLogFine) == kBatchThreads,
              "batched blocks hold whole transforms");
static_assert(kNodeThreads == kBatchThreads, "node blocks have the batched block size");

// Calls BODY with a compile-time length LOG_ for the member's fine-grid side.
#define PHI_BATCH_LOG(LOGV, BODY)                                        \
    switch (LOGV) {                                                      \
        case 8: { constexpr int LOG_ = 8; BODY; break; }                 \
        case 9: { constexpr int LOG_ = 9; BODY; break; }                 \
        case 10: { constexpr int LOG_ = 10; BODY; break; }               \
        case 11: { constexpr int LOG_ = 11; BODY; break; }               \
        case 12: { constexpr int LOG_ = 12; BODY; break; }               \
        default: break;                                                  \
    }

template <typename R, int DIR>
__global__ __launch_bounds__(kBatchThreads) void kb_rows_forward(BatchDev B, const R* __restrict__ in) {
    __shared__ cpx<R> lds_all[kBatchLds];
    const WorkItem w = B.rows[xcd_logical_block(blockIdx.x, gridDim.x)];
    const DevPlan P = B.members[w.member];
    const R* rho = in + B.offsets[w.member];
    // members whose side is F/2 take the exact-bounds body (a uniform branch)
    if (2 * P.n == P.n_fine) {
        PHI_BATCH_LOG(P.log_fine, (rows_forward_body<R, LOG_, DIR, batch_lines(LOG_), true>(P, rho, w.item, lds_all)));
    } else {
        PHI_BATCH_LOG(P.log_fine, (rows_forward_body<R, LOG_, DIR, batch_lines(LOG_), false>(P, rho, w.item, lds_all)));
    }
}

// A launch over one column list: I1 spectrum columns (kind 0) or type-2 window
// columns (kind 1).  MIXED: the list of I1 columns of the members with the mixed
// multiplier (an instantiation of its own, so the other members' code is
// unchanged).
template <typename R, int DIR, bool MIXED>
__global__ __launch_bounds__(kBatchThreads) void kb_cols(BatchDev B, const WorkItem* __restrict__ list) {
    __shared__ cpx<R> lds_all[kBatchLds];
    const WorkItem w = list[xcd_logical_block(blockIdx.x, gridDim.x)];
    const DevPlan P = B.members[w.member];
    if (w.kind == 0 && 2 * P.n == P.n_fine) {
        PHI_BATCH_LOG(P.log_fine, (cols_highfreq_body<R, LOG_, DIR, batch_lines(LOG_),
                                                    MIXED ? kKindMixed : kKindQuadratic, true>(P, w.item, lds_all)));
    } else if (w.kind == 0) {
        PHI_BATCH_LOG(P.log_fine, (cols_highfreq_body<R, LOG_, DIR, batch_lines(LOG_),
                                                    MIXED ? kKindMixed : kKindQuadratic, false>(P, w.item, lds_all)));
    } else {
        PHI_BATCH_LOG(P.log_fine, (cols_type2_body<R, LOG_, DIR, batch_lines(LOG_), false>(P, w.item, lds_all)));
    }
}

template <typename R, int WMAX>
__global__ __launch_bounds__(kBatchThreads) void kb_nodes(BatchDev B) {
    __shared__ NodeLds<R, WMAX> s;
    const WorkItem w = B.nodes[blockIdx.x];
    const DevPlan P = B.members[w.member];
    nodes_body<R, 0, kNodeThreads, WMAX>(P, w.item, nullptr, nullptr, s);
}

template <typename R, int DIR>
__global__ __launch_bounds__(kBatchThreads) void kb_cols_type1(BatchDev B) {
    __shared__ cpx<R> lds_all[kBatchLds];
    const WorkItem w = B.cols1[blockIdx.x];
    const DevPlan P = B.members[w.member];
    PHI_BATCH_LOG(P.log_fine,
                  (cols_type1_body<R, LOG_, DIR, batch_lines(LOG_), batch_lines(LOG_), false>(P, w.item, lds_all)));
}

template <typename R, int DIR>
__global__ __launch_bounds__(kBatchThreads) void kb_rows_inverse(BatchDev B, R* __restrict__ out) {
    __shared__ cpx<R> lds_all[kBatchLds];
    const WorkItem w = B.rows[xcd_logical_block(blockIdx.x, gridDim.x)];
    const DevPlan P = B.members[w.member];
    R* dst = out + B.offsets[w.member];
    if (2 * P.n == P.n_fine) {
        PHI_BATCH_LOG(P.log_fine,
                      (rows_inverse_body<R, LOG_, DIR, true, true, batch_lines(LOG_), true>(P, dst, w.item, lds_all)));
    } else {
        PHI_BATCH_LOG(P.log_fine,
                      (rows_inverse_body<R, LOG_, DIR, true, true, batch_lines(LOG_), false>(P, dst, w.item, lds_all)));
    }
}

#define PHI_TRY_B(expr)                  \
    do {                                 \
        hipError_t e_ = (expr);          \
        if (e_ != hipSuccess) return e_; \
    } while (0)

#define PHI_LAUNCH_B(name, count, strm, launch)                    \
    do {                                                           \
        if ((count) > 0) {                                         \
            PHI_TRY_B(mark_kernel(timer, name, false, strm));      \
            launch;                                                \
            PHI_TRY_B(hipGetLastError());                          \
            PHI_TRY_B(mark_kernel(timer, name, true, strm));       \
        }                                                          \
    } while (0)

template <typename R, int DIR>
hipError_t enqueue_batch_dir(const BatchDev& B, const StreamSet& ss, const void* in, void* out, hipStream_t s,
                             KernelTimer* timer) {
    const dim3 blk(kBatchThreads);
    PHI_LAUNCH_B("rows_forward", B.n_rows, s,
                 PHI_LAUNCH((kb_rows_forward<R, DIR>), dim3(B.n_rows), blk, 0, s, B,
                                    static_cast<const R*>(in)));
    PHI_LAUNCH_B("cols_type2", B.n_cols_t2, s,
                 PHI_LAUNCH((kb_cols<R, DIR, false>), dim3(B.n_cols_t2), blk, 0, s, B, B.cols_t2));
    hipStream_t side = ss.side ? ss.side : s;
    if (ss.side) {
        PHI_TRY_B(hipEventRecord(ss.fork, s));
        PHI_TRY_B(hipStreamWaitEvent(side, ss.fork, 0));
    }
    if (B.wide_kernel)
        PHI_LAUNCH_B("nodes", B.n_nodes, side,
                     PHI_LAUNCH((kb_nodes<R, kMaxKernelWidth>), dim3(B.n_nodes), blk, 0, side, B));
    else
        PHI_LAUNCH_B("nodes", B.n_nodes, side,
                     PHI_LAUNCH((kb_nodes<R, kMaxEsWidth>), dim3(B.n_nodes), blk, 0, side, B));
    PHI_LAUNCH_B("cols_type1", B.n_cols1, side,
                 PHI_LAUNCH((kb_cols_type1<R, -DIR>), dim3(B.n_cols1), blk, 0, side, B));
    if (ss.side) PHI_TRY_B(hipEventRecord(ss.join, side));
    PHI_LAUNCH_B("cols", B.n_cols, s,
                 PHI_LAUNCH((kb_cols<R, DIR, false>), dim3(B.n_cols), blk, 0, s, B, B.cols));
    PHI_LAUNCH_B("cols_mixed", B.n_cols_mixed, s,
                 PHI_LAUNCH((kb_cols<R, DIR, true>), dim3(B.n_cols_mixed), blk, 0, s, B, B.cols_mixed));
    if (ss.side) PHI_TRY_B(hipStreamWaitEvent(s, ss.join, 0));
    PHI_LAUNCH_B("rows_inverse", B.n_rows, s,
                 PHI_LAUNCH((kb_rows_inverse<R, -DIR>), dim3(B.n_rows), blk, 0, s, B, static_cast<R*>(out)));
    return hipSuccess;
}

}  // namespace

hipError_t enqueue_batch(const BatchDev& B, const StreamSet& ss, const void* in, void* out, int adjoint,
                         hipStream_t s, KernelTimer* timer) {
    // forward solve: first transforms with e^{-...}; the transposed solve reverses them
    if (B.dtype == PHI_F32) {
        return adjoint ? enqueue_batch_dir<float, 1>(B, ss, in, out, s, timer)
                       : enqueue_batch_dir<float, -1>(B, ss, in, out, s, timer);
    }
    return adjoint ? enqueue_batch_dir<double, 1>(B, ss, in, out, s, timer)
                   : enqueue_batch_dir<double, -1>(B, ss, in, out, s, timer);
}

}  // namespace phi

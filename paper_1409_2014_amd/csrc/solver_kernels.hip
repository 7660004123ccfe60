// HIP kernels of the split potential solve for gfx950 (see phi_solve.h).
//
// N = grid side (even), F = the side of both the zero-padded I1 box and the
// NUFFT fine grid (the smallest power of two >= kappa N, so F >= 2N), Q = side
// of the fine-grid window around frequency 0 that the polar nodes' kernel taps
// touch, M = number of polar nodes, w = kernel width.
// A solve runs six kernels; the node-side chain runs on a second stream
// concurrently with the I1 column pass:
//
//   rows_forward   per grid row: z = rho + i rho d(n1) d(n2) at centred
//                  positions, one F-point FFT; the transform of the real part
//                  on m = 0..F/2 (I1 half spectrum) goes to the column-major XT,
//                  that of the imaginary part on the Q window frequencies (the
//                  type-2 row window) to TT.   [Sec. 2.1 eq. (9); Sec. 2.2 eq. (16)]
//   cols_highfreq  per spectrum column: F-point FFT, times g1(k)/F^2, inverse
//                  FFT, the N centred rows back into XT.            [eq. (9)]
//   side stream:
//   cols_type2     per window column of TT: F-point FFT, the Q window rows -> WIN.
//   nodes          per subproblem (<= 64 nodes of one bin): stage the window
//                  tile and the nodes' precomputed kernel taps in LDS,
//                  interpolate c_j, a_j = q_j h^2 c_j, spread the a_j into the
//                  subproblem's own tile (no atomics).  [eq. (12), (15), (16)]
//   cols_type1     per window column: sum the tile entries of each cell in a
//                  fixed order, F-point FFT (only the Q window inputs are
//                  non-zero), the N centred rows times d(n2) -> U.
//   main stream, after both:
//   rows_inverse   per grid row: the Hermitian I1 row spectrum plus i times the
//                  Hermitian part of the type-1 row, one F-point FFT;
//                  Phi = Re + Im d(n1).                 [eq. (8): Phi = I1 + Re I2]
//
// The transposed solve runs the same kernels with every FFT direction reversed.
//
// One-stream layout (the default on padded sides up to 1024, and 2048 in FP32;
// shared_kernels.hip): rows_forward, cols_type2, nodes, then one launch of the
// type-1 window columns together with every I1 spectrum column, then
// rows_inverse, all on the solve's stream.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "solver_device.hpp"

namespace phi {

// ---------------------------------------------------------------------------
// Single-solve kernels: one work item per block
// ---------------------------------------------------------------------------
// The row kernels come in two widths: rows_per_block rows per block, and one
// wave per block (rows_per_wave) for grids with fewer rows than it takes to give
// every CU a wide block; the rows' arithmetic is the same in both.
template <typename R, int LOG>
constexpr int rows_per_wave() {
    constexpr int nt = FftShape<LOG>::NT;
    constexpr int g = nt >= 64 ? 1 : 64 / nt;
    return g < rows_per_block<R, LOG>() ? g : rows_per_block<R, LOG>();
}
constexpr int kRowsWideMinBlocks = 256;   // one wide block per CU at least, else the narrow width

template <typename R, int LOG, int DIR, bool EXACT, int G>
__global__ __launch_bounds__((FftShape<LOG>::NT * G)) void k_rows_forward(DevPlan P, const R* __restrict__ rho) {
    __shared__ cpx<R> lds_all[G * lds_group_stride(1 << LOG)];
    rows_forward_body<R, LOG, DIR, G, EXACT>(P, rho, xcd_logical_block(blockIdx.x, gridDim.x) * G, lds_all);
}

template <typename R, int LOG, int DIR, int KIND, bool EXACT>
__global__ __launch_bounds__(FftShape<LOG>::NT * lines_per_block<LOG>()) void k_cols_highfreq(DevPlan P) {
    constexpr int G = lines_per_block<LOG>();
    __shared__ cpx<R> lds_all[G * lds_group_stride(1 << LOG)];
    cols_highfreq_body<R, LOG, DIR, G, KIND, EXACT>(P, xcd_logical_block(blockIdx.x, gridDim.x) * G, lds_all);
}

// one window column per block: the Q columns are few, so at small N blocks of
// several columns would leave most of the chip idle on this critical path
template <typename R, int LOG, int DIR>
__global__ __launch_bounds__(FftShape<LOG>::NT) void k_cols_type2(DevPlan P) {
    __shared__ cpx<R> lds_all[lds_group_stride(1 << LOG)];
    cols_type2_body<R, LOG, DIR, 1, false>(P, blockIdx.x, lds_all);
}

template <typename R, int MODE, int WMAX, int W>
__global__ __launch_bounds__(kNodeThreadsSingle) void k_nodes(DevPlan P, const cpx<R>* __restrict__ coef,
                                                        cpx<R>* __restrict__ out) {
    __shared__ NodeLds<R, WMAX> s;
    nodes_body<R, MODE, kNodeThreadsSingle, WMAX, W>(P, blockIdx.x, coef, out, s);
}

template <typename R, int LOG, int DIR>
__global__ __launch_bounds__(FftShape<LOG>::NT * lines_per_block<LOG>()) void k_cols_type1(DevPlan P) {
    constexpr int G = lines_per_block<LOG>();
    __shared__ cpx<R> lds_all[G * lds_group_stride(1 << LOG)];
    cols_type1_body<R, LOG, DIR, G, 1, false>(P, blockIdx.x, lds_all);
}

template <typename R, int LOG, int DIR, bool USE_I1, bool USE_I2, bool EXACT, int G>
__global__ __launch_bounds__((FftShape<LOG>::NT * G)) void k_rows_inverse(DevPlan P, R* __restrict__ out) {
    __shared__ cpx<R> lds_all[G * lds_group_stride(1 << LOG)];
    rows_inverse_body<R, LOG, DIR, USE_I1, USE_I2, G, EXACT>(P, out, xcd_logical_block(blockIdx.x, gridDim.x) * G,
                                                             lds_all);
}

// ---------------------------------------------------------------------------
// Host-side launchers
// ---------------------------------------------------------------------------
namespace {

template <typename R, int LOG, int DIR, int G>
hipError_t launch_rows_forward_g(const DevPlan& P, const R* src, hipStream_t s) {
    constexpr int block = FftShape<LOG>::NT * G;
    const int grid = (P.n + G - 1) / G;   // one work item per block
    if (2 * P.n == P.n_fine) PHI_LAUNCH((k_rows_forward<R, LOG, DIR, true, G>), dim3(grid), dim3(block), 0, s, P, src);
    else PHI_LAUNCH((k_rows_forward<R, LOG, DIR, false, G>), dim3(grid), dim3(block), 0, s, P, src);
    return hipGetLastError();
}

template <typename R, int LOG, int DIR>
hipError_t launch_rows_forward_dir(const DevPlan& P, const R* src, hipStream_t s) {
    constexpr int GW = rows_per_block<R, LOG>();
    if ((P.n + GW - 1) / GW < kRowsWideMinBlocks)
        return launch_rows_forward_g<R, LOG, DIR, rows_per_wave<R, LOG>()>(P, src, s);
    return launch_rows_forward_g<R, LOG, DIR, GW>(P, src, s);
}

template <typename R, int LOG>
hipError_t launch_rows_forward(const DevPlan& P, const void* rho, int dir, hipStream_t s) {
    const R* src = static_cast<const R*>(rho);
    return dir < 0 ? launch_rows_forward_dir<R, LOG, -1>(P, src, s) : launch_rows_forward_dir<R, LOG, 1>(P, src, s);
}

template <typename R, int LOG, int DIR>
hipError_t launch_cols_highfreq_dir(const DevPlan& P, hipStream_t s) {
    constexpr int G = lines_per_block<LOG>();
    constexpr int block = FftShape<LOG>::NT * G;
    const int items = (P.n_fine / 2 + 1 + G - 1) / G;
    const int grid = items;   // one work item per block
    // the exact-bounds variants are taken wherever the batched kernels take them
    // (the DS, y and mixed multipliers), so a batch member and its single plan
    // run the same code; the Coulomb multipliers use the general bounds only
    const bool exact = 2 * P.n == P.n_fine;
    if (P.component == 2 && exact)
        PHI_LAUNCH((k_cols_highfreq<R, LOG, DIR, kKindMixed, true>), dim3(grid), dim3(block), 0, s, P);
    else if (P.component == 2)
        PHI_LAUNCH((k_cols_highfreq<R, LOG, DIR, kKindMixed, false>), dim3(grid), dim3(block), 0, s, P);
    else if (P.component == 3 && P.partition_erfc)
        PHI_LAUNCH((k_cols_highfreq<R, LOG, DIR, kKindCoulombErfc, false>), dim3(grid), dim3(block), 0, s, P);
    else if (P.component == 3)
        PHI_LAUNCH((k_cols_highfreq<R, LOG, DIR, kKindCoulombGauss, false>), dim3(grid), dim3(block), 0, s, P);
    else if (exact)
        PHI_LAUNCH((k_cols_highfreq<R, LOG, DIR, kKindQuadratic, true>), dim3(grid), dim3(block), 0, s, P);
    else
        PHI_LAUNCH((k_cols_highfreq<R, LOG, DIR, kKindQuadratic, false>), dim3(grid), dim3(block), 0, s, P);
    return hipGetLastError();
}

template <typename R, int LOG>
hipError_t launch_cols_highfreq(const DevPlan& P, int dir, hipStream_t s) {
    return dir < 0 ? launch_cols_highfreq_dir<R, LOG, -1>(P, s) : launch_cols_highfreq_dir<R, LOG, 1>(P, s);
}

template <typename R, int LOG>
hipError_t launch_cols_type2(const DevPlan& P, int dir, hipStream_t s) {
    const int blocks = P.patch;
    if (dir < 0) PHI_LAUNCH((k_cols_type2<R, LOG, -1>), dim3(blocks), dim3(FftShape<LOG>::NT), 0, s, P);
    else PHI_LAUNCH((k_cols_type2<R, LOG, 1>), dim3(blocks), dim3(FftShape<LOG>::NT), 0, s, P);
    return hipGetLastError();
}

template <typename R, int LOG>
hipError_t launch_cols_type1(const DevPlan& P, int dir, hipStream_t s) {
    constexpr int G = lines_per_block<LOG>();
    const int blocks = P.patch;   // one window column per block
    if (dir < 0) PHI_LAUNCH((k_cols_type1<R, LOG, -1>), dim3(blocks), dim3(FftShape<LOG>::NT * G), 0, s, P);
    else PHI_LAUNCH((k_cols_type1<R, LOG, 1>), dim3(blocks), dim3(FftShape<LOG>::NT * G), 0, s, P);
    return hipGetLastError();
}

template <typename R, int LOG, int DIR, bool I1, bool I2, int G>
hipError_t launch_rows_inverse_g(const DevPlan& P, R* dst, hipStream_t s) {
    constexpr int block = FftShape<LOG>::NT * G;
    const int grid = (P.n + G - 1) / G;   // one work item per block
    // the full solve (I1 and I2) has an exact-bounds variant; the stage variants use the general one
    if (I1 && I2 && 2 * P.n == P.n_fine)
        PHI_LAUNCH((k_rows_inverse<R, LOG, DIR, I1, I2, I1 && I2, G>), dim3(grid), dim3(block), 0, s, P, dst);
    else
        PHI_LAUNCH((k_rows_inverse<R, LOG, DIR, I1, I2, false, G>), dim3(grid), dim3(block), 0, s, P, dst);
    return hipGetLastError();
}

template <typename R, int LOG, int DIR, bool I1, bool I2>
hipError_t launch_rows_inverse_parts(const DevPlan& P, R* dst, hipStream_t s) {
    constexpr int GW = rows_per_block<R, LOG>();
    if ((P.n + GW - 1) / GW < kRowsWideMinBlocks)
        return launch_rows_inverse_g<R, LOG, DIR, I1, I2, rows_per_wave<R, LOG>()>(P, dst, s);
    return launch_rows_inverse_g<R, LOG, DIR, I1, I2, GW>(P, dst, s);
}

template <typename R, int LOG, int DIR>
hipError_t launch_rows_inverse_dir(const DevPlan& P, R* dst, int use_i1, int use_i2, hipStream_t s) {
    if (use_i1 && use_i2) return launch_rows_inverse_parts<R, LOG, DIR, true, true>(P, dst, s);
    if (use_i1) return launch_rows_inverse_parts<R, LOG, DIR, true, false>(P, dst, s);
    if (use_i2) return launch_rows_inverse_parts<R, LOG, DIR, false, true>(P, dst, s);
    return hipErrorInvalidValue;
}

template <typename R, int LOG>
hipError_t launch_rows_inverse(const DevPlan& P, void* out, int dir, int use_i1, int use_i2, hipStream_t s) {
    R* dst = static_cast<R*>(out);
    if (dir < 0) return launch_rows_inverse_dir<R, LOG, -1>(P, dst, use_i1, use_i2, s);
    return launch_rows_inverse_dir<R, LOG, 1>(P, dst, use_i1, use_i2, s);
}

template <int LOG>
bool twiddles_match(const DevPlan& P) {
    return P.twr_count == FftShape<LOG>::tw_size();
}

#define PHI_DISPATCH_LOG(LOGV, CALL)                     \
    switch (LOGV) {                                      \
        case 4: { constexpr int L_ = 4; return CALL; }   \
        case 5: { constexpr int L_ = 5; return CALL; }   \
        case 6: { constexpr int L_ = 6; return CALL; }   \
        case 7: { constexpr int L_ = 7; return CALL; }   \
        case 8: { constexpr int L_ = 8; return CALL; }   \
        case 9: { constexpr int L_ = 9; return CALL; }   \
        case 10: { constexpr int L_ = 10; return CALL; } \
        case 11: { constexpr int L_ = 11; return CALL; } \
        case 12: { constexpr int L_ = 12; return CALL; } \
        case 13: { constexpr int L_ = 13; return CALL; } \
        default: return hipErrorInvalidValue;            \
    }

hipError_t check_twiddles(const DevPlan& P) {
    PHI_DISPATCH_LOG(P.log_fine, (twiddles_match<L_>(P) ? hipSuccess : hipErrorInvalidValue));
}
template <typename R>
hipError_t run_rows_forward(const DevPlan& P, const void* rho, int dir, hipStream_t s) {
    PHI_DISPATCH_LOG(P.log_fine, (launch_rows_forward<R, L_>(P, rho, dir, s)));
}
template <typename R>
hipError_t run_cols_highfreq(const DevPlan& P, int dir, hipStream_t s) {
    PHI_DISPATCH_LOG(P.log_fine, (launch_cols_highfreq<R, L_>(P, dir, s)));
}
template <typename R>
hipError_t run_cols_type2(const DevPlan& P, int dir, hipStream_t s) {
    PHI_DISPATCH_LOG(P.log_fine, (launch_cols_type2<R, L_>(P, dir, s)));
}
template <typename R>
hipError_t run_cols_type1(const DevPlan& P, int dir, hipStream_t s) {
    PHI_DISPATCH_LOG(P.log_fine, (launch_cols_type1<R, L_>(P, dir, s)));
}
template <typename R>
hipError_t run_rows_inverse(const DevPlan& P, void* out, int dir, int use_i1, int use_i2, hipStream_t s) {
    PHI_DISPATCH_LOG(P.log_fine, (launch_rows_inverse<R, L_>(P, out, dir, use_i1, use_i2, s)));
}

template <typename R, int MODE>
hipError_t run_nodes(const DevPlan& P, const void* coef, void* out, hipStream_t s) {
    const dim3 grid(P.n_sub), block(kNodeThreadsSingle);
    const cpx<R>* c = static_cast<const cpx<R>*>(coef);
    cpx<R>* o = static_cast<cpx<R>*>(out);
    // the node stage of a solve takes its kernel width as a template argument
    // whenever the width fits the ES tap store (every ES kernel, narrow Gaussians)
#define PHI_NODES_W(WV) \
    case WV: PHI_LAUNCH((k_nodes<R, MODE, kMaxEsWidth, WV>), grid, block, 0, s, P, c, o); break;
    static_assert(kMaxEsWidth == 16, "one case per ES width");
    if constexpr (MODE == 0) {
        if (P.width <= kMaxEsWidth) {
            switch (P.width) {
                PHI_NODES_W(2) PHI_NODES_W(3) PHI_NODES_W(4) PHI_NODES_W(5) PHI_NODES_W(6) PHI_NODES_W(7)
                PHI_NODES_W(8) PHI_NODES_W(9) PHI_NODES_W(10) PHI_NODES_W(11) PHI_NODES_W(12) PHI_NODES_W(13)
                PHI_NODES_W(14) PHI_NODES_W(15) PHI_NODES_W(16)
                default: PHI_LAUNCH((k_nodes<R, MODE, kMaxEsWidth, 0>), grid, block, 0, s, P, c, o); break;
            }
            return hipGetLastError();
        }
    }
    if (P.width > kMaxEsWidth) {
        PHI_LAUNCH((k_nodes<R, MODE, kMaxKernelWidth, 0>), grid, block, 0, s, P, c, o);
    } else {
        PHI_LAUNCH((k_nodes<R, MODE, kMaxEsWidth, 0>), grid, block, 0, s, P, c, o);
    }
#undef PHI_NODES_W
    return hipGetLastError();
}

#define PHI_TRY(expr)                    \
    do {                                 \
        hipError_t e_ = (expr);          \
        if (e_ != hipSuccess) return e_; \
    } while (0)

#define PHI_STEP(name, stream, expr)                         \
    do {                                                     \
        PHI_TRY(mark_kernel(timer, name, false, stream));    \
        PHI_TRY(expr);                                       \
        PHI_TRY(mark_kernel(timer, name, true, stream));     \
    } while (0)

template <typename R>
hipError_t enqueue_typed(const DevPlan& P, const StreamSet& ss, Stage stage, const void* in, void* out, int adjoint,
                         hipStream_t s, KernelTimer* timer) {
    PHI_TRY(check_twiddles(P));
    // forward solve: type-2 side and the first I1 transforms with e^{-...};
    // the transposed solve reverses every direction
    const int dir = adjoint ? 1 : -1;
    switch (stage) {
        case Stage::Solve: {
            PHI_STEP("rows_forward", s, (run_rows_forward<R>(P, in, dir, s)));
            if (P.shared) {
                PHI_STEP("cols_type2", s, (run_cols_type2<R>(P, dir, s)));
                PHI_STEP("nodes", s, (run_nodes<R, 0>(P, nullptr, nullptr, s)));
                PHI_STEP("type1_highfreq", s, (launch_type1_highfreq(P, dir, s)));
                PHI_STEP("rows_inverse", s, (run_rows_inverse<R>(P, out, -dir, 1, 1, s)));
                return hipSuccess;
            }
            hipStream_t side = ss.side ? ss.side : s;
            if (ss.side) {
                PHI_TRY(hipEventRecord(ss.fork, s));
                PHI_TRY(hipStreamWaitEvent(side, ss.fork, 0));
            }
            // the branch enqueued first is served first by the dispatcher (the
            // plan picks it by the size of the column work)
            if (P.highfreq_first) PHI_STEP("cols_highfreq", s, (run_cols_highfreq<R>(P, dir, s)));
            PHI_STEP("cols_type2", side, (run_cols_type2<R>(P, dir, side)));
            PHI_STEP("nodes", side, (run_nodes<R, 0>(P, nullptr, nullptr, side)));
            PHI_STEP("cols_type1", side, (run_cols_type1<R>(P, -dir, side)));
            if (ss.side) PHI_TRY(hipEventRecord(ss.join, side));
            if (!P.highfreq_first) PHI_STEP("cols_highfreq", s, (run_cols_highfreq<R>(P, dir, s)));
            if (ss.side) PHI_TRY(hipStreamWaitEvent(s, ss.join, 0));
            PHI_STEP("rows_inverse", s, (run_rows_inverse<R>(P, out, -dir, 1, 1, s)));
            return hipSuccess;
        }
        case Stage::HighFreq:
            PHI_STEP("rows_forward", s, (run_rows_forward<R>(P, in, dir, s)));
            PHI_STEP("cols_highfreq", s, (run_cols_highfreq<R>(P, dir, s)));
            PHI_STEP("rows_inverse", s, (run_rows_inverse<R>(P, out, -dir, 1, 0, s)));
            return hipSuccess;
        case Stage::LowFreq:
            PHI_STEP("rows_forward", s, (run_rows_forward<R>(P, in, dir, s)));
            PHI_STEP("cols_type2", s, (run_cols_type2<R>(P, dir, s)));
            PHI_STEP("nodes", s, (run_nodes<R, 0>(P, nullptr, nullptr, s)));
            PHI_STEP("cols_type1", s, (run_cols_type1<R>(P, -dir, s)));
            PHI_STEP("rows_inverse", s, (run_rows_inverse<R>(P, out, -dir, 0, 1, s)));
            return hipSuccess;
        case Stage::Type2:
            PHI_STEP("rows_forward", s, (run_rows_forward<R>(P, in, dir, s)));
            PHI_STEP("cols_type2", s, (run_cols_type2<R>(P, dir, s)));
            PHI_STEP("nodes", s, (run_nodes<R, 1>(P, nullptr, out, s)));
            return hipSuccess;
        case Stage::Type1:
            PHI_STEP("nodes", s, (run_nodes<R, 2>(P, in, nullptr, s)));
            PHI_STEP("cols_type1", s, (run_cols_type1<R>(P, 1, s)));
            PHI_STEP("rows_inverse", s, (run_rows_inverse<R>(P, out, 1, 0, 1, s)));
            return hipSuccess;
    }
    return hipErrorInvalidValue;
}

}  // namespace

LaunchEvents& launch_events() {
    static thread_local LaunchEvents ev;
    return ev;
}

hipError_t mark_kernel(KernelTimer* t, const char* name, bool end, hipStream_t s) {
    if (!t) return hipSuccess;
    if (t->count >= KernelTimer::kMax) return hipErrorInvalidValue;
    LaunchEvents& le = launch_events();
    if (!end) {
        t->names[t->count] = name;
        le.start = t->ev[2 * t->count];
        le.stop = t->ev[2 * t->count + 1];
        le.used = false;
        return hipSuccess;
    }
    hipError_t e = hipSuccess;
    if (!le.used) {   // nothing was launched in between: an empty interval
        e = hipEventRecord(t->ev[2 * t->count], s);
        if (e == hipSuccess) e = hipEventRecord(t->ev[2 * t->count + 1], s);
    }
    le = LaunchEvents();
    ++t->count;
    return e;
}


hipError_t enqueue(const DevPlan& P, const StreamSet& ss, Stage stage, const void* in, void* out, int adjoint,
                   hipStream_t s, KernelTimer* timer) {
    // the periodic operator is symmetric: its transpose is the same chain
    if (stage == Stage::Periodic) return enqueue_periodic(P, in, out, s, timer);
    if (P.dtype == PHI_F32) return enqueue_typed<float>(P, ss, stage, in, out, adjoint, s, timer);
    return enqueue_typed<double>(P, ss, stage, in, out, adjoint, s, timer);
}

}  // namespace phi

// The one-stream layout of a solve's middle part: after the type-2 window
// columns and the node subproblems (their own launches), one launch runs the
// type-1 window columns in its first blocks and every I1 spectrum column in
// the rest.
//
// The I1 columns depend only on rows_forward and nothing depends on them but
// rows_inverse, so they can share any launch of the node-side chain; beside the
// type-1 columns (the chain's last and longest stage) their work fills the chip
// around the chain's few blocks, with no cross-stream dependency and no
// in-kernel wait.  The kernel bodies are the ones of the separate launches, so
// the results are the same bit for bit as the two-stream layout's.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "solver_device.hpp"

namespace phi {

namespace {

// Blocks [0, own) transform type-1 window columns (one per block, as the
// separate cols_type1 launch does), the rest I1 spectrum columns.
template <typename R, int LOG, int DIR, int KIND, bool EXACT>
__global__ __launch_bounds__(FftShape<LOG>::NT * lines_per_block<LOG>()) void k_type1_highfreq(DevPlan P, int own) {
    constexpr int G = lines_per_block<LOG>();
    __shared__ cpx<R> lds_all[G * lds_group_stride(1 << LOG)];
    const int b = static_cast<int>(blockIdx.x);
    if (b >= own) {
        const int c = xcd_logical_block(b - own, static_cast<int>(gridDim.x) - own);
        cols_highfreq_body<R, LOG, DIR, G, KIND, EXACT>(P, c * G, lds_all);
        return;
    }
    // the chain's blocks are the launch's longest: their waves issue first on a shared SIMD
    __builtin_amdgcn_s_setprio(3);
    cols_type1_body<R, LOG, -DIR, G, 1, false>(P, b, lds_all);
}

template <typename R, int LOG, int DIR>
hipError_t launch_dir(const DevPlan& P, hipStream_t s) {
    constexpr int G = lines_per_block<LOG>();
    constexpr int block = FftShape<LOG>::NT * G;
    const int own = P.patch;
    const int blocks = own + (P.n_fine / 2 + 1 + G - 1) / G;
    // the same multiplier kind and bounds variant as the separate cols_highfreq launch
    const bool exact = 2 * P.n == P.n_fine;
    if (P.component == 2 && exact)
        PHI_LAUNCH((k_type1_highfreq<R, LOG, DIR, kKindMixed, true>), dim3(blocks), dim3(block), 0, s, P, own);
    else if (P.component == 2)
        PHI_LAUNCH((k_type1_highfreq<R, LOG, DIR, kKindMixed, false>), dim3(blocks), dim3(block), 0, s, P, own);
    else if (P.component == 3 && P.partition_erfc)
        PHI_LAUNCH((k_type1_highfreq<R, LOG, DIR, kKindCoulombErfc, false>), dim3(blocks), dim3(block), 0, s, P,
                   own);
    else if (P.component == 3)
        PHI_LAUNCH((k_type1_highfreq<R, LOG, DIR, kKindCoulombGauss, false>), dim3(blocks), dim3(block), 0, s, P,
                   own);
    else if (exact)
        PHI_LAUNCH((k_type1_highfreq<R, LOG, DIR, kKindQuadratic, true>), dim3(blocks), dim3(block), 0, s, P, own);
    else
        PHI_LAUNCH((k_type1_highfreq<R, LOG, DIR, kKindQuadratic, false>), dim3(blocks), dim3(block), 0, s, P, own);
    return hipGetLastError();
}

template <typename R, int LOG>
hipError_t launch_typed(const DevPlan& P, int dir, hipStream_t s) {
    if (P.twr_count != FftShape<LOG>::tw_size()) return hipErrorInvalidValue;
    return dir < 0 ? launch_dir<R, LOG, -1>(P, s) : launch_dir<R, LOG, 1>(P, s);
}

template <typename R>
hipError_t launch_r(const DevPlan& P, int dir, hipStream_t s) {
    static_assert(kSharedMinLogFine == 4 && kSharedMaxLogFine == 12, "instantiated sides");
    switch (P.log_fine) {
        case 4: return launch_typed<R, 4>(P, dir, s);
        case 5: return launch_typed<R, 5>(P, dir, s);
        case 6: return launch_typed<R, 6>(P, dir, s);
        case 7: return launch_typed<R, 7>(P, dir, s);
        case 8: return launch_typed<R, 8>(P, dir, s);
        case 9: return launch_typed<R, 9>(P, dir, s);
        case 10: return launch_typed<R, 10>(P, dir, s);
        case 11: return launch_typed<R, 11>(P, dir, s);
        case 12: return launch_typed<R, 12>(P, dir, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_type1_highfreq(const DevPlan& P, int dir, hipStream_t s) {
    if (P.dtype == PHI_F32) return launch_r<float>(P, dir, s);
    return launch_r<double>(P, dir, s);
}

}  // namespace phi

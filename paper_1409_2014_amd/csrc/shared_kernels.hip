// The shared layout of a solve's middle part (padded sides 16 .. 2048):
// three launches on the solve's one stream, each running one stage of the
// node-side chain in its first blocks and a slice of the I1 spectrum columns
// in the rest.
//
//   launch 0: type-2 window columns   + I1 columns [0, c0)
//   launch 1: node subproblems        + I1 columns [c0, c0 + c1)
//   launch 2: type-1 window columns   + I1 columns [c0 + c1, F/2 + 1)
//
// The I1 columns depend only on rows_forward and nothing depends on them but
// rows_inverse, so any split of them over the three launches gives the same
// results; the split (DevPlan::shared_cols, chosen by the plan) sizes each
// slice to the expected length of its chain stage, so the column work fills the
// chip beside the chain's few blocks and no launch waits long for either.
// Unlike the two-stream layout, no cross-stream dependency and no in-kernel
// wait is involved; the kernel bodies are the ones of the separate launches,
// so the results are the same bit for bit.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "solver_device.hpp"

namespace phi {

namespace {

template <typename R, int LOG>
constexpr size_t shared_lds_bytes() {
    constexpr size_t fft = static_cast<size_t>(lines_per_block<LOG>()) * lds_group_stride(1 << LOG) * sizeof(cpx<R>);
    constexpr size_t node = sizeof(NodeLds<R, kMaxEsWidth>);
    return fft > node ? fft : node;
}

// What one launch runs: `own` chain blocks of stage `stage`, then I1 column
// blocks col_block0 .. col_block0 + (gridDim.x - own) - 1.
struct SharedLaunch {
    int stage, own, col_block0;
};

template <typename R, int LOG, int DIR, int KIND, bool EXACT>
__global__ __launch_bounds__(FftShape<LOG>::NT * lines_per_block<LOG>()) void k_shared(DevPlan P, SharedLaunch S) {
    constexpr int G = lines_per_block<LOG>();
    constexpr int NTH = FftShape<LOG>::NT * G;
    __shared__ __align__(16) unsigned char lds_raw[shared_lds_bytes<R, LOG>()];
    cpx<R>* lds = reinterpret_cast<cpx<R>*>(lds_raw);
    const int b = static_cast<int>(blockIdx.x);
    if (b >= S.own) {
        const int c = S.col_block0 + xcd_logical_block(b - S.own, static_cast<int>(gridDim.x) - S.own);
        cols_highfreq_body<R, LOG, DIR, G, KIND, EXACT>(P, c * G, lds);
        return;
    }
    // the chain's blocks are the launch's longest: their waves issue first on a shared SIMD
    __builtin_amdgcn_s_setprio(3);
    if (S.stage == 0) {
        cols_type2_body<R, LOG, DIR, G, false>(P, b * G, lds);
    } else if (S.stage == 1) {
        nodes_body<R, 0, NTH, kMaxEsWidth>(P, b, nullptr, nullptr, *reinterpret_cast<NodeLds<R, kMaxEsWidth>*>(lds_raw));
    } else {
        cols_type1_body<R, LOG, -DIR, G, 1, false>(P, b, lds);
    }
}

template <typename R, int LOG, int DIR>
hipError_t launch_dir(const DevPlan& P, const SharedLaunch& S, int blocks, hipStream_t s) {
    constexpr int block = FftShape<LOG>::NT * lines_per_block<LOG>();
    // the same multiplier kind and bounds variant as the separate cols_highfreq launch
    const bool exact = 2 * P.n == P.n_fine;
    if (P.component == 2 && exact)
        PHI_LAUNCH((k_shared<R, LOG, DIR, kKindMixed, true>), dim3(blocks), dim3(block), 0, s, P, S);
    else if (P.component == 2)
        PHI_LAUNCH((k_shared<R, LOG, DIR, kKindMixed, false>), dim3(blocks), dim3(block), 0, s, P, S);
    else if (P.component == 3 && P.partition_erfc)
        PHI_LAUNCH((k_shared<R, LOG, DIR, kKindCoulombErfc, false>), dim3(blocks), dim3(block), 0, s, P, S);
    else if (P.component == 3)
        PHI_LAUNCH((k_shared<R, LOG, DIR, kKindCoulombGauss, false>), dim3(blocks), dim3(block), 0, s, P, S);
    else if (exact)
        PHI_LAUNCH((k_shared<R, LOG, DIR, kKindQuadratic, true>), dim3(blocks), dim3(block), 0, s, P, S);
    else
        PHI_LAUNCH((k_shared<R, LOG, DIR, kKindQuadratic, false>), dim3(blocks), dim3(block), 0, s, P, S);
    return hipGetLastError();
}

template <typename R, int LOG>
hipError_t launch_typed(const DevPlan& P, int stage, int dir, hipStream_t s) {
    constexpr int G = lines_per_block<LOG>();
    if (P.twr_count != FftShape<LOG>::tw_size()) return hipErrorInvalidValue;
    const int col_blocks = (P.n_fine / 2 + 1 + G - 1) / G;
    if (P.shared_cols[0] < 0 || P.shared_cols[1] < 0 || P.shared_cols[2] < 0 ||
        P.shared_cols[0] + P.shared_cols[1] + P.shared_cols[2] != col_blocks)
        return hipErrorInvalidValue;
    SharedLaunch S;
    S.stage = stage;
    S.own = stage == 0 ? (P.patch + G - 1) / G : stage == 1 ? P.n_sub : P.patch;
    S.col_block0 = 0;
    for (int k = 0; k < stage; ++k) S.col_block0 += P.shared_cols[k];
    const int blocks = S.own + P.shared_cols[stage];
    return dir < 0 ? launch_dir<R, LOG, -1>(P, S, blocks, s) : launch_dir<R, LOG, 1>(P, S, blocks, s);
}

template <typename R>
hipError_t launch_r(const DevPlan& P, int stage, int dir, hipStream_t s) {
    static_assert(kSharedMinLogFine == 4 && kSharedMaxLogFine == 11, "instantiated sides");
    switch (P.log_fine) {
        case 4: return launch_typed<R, 4>(P, stage, dir, s);
        case 5: return launch_typed<R, 5>(P, stage, dir, s);
        case 6: return launch_typed<R, 6>(P, stage, dir, s);
        case 7: return launch_typed<R, 7>(P, stage, dir, s);
        case 8: return launch_typed<R, 8>(P, stage, dir, s);
        case 9: return launch_typed<R, 9>(P, stage, dir, s);
        case 10: return launch_typed<R, 10>(P, stage, dir, s);
        case 11: return launch_typed<R, 11>(P, stage, dir, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_shared_stage(const DevPlan& P, int stage, int dir, hipStream_t s) {
    if (stage < 0 || stage > 2 || P.width > kMaxEsWidth) return hipErrorInvalidValue;
    if (P.dtype == PHI_F32) return launch_r<float>(P, stage, dir, s);
    return launch_r<double>(P, stage, dir, s);
}

}  // namespace phi

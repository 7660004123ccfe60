// Device side of the DS time stepper (gfx950): the split-step passes over an
// N x N complex field and the reductions of the L4 loss.
#pragma once

#include <hip/hip_runtime.h>

#include "phi_solve.h"

namespace phi {

// Device tables and workspace of a stepper (device pointers, data precision
// unless stated).  Complex values are interleaved (re, im).
constexpr int kDsMaxTimes = 4;   // distinct linear-substep durations of a composition

struct DsDev {
    phi_dtype dtype;
    int n, log_n;
    double c_local, c_potential, h2;   // phase = s (c_local rho + c_potential Phi)
    // Fourier multipliers of the linear substep in FFT order (index m -> k = m/(N h)
    // for m < N/2, (m - N)/(N h) otherwise), one pair per distinct duration s_i:
    const void* ex[kDsMaxTimes];   // [N] e^{-i 4 pi^2 kx^2 s_i}
    const void* ey[kDsMaxTimes];   // [N] e^{+i 4 pi^2 alpha ky^2 s_i}
    int n_times;
    const void* twr;       // register-FFT stage twiddles of length N
    int twr_count;
    void* spec;            // N x N complex, column-major [kx][y]: the field after the x transform
    double* partials;      // kDsReduceBlocks x 2 FP64 partial sums of the moments
};

constexpr int kDsReduceBlocks = 512;

// Pointwise update fused into the row pass that starts a linear substep.
enum class DsRowIn {
    Plain = 0,       // x = u
    Nonlinear = 1,   // x = v e^{i phi}, phi = s (c_l |v|^2 + c_p Phi)
    Adjoint = 2,     // x = g e^{-i phi} + 2 s (c_l q + c_p t) v
};
// Outputs of the row pass that completes a linear substep.
enum class DsRowOut {
    Field = 0,       // the field only
    Density = 1,     // the field and rho = |field|^2
    AdjointSource = 2,   // the field g and s = -Im(conj(g) v e^{i phi})
};

// First pass of a linear substep: per grid row, the pointwise update of the
// nonlinear substep of duration ntau (or its adjoint), the forward x transform
// and the x multiplier of table `time` (conjugated when conj != 0: the adjoint
// flow); the result goes to spec.
hipError_t ds_rows_forward(const DsDev& D, DsRowIn mode, int conj, int time, const void* x, const void* v,
                           const void* pot, const void* s, const void* t, double ntau, hipStream_t st);
// Second pass: per column of spec, forward y transform, y multiplier of table
// `time`, inverse y transform (in place).
hipError_t ds_cols(const DsDev& D, int conj, int time, hipStream_t st);
// Last pass: per grid row, inverse x transform and 1/N^2; writes the field to
// out_c (row-major) and, by mode, rho or the adjoint source s of the nonlinear
// substep of duration ntau to out_r.
hipError_t ds_rows_inverse(const DsDev& D, DsRowOut mode, void* out_c, void* out_r, const void* v,
                           const void* pot, double ntau, hipStream_t st);
// out[0] = h^2 sum |u|^2, out[1] = h^2 sum |u|^4 (FP64, fixed summation order).
hipError_t ds_moments(const DsDev& D, const void* u, double* out, hipStream_t st);
// g = 4 h^2 |u|^2 u: the gradient of h^2 sum |u|^4 (dJ/dRe u + i dJ/dIm u).
hipError_t ds_loss_grad(const DsDev& D, const void* u, void* g, hipStream_t st);

}  // namespace phi

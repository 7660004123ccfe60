// Device-side view of a plan and the kernel-chain entry point.
#pragma once

#include <hip/hip_runtime.h>

#include "phi_solve.h"
#include "plan_host.hpp"

namespace phi {

// Everything a kernel needs, passed by value.  All pointers are device
// pointers into the plan's single allocation.
struct DevPlan {
    phi_dtype dtype;
    int n, n_fine, log_fine;
    int patch, patch_lo, width, bin, n_nodes, n_sub, component_y;
    double beta, h2, inv_f2;
    // FP64 tables
    const double* deconv;   // [N]
    const double* gx;       // [2 (N+1)]
    const double* gy;       // [2 F]
    const double* tw_lo;    // [2 S]
    const double* tw_hi;    // [2 F/S]
    const void* twr;        // register-FFT stage twiddles, data precision, twr_count complex
    int twr_count;
    const double* ux;       // [M]
    const double* uy;       // [M]
    const double* q;        // [M] (without h^2)
    const int* sub;         // [4 n_sub]
    const int* bin_start;   // [nb*nb + 1] subproblem range of each bin
    int nb;                 // bins per window side (window side = nb * bin)
    int tile;               // tile side E = bin + width - 1
    // workspace, element type = data precision
    void* xt;       // (N+1) x N complex: I1 half spectrum, column-major
    void* tt;       // Q x N complex: type-2 row window, column-major
    void* win;      // Q x Q complex: type-2 fine-grid window
    void* pts;      // M complex: a_j = q_j rho_hat_j
    void* tiles;    // n_sub x E x E complex: each subproblem's spread tile
    void* u;        // N x Q complex: type-1 column transforms
};

enum class Stage { Solve, HighFreq, LowFreq, Type2, Type1 };

// Optional per-kernel timing: an event is recorded on the launch stream before
// each kernel of the chain and one after the last.  The events are created by
// the owner; names[i] names the kernel that starts at ev[i].
struct KernelTimer {
    static constexpr int kMax = 16;
    hipEvent_t ev[kMax];
    const char* names[kMax];
    int count = 0;
};

// Enqueue a stage chain on stream s (no host synchronisation).  adjoint = 1
// reverses every transform direction (the transposed operator).
hipError_t enqueue(const DevPlan& P, Stage stage, const void* in, void* out, int adjoint, hipStream_t s,
                   KernelTimer* timer = nullptr);

}  // namespace phi

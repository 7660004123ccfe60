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
    int log_n;              // log2 N when N is a power of two (the periodic solver), else -1
    int patch, patch_lo, width, n_nodes;
    int component;          // 0: -kx^2/|k|^2, 1: -ky^2/|k|^2, 2: -kx ky/|k|^2, 3: 1/|k| (Coulomb)
    int partition_erfc;     // Coulomb: partition erfc(|k|/sigma) (else e^{-|k|^2/sigma^2})
    double inv_sigma;       // 1 / sigma
    int highfreq_first;     // a solve enqueues the I1 columns before the node-side chain
    int shared;             // one stream: the type-1 window columns and all I1 columns in one launch
    double freq_scale;      // 1 / (n_fine h sigma): k/sigma per fine-grid frequency index
    int col_stride;         // elements between consecutive columns of xt and tt (N + pad)
    double h2, inv_f2;
    // FP64 tables
    const double* deconv;   // [N] 2 pi / (n_fine psi_hat(n'))
    const double* gx;       // [2 (F/2+1)] I1 multiplier factors along x
    const double* gy;       // [2 F] I1 multiplier factors along y
    const void* gyr;        // [F] (b, 1 - e^{-b}) pairs of gy in the data precision
    const double* q;        // [M] I2 weights q_j (without h^2)
    // node tables
    const int* cell;        // [2 M] first-tap window cell (x, y)
    const void* taps;       // [M][2][w] kernel tap values, data precision
    const int* sub;         // [4 n_sub] bin x, bin y, first node, node count
    const int* contrib_start;  // [Q^2 + 1] tile entries summed into window cell x*Q + y
    const int* contrib;        // flat tile indices
    int n_sub, bin, tile;      // subproblems, bin side, tile side E = bin + w - 1
    const void* twr;        // register-FFT stage twiddles, data precision, twr_count complex
    int twr_count;
    const void* twn;        // the same for length N (periodic solver), twn_count complex
    int twn_count;
    // workspace, element type = data precision
    void* xt;       // (F/2+1) columns of N complex: I1 half spectrum, column-major, col_stride apart
    void* tt;       // Q columns of N complex: type-2 row window, column-major, col_stride apart
    void* win;      // Q x Q complex: type-2 fine-grid window, [y][x]
    void* pts;      // M complex: a_j = q_j rho_hat_j
    void* tiles;    // n_sub x E x E complex: each subproblem's spread tile
    void* u;        // N x Q complex: type-1 column transforms, [n2][x]
};

// Streams and events a plan uses to run the node-side chain concurrently with
// the I1 column pass (all default priority).
struct StreamSet {
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
};

enum class Stage { Solve, HighFreq, LowFreq, Type2, Type1, Periodic };

// Optional per-kernel timing: events recorded on the kernel's launch stream
// just before and just after each kernel.  The events are created by the owner.
struct KernelTimer {
    static constexpr int kMax = 16;
    hipEvent_t ev[2 * kMax];
    const char* names[kMax];
    int count = 0;
};

// The standard periodic FFT solver on the plan's grid (three passes of N-point
// FFTs over the I1 half-spectrum workspace); N >= 16.
hipError_t enqueue_periodic(const DevPlan& P, const void* in, void* out, hipStream_t s, KernelTimer* timer);

// Starts (end = false) or closes (end = true) the timing of kernel `name` on
// stream s; no-op without a timer.  The kernel launched in between receives the
// timer's two events through launch_events(), and the runtime records in them
// the kernel's own start and end (as the profiler sees it, not the enqueue
// around it).
hipError_t mark_kernel(KernelTimer* t, const char* name, bool end, hipStream_t s);

// Events for the next kernel launch of this host thread (null when nothing is timed).
struct LaunchEvents {
    hipEvent_t start = nullptr, stop = nullptr;
    bool used = false;
};
LaunchEvents& launch_events();

// Every solver kernel is launched through this macro: a plain launch, or, while
// a kernel is being timed, the runtime's launch with start and stop events
// (hipExtLaunchKernelGGL; kernel sources include <hip/hip_ext.h>).
#define PHI_LAUNCH(KERNEL, GRID, BLOCK, SHMEM, STREAM, ...)                                             \
    do {                                                                                               \
        ::phi::LaunchEvents& ev_ = ::phi::launch_events();                                             \
        if (ev_.start && !ev_.used) {                                                                  \
            ev_.used = true;                                                                           \
            hipExtLaunchKernelGGL(KERNEL, GRID, BLOCK, SHMEM, STREAM, ev_.start, ev_.stop, 0, __VA_ARGS__); \
        } else {                                                                                       \
            hipLaunchKernelGGL(KERNEL, GRID, BLOCK, SHMEM, STREAM, __VA_ARGS__);                        \
        }                                                                                              \
    } while (0)

// Padded sides (log2) for which the one-stream layout's kernel is built.
constexpr int kSharedMinLogFine = 4;
constexpr int kSharedMaxLogFine = 12;

// The one-stream layout's last launch on stream s: the type-1 window columns
// (one per block) and then every I1 spectrum column.  dir is the solve's
// transform direction (the type-1 columns run the reverse one).
hipError_t launch_type1_highfreq(const DevPlan& P, int dir, hipStream_t s);


// Enqueue a stage chain on stream s (no host synchronisation).  adjoint = 1
// reverses every transform direction (the transposed operator).
hipError_t enqueue(const DevPlan& P, const StreamSet& ss, Stage stage, const void* in, void* out, int adjoint,
                   hipStream_t s, KernelTimer* timer = nullptr);

// ---- batches of independent solves of different sizes -----------------------
// Batched kernels run 256-thread blocks; a block takes one entry of a work table
// (member, first row / column / subproblem, kind) and dispatches on the
// member's transform length, so one launch per stage covers every member.
constexpr int kBatchThreads = 256;
constexpr int kBatchMinLogFine = 8;    // N = 128
constexpr int kBatchMaxLogFine = 12;   // N = 2048

// rows or columns per batched block at fine-grid side 2^log_fine (F/16 threads
// per transform)
constexpr int batch_lines(int log_fine) {
    const int nt = (1 << log_fine) / 16;
    return nt >= kBatchThreads ? 1 : kBatchThreads / nt;
}

struct WorkItem {
    int member;   // index into BatchDev::members
    int item;     // first grid row, spectrum / window column, or subproblem
    int kind;     // column pass: 0 = I1 spectrum column, 1 = type-2 window column
    int pad;
};

// Device tables of a batch (all device pointers).  Member i reads its input at
// in + offsets[i] and writes its output at out + offsets[i] (elements).
struct BatchDev {
    phi_dtype dtype = PHI_F32;
    const DevPlan* members = nullptr;
    const int64_t* offsets = nullptr;
    const WorkItem* rows = nullptr;    // rows_forward and rows_inverse
    const WorkItem* cols = nullptr;    // I1 spectrum columns
    const WorkItem* cols_t2 = nullptr; // type-2 window columns
    const WorkItem* cols_mixed = nullptr;  // I1 columns of the members with the mixed multiplier
    const WorkItem* nodes = nullptr;   // subproblems
    const WorkItem* cols1 = nullptr;   // type-1 window columns
    int n_rows = 0, n_cols = 0, n_cols_t2 = 0, n_cols_mixed = 0, n_nodes = 0, n_cols1 = 0;
    int wide_kernel = 0;               // some member's kernel is wider than kMaxEsWidth
};

// The static device scratch of phi_solve_noalloc: its size in bytes, and its
// address on `device`, which must be the current device (looked up on the
// first call per device and kept).
size_t scratch_capacity();
hipError_t scratch_region(int device, void** ptr);

// Enqueue one solve (adjoint = 0) or transposed solve (adjoint = 1) of every
// member on stream s (the node-side launches on ss.side, joined before the
// last launch; on s alone when ss.side is null).
hipError_t enqueue_batch(const BatchDev& B, const StreamSet& ss, const void* in, void* out, int adjoint,
                         hipStream_t s, KernelTimer* timer = nullptr);

}  // namespace phi

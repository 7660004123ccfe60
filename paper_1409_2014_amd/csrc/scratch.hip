// Static device scratch of the solve entry point that allocates nothing
// (phi_solve_noalloc in phi_solve.h).
//
// The array below is a file-scope device variable: every device that loads
// the library holds its own copy, at its own address, until the process ends.
// In host code its name is only a stand-in for the symbol, so the device
// address is looked up once per device (with that device current) and kept;
// kernels are only ever given that looked-up address.
#include <hip/hip_runtime.h>

#include <mutex>

#include "solver_kernels.hpp"

// 80 MiB: the workspace of any single-plan solve up to N = 2048 in either
// precision at the default node counts (74 MB for FP64 at 2048^2).
static constexpr size_t kScratchBytes = static_cast<size_t>(80) << 20;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace phi {

namespace {

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_addr[kMaxScratchDevices] = {};

}  // namespace

size_t scratch_capacity() { return kScratchBytes; }

hipError_t scratch_region(int device, void** ptr) {
    *ptr = nullptr;
    if (device < 0 || device >= kMaxScratchDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_addr[device]) {
        // the caller has made `device` current; the symbol resolves to this
        // device's copy of the array
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_addr[device] = p;
    }
    *ptr = g_scratch_addr[device];
    return hipSuccess;
}

}  // namespace phi

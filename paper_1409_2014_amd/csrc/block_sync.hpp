// Dependencies between the blocks of one launch (gfx950).
//
// Blocks with a role that depends on others wait on a device counter that the
// producing blocks increment.  The host guarantees progress: fewer blocks can
// ever wait than the device holds resident at once, so whatever the order in
// which blocks are dispatched, some resident block is always a producer (or
// independent work) that runs to completion and frees its slot; by induction
// every producer runs and every wait ends.  A wait is also bounded by a spin
// count: past it the block records an error flag and goes on, so the launch
// always drains.
//
// Visibility across the chip (each XCD has its own L2): a producer block makes
// its stores visible at agent scope before it counts itself done (release), and
// a waiting block, once the count is reached, issues one acquire fence before
// any thread of it reads the data.  Every access to a counter is a vector-memory
// atomic; each counter has a cache line of its own.
//
// The counters are zeroed by the kernel that precedes the launch in the same
// solve (a kernel boundary orders the stores), and once when a plan is created.
#pragma once

#include <hip/hip_runtime.h>

#include "solver_kernels.hpp"

namespace phi {

constexpr unsigned kSpinLimit = 1u << 21;   // about a second of polling

// Blocks until the counter reaches `target` (or the spin limit passes, which
// sets the error flag).  Afterwards every thread of the block may read what the
// counted blocks wrote.
__device__ __forceinline__ void wait_count(unsigned* sync, int slot, unsigned target) {
    if (threadIdx.x == 0) {
        // poll with a read-modify-write that changes nothing: it is performed
        // where the counter's atomics are, so it sees the current count (a
        // plain load may be served by a stale line of this XCD's L2, and an
        // acquire load would invalidate the caches on every poll, which every
        // block on the XCD pays for); one acquire fence once the count is reached
        unsigned spins = 0;
        while (__hip_atomic_fetch_or(sync + slot * kSyncStride, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
               target) {
            __builtin_amdgcn_s_sleep(4);
            if (++spins > kSpinLimit) {
                __hip_atomic_fetch_or(sync + kSyncError * kSyncStride, 1u, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
}

// Counts the calling block done in `slot` once every thread's stores are
// visible at agent scope: the barrier orders the block's stores before thread
// 0's release, which is cumulative over them (one cache write-back per block
// instead of one per wave).
__device__ __forceinline__ void signal_done(unsigned* sync, int slot) {
    __syncthreads();
    if (threadIdx.x == 0)
        __hip_atomic_fetch_add(sync + slot * kSyncStride, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Zeroes the counters of the next launch (the error flag stays); called by one
// thread of a kernel that precedes that launch in stream order.
__device__ __forceinline__ void reset_counters(unsigned* sync) {
    sync[kSyncT2Done * kSyncStride] = 0u;
    sync[kSyncNodesDone * kSyncStride] = 0u;
}

}  // namespace phi

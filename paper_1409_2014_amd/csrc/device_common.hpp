// Device-side helpers shared by the solver kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

namespace phi {

template <typename R>
struct cpx {
    R x, y;
};

template <typename R>
__device__ __forceinline__ cpx<R> cadd(cpx<R> a, cpx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R>
__device__ __forceinline__ cpx<R> csub(cpx<R> a, cpx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R>
__device__ __forceinline__ cpx<R> cmul(cpx<R> a, cpx<R> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename R>
__device__ __forceinline__ cpx<R> cconj(cpx<R> a) { return {a.x, -a.y}; }
template <typename R>
__device__ __forceinline__ cpx<R> cscale(cpx<R> a, R s) { return {a.x * s, a.y * s}; }
// multiply by s * i, s = +-1
template <typename R>
__device__ __forceinline__ cpx<R> cmul_si(cpx<R> a, R s) { return {-s * a.y, s * a.x}; }

// Workgroups of a 1-D grid are dispatched round-robin over the 8 XCDs of the
// chip (workgroup b runs on XCD b % 8), and each XCD has its own L2.  This map
// gives every XCD a contiguous range of logical indices, so neighbouring rows
// or columns (which share cache lines in the transposed layouts) meet in the
// same L2.  It is a bijection on [0, grid).
__device__ __forceinline__ int xcd_logical_block(int b, int grid) {
    const int per = grid >> 3;
    if (b >= (per << 3)) return b;
    return (b & 7) * per + (b >> 3);
}

// LDS index with one padding slot every 16 elements: the strided Stockham
// writes (stride = radix) then fall into distinct banks.
__device__ __forceinline__ int lds_pad(int i) { return i + (i >> 4); }
__host__ __device__ constexpr int lds_padded_size(int n) { return n + (n >> 4); }

template <typename R>
__device__ __forceinline__ cpx<R> load_cpx(const double* p) {
    return {static_cast<R>(p[0]), static_cast<R>(p[1])};
}

}  // namespace phi

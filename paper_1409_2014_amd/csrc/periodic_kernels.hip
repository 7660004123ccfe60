// The standard periodic FFT potential solver (gfx950): the baseline the paper
// compares its split solver with (Sec. 1: truncation to a periodic box and an
// FFT; Sec. 3.1, Tables 1 and 4).  On the N x N grid of the plan,
//
//   Phi_hat(k_m) = -kx^2/|k|^2 rho_hat(k_m),  k_m = m/(N h), Phi_hat(0) = 0,
//
// in three passes of register-resident N-point FFTs (N = 16 .. 4096):
//
//   per_rows_forward   per pair of grid rows: z = rho_a + i rho_b, one FFT; the
//                      half spectra of both rows (m = 0 .. N/2) go to the
//                      column-major workspace (the plan's I1 half-spectrum
//                      buffer), the pair's two entries adjacent.
//   per_cols           per column m: FFT along y, times -kx^2/|k|^2 / N^2 (the
//                      ratio of integers m^2 / (m^2 + m'^2), exact in the data
//                      precision; m'^2 or m m' for the y and mixed components),
//                      inverse FFT, in place.
//   per_rows_inverse   per pair of rows: the Hermitian extensions of both half
//                      spectra combined as X_a + i X_b, one inverse FFT:
//                      Phi_a = Re, Phi_b = Im.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "solver_device.hpp"

namespace phi {

namespace {

// Row pairs per block: the same budget as the padded row kernels, whose
// transform length 2^LOG also serves 2^LOG / 2 row pairs here.
template <typename R, int LOG>
constexpr int pairs_per_block() { return rows_per_block<R, LOG>(); }

template <typename R, int LOG>
__global__ __launch_bounds__((FftShape<LOG>::NT * pairs_per_block<R, LOG>())) void k_per_rows_forward(
    DevPlan P, const R* __restrict__ rho) {
    using Sh = FftShape<LOG>;
    constexpr int N = Sh::F;
    constexpr int NT = Sh::NT;
    constexpr int G = pairs_per_block<R, LOG>();
    static_assert((N / 2) % G == 0, "the row pairs of a block must tile the grid");
    constexpr int LP = lds_group_stride(N);
    __shared__ cpx<R> lds_all[G * LP];
    const int pair0 = xcd_logical_block(blockIdx.x, gridDim.x) * G;
    const int g = threadIdx.x / NT;
    const int tid = threadIdx.x - g * NT;
    cpx<R>* lds = lds_all + g * LP;
    const cpx<R>* tw = static_cast<const cpx<R>*>(P.twn);
    const R* ra = rho + static_cast<size_t>(2 * (pair0 + g)) * N;
    const R* rb = ra + N;
    cpx<R> v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = {ra[tid + NT * i], rb[tid + NT * i]};
    fft_reg<R, LOG, -1>(v, lds, tw, tid);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) lds[lds_pad(tid + NT * i)] = v[i];
    __syncthreads();
    cpx<R>* xt = static_cast<cpx<R>*>(P.xt);
    constexpr int ITEMS = (N / 2 + 1) * G;
    for (int idx = threadIdx.x; idx < ITEMS; idx += NT * G) {
        const int gg = idx % G;
        const int m = idx / G;
        const cpx<R>* l = lds_all + gg * LP;
        const cpx<R> z = l[lds_pad(m)];
        const cpx<R> zc = l[lds_pad((N - m) & (N - 1))];
        // X_a = (Z[m] + conj Z[-m]) / 2, X_b = (Z[m] - conj Z[-m]) / (2i)
        cpx<R>* dst = xt + static_cast<size_t>(m) * P.col_stride + 2 * (pair0 + gg);
        dst[0] = {R(0.5) * (z.x + zc.x), R(0.5) * (z.y - zc.y)};
        dst[1] = {R(0.5) * (z.y + zc.y), R(-0.5) * (z.x - zc.x)};
    }
}

// COMP: 0 -kx^2/|k|^2, 1 -ky^2/|k|^2, 2 -kx ky/|k|^2
template <typename R, int LOG, int COMP>
__global__ __launch_bounds__(FftShape<LOG>::NT * lines_per_block<LOG>()) void k_per_cols(DevPlan P) {
    using Sh = FftShape<LOG>;
    constexpr int N = Sh::F;
    constexpr int NT = Sh::NT;
    constexpr int G = lines_per_block<LOG>();
    __shared__ cpx<R> lds_all[G * lds_group_stride(N)];
    const int g = threadIdx.x / NT;
    const int tid = threadIdx.x - g * NT;
    cpx<R>* lds = lds_all + g * lds_group_stride(N);
    const cpx<R>* tw = static_cast<const cpx<R>*>(P.twn);
    const int m = blockIdx.x * G + g;          // column 0 .. N/2 (+ idle lanes of the last block)
    const bool active = m <= N / 2;
    const int mc = active ? m : N / 2;         // idle lanes read the last column and never store
    cpx<R>* col = static_cast<cpx<R>*>(P.xt) + static_cast<size_t>(mc) * P.col_stride;
    cpx<R> v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = col[tid + NT * i];
    fft_reg<R, LOG, -1>(v, lds, tw, tid);
    const R scale = static_cast<R>(1.0 / (static_cast<double>(N) * N));
    const R mx2 = static_cast<R>(mc * mc);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int p = tid + NT * i;
        const int ps = (p < N / 2) ? p : p - N;
        const R my2 = static_cast<R>(ps * ps);
        const R den = mx2 + my2;
        // the mixed numerator is odd in each index; a bin on a Nyquist line stands
        // for +m and -m and takes the multiplier's mean over them, 0
        const bool nyq = (mc == N / 2) || (ps == -N / 2);
        const R num = COMP == 2 ? (nyq ? R(0) : static_cast<R>(mc * ps)) : COMP == 1 ? my2 : mx2;
        // den = 0 only at m = m' = 0, where num = 0: the quotient is 0 there
        const R f = -num * recip(den + tiny_normal<R>()) * scale;
        v[i] = cscale(v[i], f);
    }
    fft_reg<R, LOG, 1>(v, lds, tw, tid);
    if (active) {
#pragma unroll
        for (int i = 0; i < 16; ++i) col[tid + NT * i] = v[i];
    }
}

template <typename R, int LOG>
__global__ __launch_bounds__((FftShape<LOG>::NT * pairs_per_block<R, LOG>())) void k_per_rows_inverse(
    DevPlan P, R* __restrict__ out) {
    using Sh = FftShape<LOG>;
    constexpr int N = Sh::F;
    constexpr int NT = Sh::NT;
    constexpr int G = pairs_per_block<R, LOG>();
    constexpr int LP = lds_group_stride(N);
    __shared__ cpx<R> lds_all[G * LP];
    const int pair0 = xcd_logical_block(blockIdx.x, gridDim.x) * G;
    const int g = threadIdx.x / NT;
    const int tid = threadIdx.x - g * NT;
    cpx<R>* lds = lds_all + g * LP;
    const cpx<R>* tw = static_cast<const cpx<R>*>(P.twn);
    const cpx<R>* xt = static_cast<const cpx<R>*>(P.xt);
    constexpr int ITEMS = (N / 2 + 1) * G;
    for (int idx = threadIdx.x; idx < ITEMS; idx += NT * G) {
        const int gg = idx % G;
        const int m = idx / G;
        const cpx<R>* src = xt + static_cast<size_t>(m) * P.col_stride + 2 * (pair0 + gg);
        const cpx<R> a = src[0];
        const cpx<R> b = src[1];
        cpx<R>* l = lds_all + gg * LP;
        // position m: X_a + i X_b;  position N - m: conj X_a + i conj X_b
        l[lds_pad(m)] = {a.x - b.y, a.y + b.x};
        if (m > 0 && m < N / 2) l[lds_pad(N - m)] = {a.x + b.y, b.x - a.y};
    }
    __syncthreads();
    cpx<R> v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = lds[lds_pad(tid + NT * i)];
    fft_reg<R, LOG, 1>(v, lds, tw, tid);
    R* oa = out + static_cast<size_t>(2 * (pair0 + g)) * N;
    R* ob = oa + N;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        oa[tid + NT * i] = v[i].x;
        ob[tid + NT * i] = v[i].y;
    }
}

template <typename R, int LOG>
hipError_t periodic_log(const DevPlan& P, const void* in, void* out, hipStream_t s, KernelTimer* timer) {
    constexpr int N = 1 << LOG;
    if (P.n != N || P.twn_count != FftShape<LOG>::tw_size()) return hipErrorInvalidValue;
    constexpr int GR = pairs_per_block<R, LOG>();
    constexpr int GC = lines_per_block<LOG>();
    constexpr int NT = FftShape<LOG>::NT;
    hipError_t e = mark_kernel(timer, "per_rows_forward", false, s);
    if (e != hipSuccess) return e;
    PHI_LAUNCH((k_per_rows_forward<R, LOG>), dim3(N / 2 / GR), dim3(NT * GR), 0, s, P,
                       static_cast<const R*>(in));
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = mark_kernel(timer, "per_rows_forward", true, s)) != hipSuccess) return e;
    if ((e = mark_kernel(timer, "per_cols", false, s)) != hipSuccess) return e;
    const int col_blocks = (N / 2 + 1 + GC - 1) / GC;
    if (P.component == 2)
        PHI_LAUNCH((k_per_cols<R, LOG, 2>), dim3(col_blocks), dim3(NT * GC), 0, s, P);
    else if (P.component == 1)
        PHI_LAUNCH((k_per_cols<R, LOG, 1>), dim3(col_blocks), dim3(NT * GC), 0, s, P);
    else
        PHI_LAUNCH((k_per_cols<R, LOG, 0>), dim3(col_blocks), dim3(NT * GC), 0, s, P);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = mark_kernel(timer, "per_cols", true, s)) != hipSuccess) return e;
    if ((e = mark_kernel(timer, "per_rows_inverse", false, s)) != hipSuccess) return e;
    PHI_LAUNCH((k_per_rows_inverse<R, LOG>), dim3(N / 2 / GR), dim3(NT * GR), 0, s, P, static_cast<R*>(out));
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return mark_kernel(timer, "per_rows_inverse", true, s);
}

template <typename R>
hipError_t periodic_typed(const DevPlan& P, const void* in, void* out, hipStream_t s, KernelTimer* timer) {
    switch (P.log_n) {
        case 4: return periodic_log<R, 4>(P, in, out, s, timer);
        case 5: return periodic_log<R, 5>(P, in, out, s, timer);
        case 6: return periodic_log<R, 6>(P, in, out, s, timer);
        case 7: return periodic_log<R, 7>(P, in, out, s, timer);
        case 8: return periodic_log<R, 8>(P, in, out, s, timer);
        case 9: return periodic_log<R, 9>(P, in, out, s, timer);
        case 10: return periodic_log<R, 10>(P, in, out, s, timer);
        case 11: return periodic_log<R, 11>(P, in, out, s, timer);
        case 12: return periodic_log<R, 12>(P, in, out, s, timer);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t enqueue_periodic(const DevPlan& P, const void* in, void* out, hipStream_t s, KernelTimer* timer) {
    if (P.dtype == PHI_F32) return periodic_typed<float>(P, in, out, s, timer);
    return periodic_typed<double>(P, in, out, s, timer);
}

}  // namespace phi

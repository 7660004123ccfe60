// Split-step passes of the DS time stepper (gfx950).
//
// The field u is N x N complex, row-major [y][x].  A linear substep
// e^{A s} (Sec. 2.3: i v_t = (-d_xx + alpha d_yy) v, exact in Fourier space,
// v_hat <- v_hat e^{-i 4 pi^2 (kx^2 - alpha ky^2) s}) is three passes, each a
// batch of register-resident N-point FFTs:
//
//   rows_forward   per row: a pointwise update (none, the nonlinear substep, or
//                  its adjoint), forward x transform, times e^{-i 4 pi^2 kx^2 s};
//                  the result goes to `spec`, column-major [kx][y], in runs of
//                  G consecutive rows.
//   cols           per column of spec: forward y transform, times
//                  e^{+i 4 pi^2 alpha ky^2 s}, inverse y transform, in place.
//   rows_inverse   per row: gather the row from spec, inverse x transform,
//                  1/N^2; writes the field and, by mode, rho = |v|^2 (the input
//                  of the potential solve) or the adjoint source s.
//
// The nonlinear substep of duration s (Sec. 2.3: w = v e^{i s (c_l |v|^2 +
// c_p Phi)}, c_l = 2 beta and c_p = 4 beta for the DS system) is pointwise and rides in the next rows_forward; its adjoint
// likewise.  The adjoint of a linear substep is the same three passes with
// conjugated multipliers (the flow backwards in time).
#include <hip/hip_runtime.h>

#include "ds_kernels.hpp"
#include "solver_device.hpp"

namespace phi {

namespace {

// Rows per block of the row passes: as many as fit 1024 threads and about
// 70 KB of LDS, a power of two (so it divides N).
template <typename R, int LOG>
constexpr int ds_rows_per_block() {
    constexpr int nt = FftShape<LOG>::NT;
    constexpr int by_threads = 1024 / nt;
    constexpr int by_lds = static_cast<int>((70 * 1024) / (lds_group_stride(1 << LOG) * sizeof(cpx<R>)));
    int lim = by_threads < by_lds ? by_threads : by_lds;
    lim = lim < (1 << LOG) ? lim : (1 << LOG);
    int g = 1;
    while (2 * g <= lim) g *= 2;
    return g;
}

// Columns per block of the column pass: blocks of at least 256 threads, at
// most the N columns there are.
template <int LOG>
constexpr int ds_cols_per_block() {
    constexpr int nt = FftShape<LOG>::NT;
    constexpr int g = nt >= 256 ? 1 : 256 / nt;
    return g < (1 << LOG) ? g : (1 << LOG);
}

__device__ __forceinline__ void sin_cos(float a, float* s, float* c) { sincosf(a, s, c); }
__device__ __forceinline__ void sin_cos(double a, double* s, double* c) { sincos(a, s, c); }

// x times m (CONJ = false) or conj(m) (CONJ = true)
template <typename R, bool CONJ>
__device__ __forceinline__ cpx<R> mul_tab(cpx<R> x, cpx<R> m) {
    if constexpr (CONJ) return {x.x * m.x + x.y * m.y, x.y * m.x - x.x * m.y};
    else return {x.x * m.x - x.y * m.y, x.x * m.y + x.y * m.x};
}

// e^{i phi} with phi = tau (c_l |v|^2 + c_p Phi)
template <typename R>
__device__ __forceinline__ cpx<R> nonlinear_rotation(cpx<R> v, R pot, R tau, R cl, R cp) {
    const R rho = v.x * v.x + v.y * v.y;
    const R ph = tau * (cl * rho + cp * pot);
    R sn, cs;
    sin_cos(ph, &sn, &cs);
    return {cs, sn};
}

template <typename R, int LOG, int MODE, bool CONJ>
__global__ __launch_bounds__((FftShape<LOG>::NT * ds_rows_per_block<R, LOG>())) void k_ds_rows_forward(
    DsDev D, const cpx<R>* __restrict__ x, const cpx<R>* __restrict__ v, const R* __restrict__ pot,
    const R* __restrict__ s, const R* __restrict__ t, const cpx<R>* __restrict__ ex, R ntau) {
    using Sh = FftShape<LOG>;
    constexpr int N = Sh::F;
    constexpr int NT = Sh::NT;
    constexpr int G = ds_rows_per_block<R, LOG>();
    constexpr int LP = lds_group_stride(N);
    __shared__ cpx<R> lds_all[G * LP];
    const int row0 = xcd_logical_block(blockIdx.x, gridDim.x) * G;
    const int g = threadIdx.x / NT;
    const int tid = threadIdx.x - g * NT;
    cpx<R>* lds = lds_all + g * LP;
    const cpx<R>* tw = static_cast<const cpx<R>*>(D.twr);
    const size_t base = static_cast<size_t>(row0 + g) * N;
    const R tau = ntau, cl = static_cast<R>(D.c_local), cp = static_cast<R>(D.c_potential);
    cpx<R> a[16];
    if constexpr (MODE == static_cast<int>(DsRowIn::Adjoint)) {
        // adjoint of the nonlinear substep: g e^{-i phi} + 2 tau (c_l q + c_p t) v.
        // Five inputs and a sine/cosine per point: all 16 points at once need more
        // registers than a SIMD holds for two waves (FP64) or four (FP32), so the
        // points go four at a time through a loop that is not unrolled, each result
        // parked in this thread's own slots of the transform buffer (read back by
        // the same thread only, before the transform's first barrier).
#pragma unroll 1
        for (int c = 0; c < 16; c += 4) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const size_t idx = base + tid + NT * (c + j);
                const cpx<R> xv = x[idx];
                const cpx<R> vv = v[idx];
                const cpx<R> e = nonlinear_rotation(vv, pot[idx], tau, cl, cp);
                const R r = R(2) * tau * (cl * s[idx] + cp * t[idx]);
                lds[lds_pad(tid + NT * (c + j))] = {xv.x * e.x + xv.y * e.y + r * vv.x,
                                                    xv.y * e.x - xv.x * e.y + r * vv.y};
            }
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) a[i] = lds[lds_pad(tid + NT * i)];
    } else {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const size_t idx = base + tid + NT * i;
            const cpx<R> xv = x[idx];
            if constexpr (MODE == static_cast<int>(DsRowIn::Plain)) a[i] = xv;
            else a[i] = cmul(xv, nonlinear_rotation(xv, pot[idx], tau, cl, cp));
        }
    }
    fft_reg<R, LOG, -1>(a, lds, tw, tid);
#pragma unroll
    for (int i = 0; i < 16; ++i) a[i] = mul_tab<R, CONJ>(a[i], ex[tid + NT * i]);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) lds[lds_pad(tid + NT * i)] = a[i];
    __syncthreads();
    // spec[m][row0 + gg], row index fastest: G-element runs of each column
    cpx<R>* spec = static_cast<cpx<R>*>(D.spec);
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int idx = threadIdx.x + k * NT * G;
        const int gg = idx % G;
        const int m = idx / G;
        spec[static_cast<size_t>(m) * N + row0 + gg] = lds_all[gg * LP + lds_pad(m)];
    }
}

template <typename R, int LOG, bool CONJ>
__global__ __launch_bounds__(FftShape<LOG>::NT * ds_cols_per_block<LOG>()) void k_ds_cols(
    DsDev D, const cpx<R>* __restrict__ ey) {
    using Sh = FftShape<LOG>;
    constexpr int N = Sh::F;
    constexpr int NT = Sh::NT;
    constexpr int G = ds_cols_per_block<LOG>();
    __shared__ cpx<R> lds_all[G * lds_group_stride(N)];
    const int g = threadIdx.x / NT;
    const int tid = threadIdx.x - g * NT;
    cpx<R>* lds = lds_all + g * lds_group_stride(N);
    const cpx<R>* tw = static_cast<const cpx<R>*>(D.twr);
    const int m = blockIdx.x * G + g;
    const bool active = m < N;
    // idle lanes of the last block read column N - 1 and never store
    cpx<R>* col = static_cast<cpx<R>*>(D.spec) + static_cast<size_t>(active ? m : N - 1) * N;
    cpx<R> a[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) a[i] = col[tid + NT * i];
    fft_reg<R, LOG, -1>(a, lds, tw, tid);
#pragma unroll
    for (int i = 0; i < 16; ++i) a[i] = mul_tab<R, CONJ>(a[i], ey[tid + NT * i]);
    fft_reg<R, LOG, 1>(a, lds, tw, tid);
    if (active) {
#pragma unroll
        for (int i = 0; i < 16; ++i) col[tid + NT * i] = a[i];
    }
}

template <typename R, int LOG, int MODE>
__global__ __launch_bounds__((FftShape<LOG>::NT * ds_rows_per_block<R, LOG>())) void k_ds_rows_inverse(
    DsDev D, cpx<R>* __restrict__ out_c, R* __restrict__ out_r, const cpx<R>* __restrict__ v,
    const R* __restrict__ pot, R ntau) {
    using Sh = FftShape<LOG>;
    constexpr int N = Sh::F;
    constexpr int NT = Sh::NT;
    constexpr int G = ds_rows_per_block<R, LOG>();
    constexpr int LP = lds_group_stride(N);
    __shared__ cpx<R> lds_all[G * LP];
    const int row0 = xcd_logical_block(blockIdx.x, gridDim.x) * G;
    const int g = threadIdx.x / NT;
    const int tid = threadIdx.x - g * NT;
    cpx<R>* lds = lds_all + g * LP;
    const cpx<R>* tw = static_cast<const cpx<R>*>(D.twr);
    const cpx<R>* spec = static_cast<const cpx<R>*>(D.spec);
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int idx = threadIdx.x + k * NT * G;
        const int gg = idx % G;
        const int m = idx / G;
        lds_all[gg * LP + lds_pad(m)] = spec[static_cast<size_t>(m) * N + row0 + gg];
    }
    __syncthreads();
    cpx<R> a[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) a[i] = lds[lds_pad(tid + NT * i)];
    fft_reg<R, LOG, 1>(a, lds, tw, tid);
    const R scale = static_cast<R>(1.0 / (static_cast<double>(N) * N));
    const R tau = ntau, cl = static_cast<R>(D.c_local), cp = static_cast<R>(D.c_potential);
    const size_t base = static_cast<size_t>(row0 + g) * N;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const size_t idx = base + tid + NT * i;
        const cpx<R> f = cscale(a[i], scale);
        out_c[idx] = f;
        if constexpr (MODE == static_cast<int>(DsRowOut::Density)) {
            out_r[idx] = f.x * f.x + f.y * f.y;
        } else if constexpr (MODE == static_cast<int>(DsRowOut::AdjointSource)) {
            // s = -Im(conj(g) w), w = v e^{i phi}: the nonlinear substep's output
            const cpx<R> vv = v[idx];
            const cpx<R> w = cmul(vv, nonlinear_rotation(vv, pot[idx], tau, cl, cp));
            out_r[idx] = -(f.x * w.y - f.y * w.x);
        }
    }
}

// ---- moments and loss gradient ------------------------------------------------
constexpr int kReduceThreads = 256;

template <typename R>
__global__ __launch_bounds__(kReduceThreads) void k_ds_moments_partial(const cpx<R>* __restrict__ u, long long count,
                                                                      double* __restrict__ partials) {
    __shared__ double red[2][kReduceThreads];
    double s2 = 0.0, s4 = 0.0;
    const long long stride = static_cast<long long>(gridDim.x) * kReduceThreads;
    for (long long i = static_cast<long long>(blockIdx.x) * kReduceThreads + threadIdx.x; i < count; i += stride) {
        const cpx<R> z = u[i];
        const double r = static_cast<double>(z.x) * z.x + static_cast<double>(z.y) * z.y;
        s2 += r;
        s4 += r * r;
    }
    red[0][threadIdx.x] = s2;
    red[1][threadIdx.x] = s4;
    __syncthreads();
    for (int off = kReduceThreads / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            red[0][threadIdx.x] += red[0][threadIdx.x + off];
            red[1][threadIdx.x] += red[1][threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = red[0][0];
        partials[2 * blockIdx.x + 1] = red[1][0];
    }
}

__global__ __launch_bounds__(kReduceThreads) void k_ds_moments_final(const double* __restrict__ partials,
                                                                    int count, double h2,
                                                                    double* __restrict__ out) {
    __shared__ double red[2][kReduceThreads];
    double s2 = 0.0, s4 = 0.0;
    for (int i = threadIdx.x; i < count; i += kReduceThreads) {
        s2 += partials[2 * i];
        s4 += partials[2 * i + 1];
    }
    red[0][threadIdx.x] = s2;
    red[1][threadIdx.x] = s4;
    __syncthreads();
    for (int off = kReduceThreads / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            red[0][threadIdx.x] += red[0][threadIdx.x + off];
            red[1][threadIdx.x] += red[1][threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = h2 * red[0][0];
        out[1] = h2 * red[1][0];
    }
}

template <typename R>
__global__ __launch_bounds__(kReduceThreads) void k_ds_loss_grad(const cpx<R>* __restrict__ u, long long count,
                                                                R scale, cpx<R>* __restrict__ g) {
    const long long i = static_cast<long long>(blockIdx.x) * kReduceThreads + threadIdx.x;
    if (i >= count) return;
    const cpx<R> z = u[i];
    const R f = scale * (z.x * z.x + z.y * z.y);
    g[i] = {f * z.x, f * z.y};
}

// ---- launchers ------------------------------------------------------------------
#define PHI_DS_DISPATCH_LOG(LOGV, CALL)                  \
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
        default: return hipErrorInvalidValue;            \
    }

template <typename R, int LOG, int MODE, bool CONJ>
hipError_t launch_rows_forward(const DsDev& D, const void* x, const void* v, const void* pot, const void* s,
                               const void* t, const void* ex, double ntau, hipStream_t st) {
    if (D.twr_count != FftShape<LOG>::tw_size() || D.n != (1 << LOG)) return hipErrorInvalidValue;
    constexpr int G = ds_rows_per_block<R, LOG>();
    hipLaunchKernelGGL((k_ds_rows_forward<R, LOG, MODE, CONJ>), dim3(D.n / G), dim3(FftShape<LOG>::NT * G), 0, st,
                       D, static_cast<const cpx<R>*>(x), static_cast<const cpx<R>*>(v),
                       static_cast<const R*>(pot), static_cast<const R*>(s), static_cast<const R*>(t),
                       static_cast<const cpx<R>*>(ex), static_cast<R>(ntau));
    return hipGetLastError();
}

template <typename R, int LOG>
hipError_t rows_forward_log(const DsDev& D, DsRowIn mode, int conj, const void* x, const void* v, const void* pot,
                            const void* s, const void* t, const void* ex, double ntau, hipStream_t st) {
    // the forward chain uses (plain | nonlinear, direct), the reverse chain (plain | adjoint, conjugated)
    if (mode == DsRowIn::Plain && !conj)
        return launch_rows_forward<R, LOG, 0, false>(D, x, v, pot, s, t, ex, ntau, st);
    if (mode == DsRowIn::Plain && conj)
        return launch_rows_forward<R, LOG, 0, true>(D, x, v, pot, s, t, ex, ntau, st);
    if (mode == DsRowIn::Nonlinear && !conj)
        return launch_rows_forward<R, LOG, 1, false>(D, x, v, pot, s, t, ex, ntau, st);
    if (mode == DsRowIn::Adjoint && conj)
        return launch_rows_forward<R, LOG, 2, true>(D, x, v, pot, s, t, ex, ntau, st);
    return hipErrorInvalidValue;
}

template <typename R, int LOG>
hipError_t cols_log(const DsDev& D, int conj, const void* ey, hipStream_t st) {
    if (D.twr_count != FftShape<LOG>::tw_size() || D.n != (1 << LOG)) return hipErrorInvalidValue;
    constexpr int G = ds_cols_per_block<LOG>();
    const int blocks = (D.n + G - 1) / G;
    if (conj)
        hipLaunchKernelGGL((k_ds_cols<R, LOG, true>), dim3(blocks), dim3(FftShape<LOG>::NT * G), 0, st, D,
                           static_cast<const cpx<R>*>(ey));
    else
        hipLaunchKernelGGL((k_ds_cols<R, LOG, false>), dim3(blocks), dim3(FftShape<LOG>::NT * G), 0, st, D,
                           static_cast<const cpx<R>*>(ey));
    return hipGetLastError();
}

template <typename R, int LOG, int MODE>
hipError_t launch_rows_inverse(const DsDev& D, void* out_c, void* out_r, const void* v, const void* pot,
                               double ntau, hipStream_t st) {
    if (D.twr_count != FftShape<LOG>::tw_size() || D.n != (1 << LOG)) return hipErrorInvalidValue;
    constexpr int G = ds_rows_per_block<R, LOG>();
    hipLaunchKernelGGL((k_ds_rows_inverse<R, LOG, MODE>), dim3(D.n / G), dim3(FftShape<LOG>::NT * G), 0, st, D,
                       static_cast<cpx<R>*>(out_c), static_cast<R*>(out_r), static_cast<const cpx<R>*>(v),
                       static_cast<const R*>(pot), static_cast<R>(ntau));
    return hipGetLastError();
}

template <typename R, int LOG>
hipError_t rows_inverse_log(const DsDev& D, DsRowOut mode, void* out_c, void* out_r, const void* v,
                            const void* pot, double ntau, hipStream_t st) {
    switch (mode) {
        case DsRowOut::Field: return launch_rows_inverse<R, LOG, 0>(D, out_c, out_r, v, pot, ntau, st);
        case DsRowOut::Density: return launch_rows_inverse<R, LOG, 1>(D, out_c, out_r, v, pot, ntau, st);
        case DsRowOut::AdjointSource: return launch_rows_inverse<R, LOG, 2>(D, out_c, out_r, v, pot, ntau, st);
    }
    return hipErrorInvalidValue;
}

template <typename R>
hipError_t rows_forward_t(const DsDev& D, DsRowIn mode, int conj, int time, const void* x, const void* v,
                          const void* pot, const void* s, const void* t, double ntau, hipStream_t st) {
    if (time < 0 || time >= D.n_times) return hipErrorInvalidValue;
    const void* ex = D.ex[time];
    PHI_DS_DISPATCH_LOG(D.log_n, (rows_forward_log<R, L_>(D, mode, conj, x, v, pot, s, t, ex, ntau, st)));
}

template <typename R>
hipError_t cols_t(const DsDev& D, int conj, int time, hipStream_t st) {
    if (time < 0 || time >= D.n_times) return hipErrorInvalidValue;
    const void* ey = D.ey[time];
    PHI_DS_DISPATCH_LOG(D.log_n, (cols_log<R, L_>(D, conj, ey, st)));
}

template <typename R>
hipError_t rows_inverse_t(const DsDev& D, DsRowOut mode, void* out_c, void* out_r, const void* v, const void* pot,
                          double ntau, hipStream_t st) {
    PHI_DS_DISPATCH_LOG(D.log_n, (rows_inverse_log<R, L_>(D, mode, out_c, out_r, v, pot, ntau, st)));
}

}  // namespace

hipError_t ds_rows_forward(const DsDev& D, DsRowIn mode, int conj, int time, const void* x, const void* v,
                           const void* pot, const void* s, const void* t, double ntau, hipStream_t st) {
    if (D.dtype == PHI_F32) return rows_forward_t<float>(D, mode, conj, time, x, v, pot, s, t, ntau, st);
    return rows_forward_t<double>(D, mode, conj, time, x, v, pot, s, t, ntau, st);
}

hipError_t ds_cols(const DsDev& D, int conj, int time, hipStream_t st) {
    if (D.dtype == PHI_F32) return cols_t<float>(D, conj, time, st);
    return cols_t<double>(D, conj, time, st);
}

hipError_t ds_rows_inverse(const DsDev& D, DsRowOut mode, void* out_c, void* out_r, const void* v,
                           const void* pot, double ntau, hipStream_t st) {
    if (D.dtype == PHI_F32) return rows_inverse_t<float>(D, mode, out_c, out_r, v, pot, ntau, st);
    return rows_inverse_t<double>(D, mode, out_c, out_r, v, pot, ntau, st);
}

hipError_t ds_moments(const DsDev& D, const void* u, double* out, hipStream_t st) {
    const long long count = static_cast<long long>(D.n) * D.n;
    if (D.dtype == PHI_F32)
        hipLaunchKernelGGL((k_ds_moments_partial<float>), dim3(kDsReduceBlocks), dim3(kReduceThreads), 0, st,
                           static_cast<const cpx<float>*>(u), count, D.partials);
    else
        hipLaunchKernelGGL((k_ds_moments_partial<double>), dim3(kDsReduceBlocks), dim3(kReduceThreads), 0, st,
                           static_cast<const cpx<double>*>(u), count, D.partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_ds_moments_final, dim3(1), dim3(kReduceThreads), 0, st, D.partials, kDsReduceBlocks, D.h2,
                       out);
    return hipGetLastError();
}

hipError_t ds_loss_grad(const DsDev& D, const void* u, void* g, hipStream_t st) {
    const long long count = static_cast<long long>(D.n) * D.n;
    const int blocks = static_cast<int>((count + kReduceThreads - 1) / kReduceThreads);
    const double scale = 4.0 * D.h2;
    if (D.dtype == PHI_F32)
        hipLaunchKernelGGL((k_ds_loss_grad<float>), dim3(blocks), dim3(kReduceThreads), 0, st,
                           static_cast<const cpx<float>*>(u), count, static_cast<float>(scale),
                           static_cast<cpx<float>*>(g));
    else
        hipLaunchKernelGGL((k_ds_loss_grad<double>), dim3(blocks), dim3(kReduceThreads), 0, st,
                           static_cast<const cpx<double>*>(u), count, scale, static_cast<cpx<double>*>(g));
    return hipGetLastError();
}

}  // namespace phi

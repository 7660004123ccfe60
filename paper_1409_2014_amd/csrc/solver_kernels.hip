// HIP kernels of the split potential solve for gfx950 (see phi_solve.h).
//
// One solve runs seven stream-ordered kernels (N = grid side, F = 2N the side
// of both the zero-padded I1 box and the NUFFT fine grid, Q = side of the
// fine-grid window the polar nodes touch):
//
//   rows_forward   per grid row: z = rho + i rho d(n1) d(n2) at centred
//                  positions, one F-point FFT, then split the two real
//                  transforms: the I1 half spectrum (N+1 values) goes to the
//                  column-major buffer XT, the type-2 window (Q values) to TT.
//                  [Sec. 2.1, eq. 9 zero-padded FFT; Sec. 2.2 type 2: deconvolve + FFT]
//   cols_highfreq  per spectrum column: F-point FFT, times g1(k)/F^2, inverse
//                  FFT, keep the N centred rows, in place in XT.   [eq. 9]
//   cols_type2     per window column of TT: F-point FFT, keep the Q window rows.
//   interp         per bin-sorted subproblem: stage the fine-grid tile in LDS,
//                  interpolate rho_hat(k_j) = h^2 sum_taps b psi psi with 16-lane
//                  reductions, multiply by q_j.             [eq. 12, a_j = q_j rho_hat_j]
//   spread         per subproblem: the transposed taps accumulate a_j psi psi
//                  into an LDS tile (compensated sums in FP32); the tile goes
//                  to the subproblem's own slot (no atomics).  [type 1 spreading]
//   cols_type1     per window column: sum the tiles covering it in a fixed
//                  order, F-point FFT (only Q non-zero inputs), keep the N
//                  centred rows, times d(n2).
//   rows_inverse   per grid row: rebuild the full Hermitian I1 row spectrum plus
//                  i times the Hermitian part of the type-1 row, one F-point
//                  FFT; Phi = Re + Im d(n1).       [eq. 8: Phi = I1 + Re I2]
//
// The transposed solve runs the same kernels with every FFT direction reversed.
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "fft_lds.hpp"
#include "fft_reg.hpp"
#include "solver_kernels.hpp"

namespace phi {

namespace {

__device__ __forceinline__ int posmod_dev(int a, int b) {
    int r = a % b;
    return r < 0 ? r + b : r;
}

// Centred grid index n (0..N-1, n' = n - N/2) -> position n' mod F on the fine grid.
template <int LOG>
__device__ __forceinline__ int centred_pos(int n) {
    constexpr int F = 1 << LOG;
    constexpr int N = F / 2;
    return (n - N / 2) & (F - 1);
}

// Inverse of centred_pos: position p -> grid index, or -1 for a padding position.
template <int LOG>
__device__ __forceinline__ int pos_to_grid(int p) {
    constexpr int F = 1 << LOG;
    constexpr int N = F / 2;
    if (p < N / 2) return p + N / 2;
    if (p >= F - N / 2) return p - (F - N / 2);
    return -1;
}

template <int LOG>
constexpr int threads_for() {
    constexpr int F = 1 << LOG;
    return (F / 16 < 64) ? 64 : (F / 16 > 256 ? 256 : F / 16);
}

}  // namespace

// ---------------------------------------------------------------------------
// rows_forward
// ---------------------------------------------------------------------------

// Grid rows per block of the row kernels: as many as fit 1024 threads and about
// 136 KB of LDS (one FFT buffer per row), so the column-major spectrum is
// written and read in segments of G consecutive rows.
template <typename R, int LOG>
constexpr int rows_per_block() {
    constexpr int nt = FftShape<LOG>::NT;
    constexpr int by_threads = 1024 / nt;
    constexpr int by_lds = static_cast<int>((136 * 1024) / (lds_padded_size(1 << LOG) * sizeof(cpx<R>)));
    constexpr int g = by_threads < by_lds ? by_threads : by_lds;
    constexpr int n = (1 << LOG) / 2;
    return g < 1 ? 1 : (g > n ? n : g);
}

// Row `row` of the grid, at centred positions n' mod F: z = rho + i rho d(n1) d(n2)
// (the type-2 deconvolution rides in the imaginary part), one F-point FFT; the
// transform of the real part on m = 0..N is the I1 half spectrum, that of the
// imaginary part on the Q window frequencies is the type-2 row window.
template <typename R, int LOG>
__global__ __launch_bounds__((FftShape<LOG>::NT * rows_per_block<R, LOG>())) void k_rows_forward(
    DevPlan P, const R* __restrict__ rho, R dir) {
    using Sh = FftShape<LOG>;
    constexpr int F = Sh::F;
    constexpr int N = F / 2;
    constexpr int NT = Sh::NT;
    constexpr int G = rows_per_block<R, LOG>();
    constexpr int LP = lds_padded_size(F);
    __shared__ cpx<R> lds_all[G * LP];
    const int g = threadIdx.x / NT;
    const int tid = threadIdx.x - g * NT;
    cpx<R>* lds = lds_all + g * LP;
    const cpx<R>* tw = static_cast<const cpx<R>*>(P.twr);
    const int row0 = xcd_logical_block(blockIdx.x, gridDim.x) * G;
    const int row = row0 + g;
    const double dy = P.deconv[row];
    const R* src = rho + static_cast<size_t>(row) * N;
    const cpx<R> zero = {R(0), R(0)};
    cpx<R> v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        if (i < 4 || i >= 12) {
            const int n1 = (i < 4) ? tid + NT * i + N / 2 : tid + NT * (i - 12);
            const R r = src[n1];
            v[i] = {r, static_cast<R>(static_cast<double>(r) * P.deconv[n1] * dy)};
        } else {
            v[i] = zero;
        }
    }
    fft_reg<R, LOG>(v, lds, tw, tid, dir);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) lds[lds_pad(tid + NT * i)] = v[i];
    __syncthreads();
    // outputs of the G rows, row index fastest: G-element runs of each column
    cpx<R>* xt = static_cast<cpx<R>*>(P.xt);
    for (int idx = threadIdx.x; idx < (N + 1) * G; idx += NT * G) {
        const int gg = idx % G;
        const int m = idx / G;
        const cpx<R>* l = lds_all + gg * LP;
        const cpx<R> a = l[lds_pad(m)];
        const cpx<R> b = l[lds_pad((F - m) & (F - 1))];
        // transform of the real part: X[m] = (Z[m] + conj Z[-m]) / 2
        xt[static_cast<size_t>(m) * N + row0 + gg] = {R(0.5) * (a.x + b.x), R(0.5) * (a.y - b.y)};
    }
    cpx<R>* tt = static_cast<cpx<R>*>(P.tt);
    for (int idx = threadIdx.x; idx < P.patch * G; idx += NT * G) {
        const int gg = idx % G;
        const int i = idx / G;
        const int lf = P.patch_lo + i;
        const cpx<R>* l = lds_all + gg * LP;
        const cpx<R> a = l[lds_pad(lf & (F - 1))];
        const cpx<R> b = l[lds_pad((-lf) & (F - 1))];
        // transform of the imaginary part: (Z[l] - conj Z[-l]) / (2i)
        tt[static_cast<size_t>(i) * N + row0 + gg] = {R(0.5) * (a.y + b.y), R(-0.5) * (a.x - b.x)};
    }
}

// ---------------------------------------------------------------------------
// cols_highfreq: FFT along y, multiplier, inverse FFT along y (in place in XT)
// ---------------------------------------------------------------------------

// Sequences per block of a register-FFT kernel: blocks of at least 256 threads.
template <int LOG>
constexpr int lines_per_block() {
    constexpr int nt = FftShape<LOG>::NT;
    return nt >= 256 ? 1 : 256 / nt;
}

template <typename R>
__device__ __forceinline__ R recip(R x) {
    if constexpr (sizeof(R) == 4) {
        const float r = __builtin_amdgcn_rcpf(x);
        return r * (2.0f - x * r);      // one Newton step: correctly rounded to within an ulp
    } else {
        return 1.0 / x;
    }
}

// Column m1 of the half spectrum (contiguous in XT, N values at centred y
// positions) is transformed along y with the zero padding implicit: in the
// register layout position tid + NT i holds a grid row only for i < 4
// (p < N/2) and i >= 12 (p >= F - N/2), so the other inputs are compile-time
// zeros and the inverse transform's outputs there are never formed.
template <typename R, int LOG>
__global__ __launch_bounds__(FftShape<LOG>::NT * lines_per_block<LOG>()) void k_cols_highfreq(DevPlan P, R dir) {
    using Sh = FftShape<LOG>;
    constexpr int F = Sh::F;
    constexpr int N = F / 2;
    constexpr int NT = Sh::NT;
    constexpr int G = lines_per_block<LOG>();
    __shared__ cpx<R> lds_all[G * lds_padded_size(F)];
    const int g = threadIdx.x / NT;
    const int tid = threadIdx.x - g * NT;
    cpx<R>* lds = lds_all + g * lds_padded_size(F);
    const cpx<R>* tw = static_cast<const cpx<R>*>(P.twr);
    const int m1 = xcd_logical_block(blockIdx.x, gridDim.x) * G + g;   // 0..N (+ idle lanes of the last block)
    const bool active = m1 <= N;
    cpx<R>* col = static_cast<cpx<R>*>(P.xt) + static_cast<size_t>(active ? m1 : 0) * N;
    const cpx<R> zero = {R(0), R(0)};
    cpx<R> v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        if (i < 4) {
            v[i] = active ? col[tid + NT * i + N / 2] : zero;
        } else if (i >= 12) {
            v[i] = active ? col[tid + NT * (i - 12)] : zero;
        } else {
            v[i] = zero;
        }
    }
    fft_reg<R, LOG>(v, lds, tw, tid, dir);
    // g1 = -(k_a^2/|k|^2) (1 - e^{-|k|^2/sigma^2}) / F^2 with
    // 1 - e^{-(a+b)} = A + B - A B, A = 1 - e^{-a}, B = 1 - e^{-b} (all terms >= 0)
    const int mc = active ? m1 : 0;
    const R a = static_cast<R>(P.gx[2 * mc]);
    const R A = static_cast<R>(P.gx[2 * mc + 1]);
    const R scale = static_cast<R>(P.inv_f2);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int m2 = tid + NT * i;
        const R b = static_cast<R>(P.gy[2 * m2]);
        const R B = static_cast<R>(P.gy[2 * m2 + 1]);
        const R num = P.component_y ? b : a;
        const R den = a + b;
        const R gfac = (den > R(0)) ? -(num * recip(den)) * (A + B - A * B) * scale : R(0);
        v[i] = cscale(v[i], gfac);
    }
    fft_reg<R, LOG>(v, lds, tw, tid, -dir);
    if (active) {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            if (i < 4) col[tid + NT * i + N / 2] = v[i];
            else if (i >= 12) col[tid + NT * (i - 12)] = v[i];
        }
    }
}

// ---------------------------------------------------------------------------
// cols_type2: FFT along y of the type-2 row window, keep the Q window rows
// ---------------------------------------------------------------------------
template <typename R, int LOG, int NT>
__global__ __launch_bounds__(NT) void k_cols_type2(DevPlan P, R dir) {
    constexpr int F = 1 << LOG;
    constexpr int N = F / 2;
    __shared__ cpx<R> buf[lds_padded_size(F)];
    __shared__ TwiddleLds<R, LOG> tw;
    const int tid = threadIdx.x;
    const int i1 = blockIdx.x;
    twiddle_fill<R, LOG>(tw, P.tw_lo, P.tw_hi, tid, NT);
    const cpx<R>* col = static_cast<const cpx<R>*>(P.tt) + static_cast<size_t>(i1) * N;
    for (int p = tid; p < F; p += NT) {
        const int n2 = pos_to_grid<LOG>(p);
        buf[lds_pad(p)] = (n2 >= 0) ? col[n2] : cpx<R>{R(0), R(0)};
    }
    __syncthreads();
    fft_lds<R, LOG, NT>(buf, tw, tid, dir);
    cpx<R>* win = static_cast<cpx<R>*>(P.win);
    for (int i2 = tid; i2 < P.patch; i2 += NT)
        win[static_cast<size_t>(i2) * P.patch + i1] = buf[lds_pad((P.patch_lo + i2) & (F - 1))];
}

// ---------------------------------------------------------------------------
// cols_type1: sum the spread tiles onto one column of the fine-grid window,
// FFT along y (only the Q window rows are non-zero), keep the N centred rows,
// times d(n2)
// ---------------------------------------------------------------------------

// Range of bins b (0 <= b < nb) whose tile starts at b * bin and covers window
// index i (i - b * bin in [0, E)).
__device__ __forceinline__ void covering_bins(int i, int bin, int E, int nb, int* lo, int* hi) {
    const int a = i - E + 1;
    int b0 = (a >= 0) ? (a + bin - 1) / bin : -((-a) / bin);   // ceil(a / bin)
    *lo = b0 > 0 ? b0 : 0;
    const int b1 = i / bin;
    *hi = b1 < nb - 1 ? b1 : nb - 1;
}

// b[i1][i2] = sum of the tile values of every subproblem whose tile covers
// window cell (i1, i2), in the fixed order (x period, x bin, y period, y bin,
// subproblem).  When the window is the whole periodic fine grid (Q = F) a
// tile may wrap around it, possibly more than once.
template <typename R>
__device__ __forceinline__ cpx<R> gather_tiles(const DevPlan& P, int i1, int i2) {
    const int q = P.patch, E = P.tile, bin = P.bin, nb = P.nb;
    const int periods = (q == P.n_fine) ? (q + E - 2) / q + 1 : 1;
    const cpx<R>* tiles = static_cast<const cpx<R>*>(P.tiles);
    R sx = 0, sy = 0, cx = 0, cy = 0;
    for (int t1 = 0; t1 < periods; ++t1) {
        const int x = i1 + t1 * q;
        int bx0, bx1;
        covering_bins(x, bin, E, nb, &bx0, &bx1);
        for (int bx = bx0; bx <= bx1; ++bx) {
            const int ox = x - bx * bin;
            for (int t2 = 0; t2 < periods; ++t2) {
                const int y = i2 + t2 * q;
                int by0, by1;
                covering_bins(y, bin, E, nb, &by0, &by1);
                for (int by = by0; by <= by1; ++by) {
                    const int oy = y - by * bin;
                    const int b = by * nb + bx;
                    for (int sidx = P.bin_start[b]; sidx < P.bin_start[b + 1]; ++sidx) {
                        const cpx<R> v = tiles[static_cast<size_t>(sidx) * E * E + oy * E + ox];
                        if constexpr (sizeof(R) == 4) {
                            const R yx = v.x - cx, tx = sx + yx;
                            cx = (tx - sx) - yx;
                            sx = tx;
                            const R yy = v.y - cy, ty = sy + yy;
                            cy = (ty - sy) - yy;
                            sy = ty;
                        } else {
                            sx += v.x;
                            sy += v.y;
                        }
                    }
                }
            }
        }
    }
    return {sx - cx, sy - cy};
}

template <typename R, int LOG, int NT>
__global__ __launch_bounds__(NT) void k_cols_type1(DevPlan P, R dir) {
    constexpr int F = 1 << LOG;
    constexpr int N = F / 2;
    __shared__ cpx<R> buf[lds_padded_size(F)];
    __shared__ TwiddleLds<R, LOG> tw;
    const int tid = threadIdx.x;
    const int i1 = blockIdx.x;
    twiddle_fill<R, LOG>(tw, P.tw_lo, P.tw_hi, tid, NT);
    for (int p = tid; p < F; p += NT) buf[lds_pad(p)] = {R(0), R(0)};
    __syncthreads();
    for (int i2 = tid; i2 < P.patch; i2 += NT)
        buf[lds_pad((P.patch_lo + i2) & (F - 1))] = gather_tiles<R>(P, i1, i2);
    __syncthreads();
    fft_lds<R, LOG, NT>(buf, tw, tid, dir);
    cpx<R>* u = static_cast<cpx<R>*>(P.u);
    for (int n2 = tid; n2 < N; n2 += NT) {
        const cpx<R> v = buf[lds_pad(centred_pos<LOG>(n2))];
        const double d = P.deconv[n2];
        u[static_cast<size_t>(n2) * P.patch + i1] = {static_cast<R>(v.x * d), static_cast<R>(v.y * d)};
    }
}

// ---------------------------------------------------------------------------
// rows_inverse: Phi row = Re IFFT(S1 + i H) + Im IFFT(S1 + i H) d(n1)
// ---------------------------------------------------------------------------

// For each of the block's G rows the full F-point row spectrum is assembled in
// LDS: the Hermitian extension of the I1 half spectrum (column m of XT, conj at
// F - m) plus i times the Hermitian part H[l] = (U[l] + conj U[-l]) / 2 of the
// type-1 row on the window frequencies.  One inverse FFT then gives I1 in the
// real part and Re(type-1 field) / d(n1) in the imaginary part.
template <typename R, int LOG>
__global__ __launch_bounds__((FftShape<LOG>::NT * rows_per_block<R, LOG>())) void k_rows_inverse(
    DevPlan P, R* __restrict__ out, R dir, int use_i1, int use_i2) {
    using Sh = FftShape<LOG>;
    constexpr int F = Sh::F;
    constexpr int N = F / 2;
    constexpr int NT = Sh::NT;
    constexpr int G = rows_per_block<R, LOG>();
    constexpr int LP = lds_padded_size(F);
    __shared__ cpx<R> lds_all[G * LP];
    const int g = threadIdx.x / NT;
    const int tid = threadIdx.x - g * NT;
    cpx<R>* lds = lds_all + g * LP;
    const cpx<R>* tw = static_cast<const cpx<R>*>(P.twr);
    const int row0 = xcd_logical_block(blockIdx.x, gridDim.x) * G;
    const int row = row0 + g;
    const cpx<R>* xt = static_cast<const cpx<R>*>(P.xt);
    const cpx<R>* u = static_cast<const cpx<R>*>(P.u);
    const int q = P.patch, lo = P.patch_lo;
    for (int idx = threadIdx.x; idx < (N + 1) * G; idx += NT * G) {
        const int gg = idx % G;
        const int m = idx / G;
        const int r = row0 + gg;
        cpx<R> x = {R(0), R(0)};
        if (use_i1) x = xt[static_cast<size_t>(m) * N + r];
        cpx<R> hh = {R(0), R(0)};
        if (use_i2) {
            const int ia = posmod_dev(m - lo, F);
            const int ib = posmod_dev(-m - lo, F);
            if (ia < q || ib < q) {
                const cpx<R>* urow = u + static_cast<size_t>(r) * q;
                const cpx<R> ua = (ia < q) ? urow[ia] : cpx<R>{R(0), R(0)};
                const cpx<R> ub = (ib < q) ? urow[ib] : cpx<R>{R(0), R(0)};
                hh = {R(0.5) * (ua.x + ub.x), R(0.5) * (ua.y - ub.y)};
            }
        }
        cpx<R>* l = lds_all + gg * LP;
        // position m: X + i H;  position F - m: conj X + i conj H
        l[lds_pad(m)] = {x.x - hh.y, x.y + hh.x};
        if (m > 0 && m < N) l[lds_pad(F - m)] = {x.x + hh.y, -x.y + hh.x};
    }
    __syncthreads();
    cpx<R> v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = lds[lds_pad(tid + NT * i)];
    fft_reg<R, LOG>(v, lds, tw, tid, dir);
    R* dst = out + static_cast<size_t>(row) * N;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        if (i < 4 || i >= 12) {
            const int n1 = (i < 4) ? tid + NT * i + N / 2 : tid + NT * (i - 12);
            dst[n1] = static_cast<R>(static_cast<double>(v[i].x) + static_cast<double>(v[i].y) * P.deconv[n1]);
        }
    }
}

// ---------------------------------------------------------------------------
// Kernel taps of the bin-sorted subproblems
// ---------------------------------------------------------------------------
namespace {

constexpr int kSubThreads = 256;
constexpr int kTileMax = kBinSize + kMaxKernelWidth - 1;

template <typename R>
struct SubLds {
    cpx<R> tile[kTileMax * kTileMax];
    R psx[kMaxNodesPerSub][kMaxKernelWidth];
    R psy[kMaxNodesPerSub][kMaxKernelWidth];
    int offx[kMaxNodesPerSub];
    int offy[kMaxNodesPerSub];
    cpx<R> val[kMaxNodesPerSub];
};

__device__ __forceinline__ double es_kernel_dev(double z, double beta) {
    return (fabs(z) < 1.0) ? exp(beta * (sqrt(1.0 - z * z) - 1.0)) : 0.0;
}

// Kernel values psi(u_j - l) for the w taps l = l0 .. l0+w-1 of every node of
// the subproblem (separable in x and y), and each node's first-tap offset in
// the tile.  FP64 evaluation, stored in the data precision.
template <typename R>
__device__ void subproblem_taps(const DevPlan& P, SubLds<R>& s, int tile_lo1, int tile_lo2, int first,
                                int count) {
    const int w = P.width;
    const double half = 0.5 * w;
    const int F = P.n_fine;
    for (int e = threadIdx.x; e < count * w * 2; e += kSubThreads) {
        const int axis = e / (count * w);
        const int r = e - axis * count * w;
        const int jj = r / w;
        const int t = r - jj * w;
        const int j = first + jj;
        const double u = axis ? P.uy[j] : P.ux[j];
        const int l0 = static_cast<int>(ceil(u - half));
        const R v = static_cast<R>(es_kernel_dev((u - (l0 + t)) / half, P.beta));
        if (axis == 0) {
            s.psx[jj][t] = v;
            if (t == 0) s.offx[jj] = P.patch_lo + posmod_dev(l0 - P.patch_lo, F) - tile_lo1;
        } else {
            s.psy[jj][t] = v;
            if (t == 0) s.offy[jj] = P.patch_lo + posmod_dev(l0 - P.patch_lo, F) - tile_lo2;
        }
    }
}

}  // namespace

// rho_hat_j = h^2 sum_taps b[l] psi(u_jx - l1) psi(u_jy - l2); a_j = q_j rho_hat_j
// (mode 0: q_j h^2 from the plan; mode 1: h^2 only, for the type-2 entry point).
template <typename R>
__global__ __launch_bounds__(kSubThreads) void k_interp(DevPlan P, cpx<R>* __restrict__ out, int mode) {
    __shared__ SubLds<R> s;
    const int* sub = P.sub + 4 * blockIdx.x;
    const int lo1 = sub[0], lo2 = sub[1], first = sub[2], count = sub[3];
    const int w = P.width;
    const int E = P.bin + w - 1;
    const int F = P.n_fine;
    const int q = P.patch;
    const cpx<R>* win = static_cast<const cpx<R>*>(P.win);
    for (int c = threadIdx.x; c < E * E; c += kSubThreads) {
        const int ca = c % E, cb = c / E;
        const int wi1 = posmod_dev(lo1 + ca - P.patch_lo, F);
        const int wi2 = posmod_dev(lo2 + cb - P.patch_lo, F);
        s.tile[c] = (wi1 < q && wi2 < q) ? win[static_cast<size_t>(wi2) * q + wi1] : cpx<R>{R(0), R(0)};
    }
    subproblem_taps<R>(P, s, lo1, lo2, first, count);
    __syncthreads();
    // 16 lanes per node, tree reduction over the lanes of the group
    const int lane = threadIdx.x & 15;
    const int group = threadIdx.x >> 4;
    const int ntap = w * w;
    for (int jj0 = 0; jj0 < count; jj0 += kSubThreads / 16) {
        const int jj = jj0 + group;
        cpx<R> acc = {R(0), R(0)};
        if (jj < count) {
            const int ox = s.offx[jj], oy = s.offy[jj];
            for (int t = lane; t < ntap; t += 16) {
                const int ay = t / w;
                const int ax = t - ay * w;
                const R k = s.psx[jj][ax] * s.psy[jj][ay];
                const cpx<R> b = s.tile[(oy + ay) * E + ox + ax];
                acc.x += b.x * k;
                acc.y += b.y * k;
            }
        }
#pragma unroll
        for (int off = 8; off > 0; off >>= 1) {
            acc.x += __shfl_xor(acc.x, off, 16);
            acc.y += __shfl_xor(acc.y, off, 16);
        }
        if (jj < count && lane == 0) {
            const int j = first + jj;
            const double scale = (mode == 0) ? P.q[j] * P.h2 : P.h2;
            out[j] = {static_cast<R>(acc.x * scale), static_cast<R>(acc.y * scale)};
        }
    }
}

// Tile of subproblem s: T_s[l] = sum_j a_j psi(l1 - u_jx) psi(l2 - u_jy) over the
// subproblem's nodes, for the E x E cells l of its bin's tile.  Each thread owns
// tile cells and sums the taps that land on them in node order (compensated
// summation in FP32), then writes the whole tile, zeros included, to the
// subproblem's own slot: no atomics, so the result is bitwise reproducible.
// The tiles are summed onto the fine-grid window by cols_type1.
template <typename R>
__global__ __launch_bounds__(kSubThreads) void k_spread(DevPlan P, const cpx<R>* __restrict__ coef) {
    __shared__ SubLds<R> s;
    const int* sub = P.sub + 4 * blockIdx.x;
    const int lo1 = sub[0], lo2 = sub[1], first = sub[2], count = sub[3];
    const int w = P.width;
    const int E = P.tile;
    subproblem_taps<R>(P, s, lo1, lo2, first, count);
    for (int jj = threadIdx.x; jj < count; jj += kSubThreads) s.val[jj] = coef[first + jj];
    __syncthreads();
    cpx<R>* tile = static_cast<cpx<R>*>(P.tiles) + static_cast<size_t>(blockIdx.x) * E * E;
    for (int c = threadIdx.x; c < E * E; c += kSubThreads) {
        const int ca = c % E, cb = c / E;
        R sx = 0, sy = 0, cx = 0, cy = 0;   // sums and compensations
        for (int jj = 0; jj < count; ++jj) {
            const int ax = ca - s.offx[jj];
            const int ay = cb - s.offy[jj];
            if (static_cast<unsigned>(ax) < static_cast<unsigned>(w) &&
                static_cast<unsigned>(ay) < static_cast<unsigned>(w)) {
                const R k = s.psx[jj][ax] * s.psy[jj][ay];
                const R vx = s.val[jj].x * k;
                const R vy = s.val[jj].y * k;
                if constexpr (sizeof(R) == 4) {
                    const R yx = vx - cx, tx = sx + yx;
                    cx = (tx - sx) - yx;
                    sx = tx;
                    const R yy = vy - cy, ty = sy + yy;
                    cy = (ty - sy) - yy;
                    sy = ty;
                } else {
                    sx += vx;
                    sy += vy;
                }
            }
        }
        tile[c] = {sx - cx, sy - cy};
    }
}

// ---------------------------------------------------------------------------
// Host-side launchers
// ---------------------------------------------------------------------------
namespace {

template <typename R, int LOG>
hipError_t launch_rows_forward(const DevPlan& P, const void* rho, R dir, hipStream_t s) {
    if (P.twr_count != FftShape<LOG>::tw_size()) return hipErrorInvalidValue;
    constexpr int G = rows_per_block<R, LOG>();
    hipLaunchKernelGGL((k_rows_forward<R, LOG>), dim3(P.n / G), dim3(FftShape<LOG>::NT * G), 0, s, P,
                       static_cast<const R*>(rho), dir);
    return hipGetLastError();
}

template <typename R, int LOG>
hipError_t launch_cols_highfreq(const DevPlan& P, R dir, hipStream_t s) {
    if (P.twr_count != FftShape<LOG>::tw_size()) return hipErrorInvalidValue;
    constexpr int G = lines_per_block<LOG>();
    const int blocks = (P.n + 1 + G - 1) / G;
    hipLaunchKernelGGL((k_cols_highfreq<R, LOG>), dim3(blocks), dim3(FftShape<LOG>::NT * G), 0, s, P, dir);
    return hipGetLastError();
}

template <typename R, int LOG>
hipError_t launch_cols_type2(const DevPlan& P, R dir, hipStream_t s) {
    constexpr int NT = threads_for<LOG>();
    hipLaunchKernelGGL((k_cols_type2<R, LOG, NT>), dim3(P.patch), dim3(NT), 0, s, P, dir);
    return hipGetLastError();
}

template <typename R, int LOG>
hipError_t launch_cols_type1(const DevPlan& P, R dir, hipStream_t s) {
    constexpr int NT = threads_for<LOG>();
    hipLaunchKernelGGL((k_cols_type1<R, LOG, NT>), dim3(P.patch), dim3(NT), 0, s, P, dir);
    return hipGetLastError();
}

template <typename R, int LOG>
hipError_t launch_rows_inverse(const DevPlan& P, void* out, R dir, int use_i1, int use_i2, hipStream_t s) {
    if (P.twr_count != FftShape<LOG>::tw_size()) return hipErrorInvalidValue;
    constexpr int G = rows_per_block<R, LOG>();
    hipLaunchKernelGGL((k_rows_inverse<R, LOG>), dim3(P.n / G), dim3(FftShape<LOG>::NT * G), 0, s, P,
                       static_cast<R*>(out), dir, use_i1, use_i2);
    return hipGetLastError();
}

#define PHI_DISPATCH_LOG(LOGV, CALL)        \
    switch (LOGV) {                         \
        case 4: { constexpr int L_ = 4; return CALL; }   \
        case 5: { constexpr int L_ = 5; return CALL; }   \
        case 6: { constexpr int L_ = 6; return CALL; }   \
        case 7: { constexpr int L_ = 7; return CALL; }   \
        case 8: { constexpr int L_ = 8; return CALL; }   \
        case 9: { constexpr int L_ = 9; return CALL; }   \
        case 10: { constexpr int L_ = 10; return CALL; } \
        case 11: { constexpr int L_ = 11; return CALL; } \
        case 12: { constexpr int L_ = 12; return CALL; } \
        case 13: { constexpr int L_ = 13; return CALL; } \
        default: return hipErrorInvalidValue;           \
    }

template <typename R>
hipError_t run_rows_forward(const DevPlan& P, const void* rho, R dir, hipStream_t s) {
    PHI_DISPATCH_LOG(P.log_fine, (launch_rows_forward<R, L_>(P, rho, dir, s)));
}
template <typename R>
hipError_t run_cols_highfreq(const DevPlan& P, R dir, hipStream_t s) {
    PHI_DISPATCH_LOG(P.log_fine, (launch_cols_highfreq<R, L_>(P, dir, s)));
}
template <typename R>
hipError_t run_cols_type2(const DevPlan& P, R dir, hipStream_t s) {
    PHI_DISPATCH_LOG(P.log_fine, (launch_cols_type2<R, L_>(P, dir, s)));
}
template <typename R>
hipError_t run_cols_type1(const DevPlan& P, R dir, hipStream_t s) {
    PHI_DISPATCH_LOG(P.log_fine, (launch_cols_type1<R, L_>(P, dir, s)));
}
template <typename R>
hipError_t run_rows_inverse(const DevPlan& P, void* out, R dir, int use_i1, int use_i2, hipStream_t s) {
    PHI_DISPATCH_LOG(P.log_fine, (launch_rows_inverse<R, L_>(P, out, dir, use_i1, use_i2, s)));
}

template <typename R>
hipError_t run_interp(const DevPlan& P, void* out, int mode, hipStream_t s) {
    hipLaunchKernelGGL((k_interp<R>), dim3(P.n_sub), dim3(kSubThreads), 0, s, P, static_cast<cpx<R>*>(out), mode);
    return hipGetLastError();
}

template <typename R>
hipError_t run_spread(const DevPlan& P, const void* coef, hipStream_t s) {
    hipLaunchKernelGGL((k_spread<R>), dim3(P.n_sub), dim3(kSubThreads), 0, s, P,
                       static_cast<const cpx<R>*>(coef));
    return hipGetLastError();
}

#define PHI_TRY(expr)                    \
    do {                                 \
        hipError_t e_ = (expr);          \
        if (e_ != hipSuccess) return e_; \
    } while (0)

// Records an event on s before kernel `name` when a timer is attached.
hipError_t mark(KernelTimer* t, const char* name, hipStream_t s) {
    if (!t) return hipSuccess;
    if (t->count >= KernelTimer::kMax) return hipErrorInvalidValue;
    t->names[t->count] = name;
    return hipEventRecord(t->ev[t->count++], s);
}

#define PHI_STEP(name, expr)                   \
    do {                                       \
        PHI_TRY(mark(timer, name, s));         \
        PHI_TRY(expr);                         \
    } while (0)

template <typename R>
hipError_t enqueue_typed(const DevPlan& P, Stage stage, const void* in, void* out, int adjoint, hipStream_t s,
                         KernelTimer* timer) {
    // forward solve: type-2 side and the first I1 transforms with e^{-...};
    // the transposed solve reverses every direction
    const R dir = adjoint ? R(1) : R(-1);
    switch (stage) {
        case Stage::Solve:
            PHI_STEP("rows_forward", (run_rows_forward<R>(P, in, dir, s)));
            PHI_STEP("cols_highfreq", (run_cols_highfreq<R>(P, dir, s)));
            PHI_STEP("cols_type2", (run_cols_type2<R>(P, dir, s)));
            PHI_STEP("interp", (run_interp<R>(P, P.pts, 0, s)));
            PHI_STEP("spread", (run_spread<R>(P, P.pts, s)));
            PHI_STEP("cols_type1", (run_cols_type1<R>(P, -dir, s)));
            PHI_STEP("rows_inverse", (run_rows_inverse<R>(P, out, -dir, 1, 1, s)));
            break;
        case Stage::HighFreq:
            PHI_STEP("rows_forward", (run_rows_forward<R>(P, in, dir, s)));
            PHI_STEP("cols_highfreq", (run_cols_highfreq<R>(P, dir, s)));
            PHI_STEP("rows_inverse", (run_rows_inverse<R>(P, out, -dir, 1, 0, s)));
            break;
        case Stage::LowFreq:
            PHI_STEP("rows_forward", (run_rows_forward<R>(P, in, dir, s)));
            PHI_STEP("cols_type2", (run_cols_type2<R>(P, dir, s)));
            PHI_STEP("interp", (run_interp<R>(P, P.pts, 0, s)));
            PHI_STEP("spread", (run_spread<R>(P, P.pts, s)));
            PHI_STEP("cols_type1", (run_cols_type1<R>(P, -dir, s)));
            PHI_STEP("rows_inverse", (run_rows_inverse<R>(P, out, -dir, 0, 1, s)));
            break;
        case Stage::Type2:
            PHI_STEP("rows_forward", (run_rows_forward<R>(P, in, dir, s)));
            PHI_STEP("cols_type2", (run_cols_type2<R>(P, dir, s)));
            PHI_STEP("interp", (run_interp<R>(P, out, 1, s)));
            break;
        case Stage::Type1:
            PHI_STEP("spread", (run_spread<R>(P, in, s)));
            PHI_STEP("cols_type1", (run_cols_type1<R>(P, R(1), s)));
            PHI_STEP("rows_inverse", (run_rows_inverse<R>(P, out, R(1), 0, 1, s)));
            break;
        default:
            return hipErrorInvalidValue;
    }
    return mark(timer, nullptr, s);   // end of the last kernel
}

}  // namespace

hipError_t enqueue(const DevPlan& P, Stage stage, const void* in, void* out, int adjoint, hipStream_t s,
                   KernelTimer* timer) {
    if (P.dtype == PHI_F32) return enqueue_typed<float>(P, stage, in, out, adjoint, s, timer);
    return enqueue_typed<double>(P, stage, in, out, adjoint, s, timer);
}

}  // namespace phi

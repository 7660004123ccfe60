// Device bodies of the solve's kernels (gfx950): each takes its work item and
// its LDS explicitly, so that the single-solve kernels (one item per block)
// and the batched kernels (a work table over many plans) share one code path.
// The block size every body expects is given next to it.
#pragma once

#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "fft_reg.hpp"
#include "solver_kernels.hpp"

namespace phi {

__device__ __forceinline__ int posmod_dev(int a, int b) {
    int r = a % b;
    return r < 0 ? r + b : r;
}


// ---------------------------------------------------------------------------
// rows_forward
// ---------------------------------------------------------------------------

// Distance between the LDS buffers of the sequences of one block: the padded
// length plus 8 entries, so that lanes working on the same position of
// different sequences fall into different banks.
__host__ __device__ constexpr int lds_group_stride(int f) { return lds_padded_size(f) + 8; }

// Grid rows per block of the row kernels: as many as fit 1024 threads and about
// 70 KB of LDS (one FFT buffer per row, two blocks per CU), so the column-major
// spectrum is written and read in segments of G consecutive rows (two rows in
// FP32, one in FP64 at the long transforms: measured best among 1, 2 and 4).
template <typename R, int LOG>
constexpr int rows_per_block() {
    constexpr int nt = FftShape<LOG>::NT;
    constexpr int by_threads = 1024 / nt;
    constexpr int by_lds = static_cast<int>((70 * 1024) / (lds_group_stride(1 << LOG) * sizeof(cpx<R>)));
    constexpr int n = (1 << LOG) / 2;
    int lim = by_threads < by_lds ? by_threads : by_lds;
    lim = lim < n ? lim : n;
    int g = 1;                      // largest power of two <= lim (the last block of a
    while (2 * g <= lim) g *= 2;    // grid whose side it does not divide is partly idle)
    return g;
}

// A grid line of n points (n even, F >= 2n) sits at the centred positions
// n' mod F of an F-point transform, n' = index - n/2: n' >= 0 at positions
// [0, n/2), n' < 0 at [F - n/2, F).  In the register layout (position
// p = tid + NT i) those are slots 0..3 and 12..15 (n/2 <= F/4), so slots 4..11
// are zero padding at compile time; the grid index of position p is
// p + n/2 (slots 0..3, p < n/2) or p - F + n/2 (slots 12..15, p >= F - n/2).
// The kernels address a line through one base pointer at index n/2 with the
// offsets p or p - F, so every load and store of a thread shares one address
// register.

// Rows of the grid, G per block, at centred positions n' mod F:
// z = rho + i rho d(n1) d(n2) (the type-2 deconvolution rides in the imaginary
// part), one F-point FFT; the transform of the real part on m = 0..F/2 (I1
// half spectrum) goes to the column-major XT, that of the imaginary part on
// the Q window frequencies (the type-2 row window) to TT.  Rows at or beyond
// N (the last block of a grid whose side G does not divide) transform zeros
// and store nothing.
// EXACT: the grid side is F/2 (a power of two at kappa = 2), so every bound
// below is a compile-time constant (the general form tests each slot and row).
template <typename R, int LOG, int DIR, int G, bool EXACT>
__device__ __forceinline__ void rows_forward_body(const DevPlan& P, const R* __restrict__ rho, int row0,
                                                  cpx<R>* lds_all) {
    using Sh = FftShape<LOG>;
    constexpr int F = Sh::F;
    constexpr int HALF = F / 2;
    constexpr int NT = Sh::NT;
    constexpr int LP = lds_group_stride(F);
    const int n = EXACT ? F / 2 : P.n;
    const int g = threadIdx.x / NT;
    const int tid = threadIdx.x - g * NT;
    cpx<R>* lds = lds_all + g * LP;
    const cpx<R>* tw = static_cast<const cpx<R>*>(P.twr);
    const bool row_ok = EXACT || row0 + g < n;
    const int row = row_ok ? row0 + g : n - 1;
    const double dy = P.deconv[row];
    // grid column n1 = position + N/2 (n' >= 0) or position - F + N/2 (n' < 0):
    // one base address per array serves every slot
    const int half = EXACT ? F / 4 : (n >> 1);
    const R* src = rho + static_cast<size_t>(row) * n + half;
    const double* dx = P.deconv + half;
    cpx<R> v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int p = tid + NT * i;
        v[i] = {R(0), R(0)};
        if (i < 4 || i >= 12) {
            const int o = (i < 4) ? p : p - F;
            const bool inside = (i < 4) ? (p < half) : (p >= F - half);
            if (row_ok && inside) {
                const R r = src[o];
                v[i] = {r, static_cast<R>(static_cast<double>(r) * dx[o] * dy)};
            }
        }
    }
    fft_reg<R, LOG, DIR>(v, lds, tw, tid);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) lds[lds_pad(tid + NT * i)] = v[i];
    __syncthreads();
    // outputs of the G rows, row index fastest: G-element runs of each column;
    // a compile-time number of passes with clamped indices
    cpx<R>* xt = static_cast<cpx<R>*>(P.xt);
    constexpr int ITEMS = (HALF + 1) * G;
    constexpr int PASSES = (ITEMS + NT * G - 1) / (NT * G);
#pragma unroll
    for (int k = 0; k < PASSES; ++k) {
        const int idx = threadIdx.x + k * NT * G;
        const int idc = idx < ITEMS ? idx : ITEMS - 1;
        const int gg = idc % G;
        const int m = idc / G;
        const cpx<R>* l = lds_all + gg * LP;
        const cpx<R> a = l[lds_pad(m)];
        const cpx<R> b = l[lds_pad((F - m) & (F - 1))];
        // transform of the real part: X[m] = (Z[m] + conj Z[-m]) / 2
        if (idx < ITEMS && (EXACT || row0 + gg < n))
            xt[static_cast<size_t>(m) * P.col_stride + row0 + gg] = {R(0.5) * (a.x + b.x), R(0.5) * (a.y - b.y)};
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
        if (EXACT || row0 + gg < n)
            tt[static_cast<size_t>(i) * P.col_stride + row0 + gg] = {R(0.5) * (a.y + b.y), R(-0.5) * (a.x - b.x)};
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
        // hardware estimate and two Newton steps (each doubles the correct bits):
        // within an ulp, at a third of the cost of an IEEE division
        double r = __builtin_amdgcn_rcp(x);
        r = fma(r, fma(-x, r, 1.0), r);
        return fma(r, fma(-x, r, 1.0), r);
    }
}

// The smallest positive normal number: added to a denominator that is either
// zero (where the numerator is zero too) or far above it, so the quotient is
// 0 at the origin without a comparison and unchanged elsewhere.
template <typename R>
__device__ __forceinline__ constexpr R tiny_normal() {
    if constexpr (sizeof(R) == 4) return 1.17549435e-38f;
    else return 2.2250738585072014e-308;
}

// Column m1 of the half spectrum (contiguous in XT, N values at centred y
// positions) is transformed along y with the zero padding implicit: in the
// register layout only slots 0..3 and 12..15 can hold grid rows (see above),
// so the other inputs are compile-time zeros and the inverse transform's
// outputs there are never formed.
// KIND selects the multiplier at compile time (separate instantiations, so that
// the DS multiplier's code is unchanged by the others):
//   0  -kx^2/|k|^2 or -ky^2/|k|^2 (P.component 0 / 1)
//   1  -kx ky/|k|^2
//   2  1/|k| with the Gaussian partition:  g1 = (1 - e^{-|k|^2/sigma^2}) / |k|
//   3  1/|k| with the erfc partition:      g1 = erf(|k|/sigma) / |k|
constexpr int kKindQuadratic = 0, kKindMixed = 1, kKindCoulombGauss = 2, kKindCoulombErfc = 3;

// erf(x)/x for x >= 0, an even entire function: the series 2/sqrt(pi) (1 - x^2/3)
// below a threshold where the next term (x^4/10) is below the precision's
// rounding, the library erf above it.
template <typename R>
__device__ __forceinline__ R erf_over_x(R x, R x2) {
    constexpr R two_over_sqrt_pi = R(1.1283791670955126);
    if constexpr (sizeof(R) == 4) {
        return x < 1e-2f ? two_over_sqrt_pi * (1.0f - x2 * (1.0f / 3.0f)) : erff(x) / x;
    } else {
        return x < 1e-5 ? two_over_sqrt_pi * (1.0 - x2 * (1.0 / 3.0)) : erf(x) / x;
    }
}

template <typename R, int LOG, int DIR, int G, int KIND, bool EXACT>
__device__ __forceinline__ void cols_highfreq_body(const DevPlan& P, int m1_base, cpx<R>* lds_all) {
    using Sh = FftShape<LOG>;
    constexpr int F = Sh::F;
    constexpr int HALF = F / 2;
    constexpr int NT = Sh::NT;
    const int n = EXACT ? F / 2 : P.n;
    const int g = threadIdx.x / NT;
    const int tid = threadIdx.x - g * NT;
    cpx<R>* lds = lds_all + g * lds_group_stride(F);
    const cpx<R>* tw = static_cast<const cpx<R>*>(P.twr);
    const int m1 = m1_base + g;   // 0..F/2 (+ idle lanes of the last block)
    const bool active = m1 <= HALF;
    // idle lanes load column F/2 and never store: no branch around the loads
    cpx<R>* col = static_cast<cpx<R>*>(P.xt) + static_cast<size_t>(active ? m1 : HALF) * P.col_stride;
    // rows n' >= 0 at positions [0, N/2), n' < 0 at [F - N/2, F): one base
    // address (row N/2 - position 0) serves every slot
    const int half = EXACT ? F / 4 : (n >> 1);
    const cpx<R>* base = col + half;
    cpx<R> v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int p = tid + NT * i;
        v[i] = {R(0), R(0)};
        if (i < 4) {
            if (p < half) v[i] = base[p];
        } else if (i >= 12) {
            if (p >= F - half) v[i] = base[p - F];
        }
    }
    fft_reg<R, LOG, DIR>(v, lds, tw, tid);
    // (b, 1 - e^{-b}) of the 16 rows this thread multiplies, fetched only now:
    // held through the transform they would take 32 more registers and, in
    // FP32, cut the resident blocks per CU from four to three
    const cpx<R>* gyr = static_cast<const cpx<R>*>(P.gyr);
    cpx<R> gb[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) gb[i] = gyr[tid + NT * i];
    // g1 = -(k_a k_b/|k|^2) (1 - e^{-|k|^2/sigma^2}) / F^2 with a = kx^2/sigma^2,
    // b = ky^2/sigma^2 and 1 - e^{-(a+b)} = A + B - A B, A = 1 - e^{-a},
    // B = 1 - e^{-b} (all terms >= 0); branch-free per point, g1(0) = 0.  The
    // numerator is a or b, or for the mixed component (kx/sigma)(ky/sigma) with
    // the signed frequency index of the point.
    // The mixed numerator is odd in each frequency, and a bin on a Nyquist line
    // (|index| = F/2) stands for +k and -k: it takes the mean of the multiplier
    // over them, 0 (also at the corner).
    const int mc = active ? m1 : HALF;
    const R a = static_cast<R>(P.gx[2 * mc]);
    const R A = static_cast<R>(P.gx[2 * mc + 1]);
    const R scale = static_cast<R>(P.inv_f2);
    const bool ycomp = P.component == 1;
    const R fs = static_cast<R>(P.freq_scale);
    const R fx = (mc == HALF) ? R(0) : static_cast<R>(mc) * fs;
    const R inv_sigma = static_cast<R>(P.inv_sigma);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const R b = gb[i].x;
        const R B = gb[i].y;
        R gfac;
        if constexpr (KIND == kKindCoulombGauss) {
            // (1 - e^{-(a+b)}) / (sigma sqrt(a+b)): 0 * finite at k = 0
            const R s2 = a + b + tiny_normal<R>();
            gfac = (A + B - A * B) * (inv_sigma * scale) / sqrt(s2);
        } else if constexpr (KIND == kKindCoulombErfc) {
            const R s2 = a + b;
            gfac = erf_over_x<R>(sqrt(s2), s2) * (inv_sigma * scale);
        } else {
            R num;
            if constexpr (KIND == kKindMixed) {
                const int p = tid + NT * i;                 // frequency index along y, FFT order
                const int ms = (p < HALF) ? p : p - F;      // p = F/2 (Nyquist) -> -F/2
                num = (p == HALF) ? R(0) : fx * (static_cast<R>(ms) * fs);
            } else {
                num = ycomp ? b : a;
            }
            // den = 0 only at k = 0, where num = 0: the quotient is 0 there
            const R den = a + b + tiny_normal<R>();
            gfac = -(num * recip(den)) * (A + B - A * B) * scale;
        }
        v[i] = cscale(v[i], gfac);
    }
    fft_reg<R, LOG, -DIR>(v, lds, tw, tid);
    if (active) {
        cpx<R>* out = col + half;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int p = tid + NT * i;
            if (i < 4) {
                if (p < half) out[p] = v[i];
            } else if (i >= 12) {
                if (p >= F - half) out[p - F] = v[i];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// cols_type2: FFT along y of the type-2 row window, keep the Q window rows
// ---------------------------------------------------------------------------
template <typename R, int LOG, int DIR, int G, bool EXACT>
__device__ __forceinline__ void cols_type2_body(const DevPlan& P, int i1_base, cpx<R>* lds_all) {
    using Sh = FftShape<LOG>;
    constexpr int F = Sh::F;
    constexpr int NT = Sh::NT;
    const int g = threadIdx.x / NT;
    const int tid = threadIdx.x - g * NT;
    cpx<R>* lds = lds_all + g * lds_group_stride(F);
    const cpx<R>* tw = static_cast<const cpx<R>*>(P.twr);
    const int q = P.patch;
    const int i1 = i1_base + g;
    const bool active = i1 < q;
    const cpx<R>* col = static_cast<const cpx<R>*>(P.tt) + static_cast<size_t>(active ? i1 : 0) * P.col_stride;
    const cpx<R> zero = {R(0), R(0)};
    const int half = EXACT ? F / 4 : (P.n >> 1);
    const cpx<R>* base = col + half;
    cpx<R> v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int p = tid + NT * i;
        v[i] = zero;
        if (i < 4) {
            if (active && p < half) v[i] = base[p];
        } else if (i >= 12) {
            if (active && p >= F - half) v[i] = base[p - F];
        }
    }
    fft_reg<R, LOG, DIR>(v, lds, tw, tid);
    cpx<R>* win = static_cast<cpx<R>*>(P.win);
    if (active) {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int i2 = posmod_dev(tid + NT * i - P.patch_lo, F);   // window row of this position
            if (i2 < q) win[static_cast<size_t>(i2) * q + i1] = v[i];
        }
    }
}

// ---------------------------------------------------------------------------
// nodes: interpolation, polar multiplier and spreading of one subproblem
// ---------------------------------------------------------------------------
// A subproblem is a run of at most 64 nodes whose first kernel taps lie in one
// bin of bin x bin window cells, so all their taps fall in the E x E tile
// (E = bin + w - 1) at the bin's corner.  The block stages that tile of the
// type-2 window, the nodes' tap values and first-tap offsets in LDS, then
//   interp:  c_j = sum_{t2} psi_y[t2] sum_{t1} tile[oy+t2][ox+t1] psi_x[t1]
//            (16 lanes per node, lane t2 sums its tap row, then a fixed
//            rotate-and-add tree across the 16 lanes)          [eq. (16), (12)]
//   a_j = q_j h^2 c_j                                          [eq. (12)]
//   spread:  T[cb][ca] = sum_j a_j psi_x[ca-ox_j] psi_y[cb-oy_j] (one thread per
//            tile cell, nodes in order, compensated in FP32)   [eq. (15)]
// and writes its whole tile T to its own slot: no atomics.  The tiles are
// summed onto the window by cols_type1 through a precomputed index list.
// MODE 0: all three steps; MODE 1: interp only, out[j] = h^2 c_j (type-2 stage);
// MODE 2: spread only, of coef (type-1 stage).  NTH threads per block: the
// order of every sum is fixed by kLanesPerNode and kSpreadParts alone, so
// blocks of any size give the same bits.
constexpr int kNodeThreads = 256;         // batched blocks
// one plan's subproblems in their own launch: 512 threads, so a block's tile
// loads, taps and spreading run in fewer rounds (graph replay on MI355X: the
// FP64 node stage 10.7 -> 9.3 us at 1024^2, the 1024^2 FP64 solve 64.2 -> 61.9 us)
constexpr int kNodeThreadsSingle = 512;
constexpr int kLanesPerNode = 16;
constexpr int kSpreadParts = 2;
constexpr int kTileMax = kMaxTile;

// WMAX: the widest kernel the block serves (kMaxEsWidth, or kMaxKernelWidth for
// the Gaussian), which sizes the tap store
template <typename R, int WMAX>
struct NodeLds {
    cpx<R> tile[kTileMax * kTileMax];
    R taps[kMaxNodesPerSub * 2 * WMAX];   // per node: w x-taps, then w y-taps
    int2 off[kMaxNodesPerSub];            // first-tap offset (x, y) in the tile
    double qh[kMaxNodesPerSub];   // q_j h^2
    cpx<R> val[kMaxNodesPerSub];
};

// Sum over the 16 lanes of each row of the wave (lanes 16r .. 16r + 15), in a
// fixed order: four rotate-and-add steps (rotations by 8, 4, 2, 1 lanes within
// the row, DPP row_ror on the vector ALU, no LDS round trip).  Every lane ends
// with the row's sum; lane 16r's association order is the same in every call.
template <int CTRL>
__device__ __forceinline__ float row_rotate(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double row_rotate(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(b & 0xffffffffll), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(double, (static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}
template <typename R>
__device__ __forceinline__ R row16_sum(R v) {
    constexpr int kRowRor = 0x120;   // DPP row_ror:n is kRowRor + n
    v += row_rotate<kRowRor + 8>(v);
    v += row_rotate<kRowRor + 4>(v);
    v += row_rotate<kRowRor + 2>(v);
    v += row_rotate<kRowRor + 1>(v);
    return v;
}

template <typename R>
__device__ __forceinline__ void kahan_add(R& s, R& c, R v) {
    if constexpr (sizeof(R) == 4) {
        const R y = v - c;
        const R t = s + y;
        c = (t - s) - y;
        s = t;
    } else {
        s += v;
    }
}

// x / d for 0 <= x < 1024 and 1 <= d <= 31 as (x * ceil(2^16 / d)) >> 16: the
// rounded-up reciprocal adds less than x / 2^16 < 1/64 to x / d, less than
// the gap 1/d between x / d and the next integer
__device__ __forceinline__ unsigned small_div_magic(int d) {
    return (65536u + static_cast<unsigned>(d) - 1u) / static_cast<unsigned>(d);
}
__device__ __forceinline__ int small_div(int x, unsigned magic) {
    return static_cast<int>((static_cast<unsigned>(x) * magic) >> 16);
}

// W: the kernel width when it is fixed at compile time (0: read from the plan).
// A fixed width lets the interpolation's tap loop unroll, so the LDS reads of a
// node's whole tap row issue together; the sums keep their order, so the bits
// are the same.
template <typename R, int MODE, int NTH, int WMAX, int W = 0>
__device__ __forceinline__ void nodes_body(const DevPlan& P, int sidx, const cpx<R>* __restrict__ coef,
                                           cpx<R>* __restrict__ out, NodeLds<R, WMAX>& s) {
    static_assert(W >= 0 && W <= WMAX, "a fixed width within the tap store");
    static_assert(NTH % kLanesPerNode == 0 && NTH % kSpreadParts == 0, "whole node and cell groups");
    static_assert(NTH >= kMaxNodesPerSub, "one thread per node for the node scalars");
    static_assert(kTileMax * kTileMax < 1024 && kTileMax <= 31 && WMAX * WMAX <= 1024 && WMAX <= kMaxKernelWidth,
                  "small_div covers the tile and tap indices");
    constexpr int TPT = (kMaxNodesPerSub * 2 * WMAX + NTH - 1) / NTH;   // taps per thread
    constexpr int CPT = (kTileMax * kTileMax + NTH - 1) / NTH;                     // tile cells per thread
    const int* sub = P.sub + 4 * sidx;
    const int bx = sub[0], by = sub[1], first = sub[2], count = sub[3];
    const int w = W > 0 ? W : P.width;
    const int E = P.tile, q = P.patch, bin = P.bin;
    const int w2 = 2 * w;
    const int x0 = bx * bin, y0 = by * bin;   // tile corner in window cells
    const unsigned magic_e = small_div_magic(E);
    // every global load of the block is issued before the first LDS store, so
    // their latencies overlap: the subproblem's taps (contiguous, w2 per node),
    // the per-node scalars, the type-2 window tile
    const R* taps = static_cast<const R*>(P.taps) + static_cast<size_t>(first) * w2;
    const int n_taps = count * w2;
    R tv[TPT];
#pragma unroll
    for (int k = 0; k < TPT; ++k) {
        const int e = threadIdx.x + k * NTH;
        tv[k] = e < n_taps ? taps[e] : R(0);
    }
    const int jn = threadIdx.x;
    const bool has_node = jn < count;
    int cx = 0, cy = 0;
    double qv = 0.0;
    cpx<R> cv = {R(0), R(0)};
    if (has_node) {
        cx = P.cell[2 * (first + jn)];
        cy = P.cell[2 * (first + jn) + 1];
        if constexpr (MODE == 0) qv = P.q[first + jn];
        if constexpr (MODE == 2) cv = coef[first + jn];
    }
    cpx<R> tl[CPT];
    if constexpr (MODE != 2) {
        // the window side is a power of two and tiles only wrap when the window
        // is the whole periodic fine grid
        const bool whole = (q == P.n_fine);
        const cpx<R>* win = static_cast<const cpx<R>*>(P.win);
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            const int c = threadIdx.x + k * NTH;
            const int cb = small_div(c, magic_e), ca = c - cb * E;
            int wx = x0 + ca, wy = y0 + cb;
            bool inside = c < E * E;
            if (whole) {
                wx &= q - 1;
                wy &= q - 1;
            } else {
                inside = inside && wx < q && wy < q;
            }
            tl[k] = inside ? win[static_cast<size_t>(wy) * q + wx] : cpx<R>{R(0), R(0)};
        }
    }
#pragma unroll
    for (int k = 0; k < TPT; ++k) {
        const int e = threadIdx.x + k * NTH;
        if (e < n_taps) s.taps[e] = tv[k];
    }
    if (has_node) {
        s.off[jn] = make_int2(cx - x0, cy - y0);
        if constexpr (MODE == 0) s.qh[jn] = qv * P.h2;
        if constexpr (MODE == 2) s.val[jn] = cv;
    }
    // the staged tile's rows are ES = E | 1 entries apart: an odd stride puts
    // the 16 lanes of a node, one tap row each, in distinct LDS banks
    const int ES = E | 1;
    if constexpr (MODE != 2) {
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            const int c = threadIdx.x + k * NTH;
            const int cb = small_div(c, magic_e), ca = c - cb * E;
            if (c < E * E) s.tile[cb * ES + ca] = tl[k];
        }
    }
    __syncthreads();
    if constexpr (MODE != 2) {
        static_assert(kLanesPerNode == 16, "one DPP row per node");
        const int lane = threadIdx.x % kLanesPerNode;
        for (int jj0 = 0; jj0 < count; jj0 += NTH / kLanesPerNode) {
            const int jj = jj0 + threadIdx.x / kLanesPerNode;
            cpx<R> acc = {R(0), R(0)};
            if (jj < count) {
                const int2 o = s.off[jj];
                const R* tj = s.taps + jj * w2;
                // lane t2 (and t2 + 16 for the widest Gaussian kernels) sums one
                // tap row: psi_y[t2] sum_t1 tile[oy+t2][ox+t1] psi_x[t1], four
                // taps at a time with clamped indices and zero weights past w,
                // so the loads of a chunk issue together without branches
                for (int t2 = lane; t2 < w; t2 += kLanesPerNode) {
                    const cpx<R>* trow = s.tile + (o.y + t2) * ES + o.x;
                    cpx<R> row = {R(0), R(0)};
                    auto chunk = [&](int t0) {
                        R k[4];
                        cpx<R> b[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const int t1 = min(t0 + u, w - 1);
                            const R kv = tj[t1];
                            k[u] = (t0 + u < w) ? kv : R(0);
                            b[u] = trow[t1];
                        }
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            row.x += b[u].x * k[u];
                            row.y += b[u].y * k[u];
                        }
                    };
                    if constexpr (W > 0) {
#pragma unroll
                        for (int t0 = 0; t0 < W; t0 += 4) chunk(t0);
                    } else {
                        for (int t0 = 0; t0 < w; t0 += 4) chunk(t0);
                    }
                    const R ky = tj[w + t2];
                    acc.x += row.x * ky;
                    acc.y += row.y * ky;
                }
            }
            acc.x = row16_sum(acc.x);
            acc.y = row16_sum(acc.y);
            if (jj < count && lane == 0) {
                const int j = first + jj;
                if constexpr (MODE == 1) {
                    out[j] = {static_cast<R>(acc.x * P.h2), static_cast<R>(acc.y * P.h2)};
                } else {
                    const double scale = s.qh[jj];
                    s.val[jj] = {static_cast<R>(acc.x * scale), static_cast<R>(acc.y * scale)};
                }
            }
        }
    }
    if constexpr (MODE == 1) return;
    if constexpr (MODE == 0) __syncthreads();
    // kSpreadParts threads per tile cell, each summing one run of the nodes (in
    // order), then a fixed shuffle tree; the node loop is unrolled and
    // branch-free so the LDS reads of several nodes are in flight together
    cpx<R>* tile_out = static_cast<cpx<R>*>(P.tiles) + static_cast<size_t>(sidx) * E * E;
    constexpr int U = 8;
    const int part = threadIdx.x % kSpreadParts;
    const int run = (count + kSpreadParts - 1) / kSpreadParts;
    const int j_lo = min(count, part * run);
    const int j_hi = min(count, j_lo + run);
    for (int c = threadIdx.x / kSpreadParts; c < E * E; c += NTH / kSpreadParts) {
        const int cb = small_div(c, magic_e), ca = c - cb * E;
        R sx = 0, sy = 0, kx = 0, ky = 0;
        for (int j0 = j_lo; j0 < j_hi; j0 += U) {
            R kk[U];
            cpx<R> vv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int jj = j0 + u;
                const bool valid = jj < j_hi;
                const int jc = valid ? jj : j_lo;
                const int2 o = s.off[jc];
                const int t1 = ca - o.x;
                const int t2 = cb - o.y;
                const bool in = valid && static_cast<unsigned>(t1) < static_cast<unsigned>(w) &&
                                static_cast<unsigned>(t2) < static_cast<unsigned>(w);
                const R* tj = s.taps + jc * w2;
                const R k = tj[in ? t1 : 0] * tj[w + (in ? t2 : 0)];
                kk[u] = in ? k : R(0);
                vv[u] = s.val[jc];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                kahan_add(sx, kx, vv[u].x * kk[u]);
                kahan_add(sy, ky, vv[u].y * kk[u]);
            }
        }
        R vx = sx - kx, vy = sy - ky;
#pragma unroll
        for (int off = kSpreadParts / 2; off > 0; off >>= 1) {
            vx += __shfl_xor(vx, off, kSpreadParts);
            vy += __shfl_xor(vy, off, kSpreadParts);
        }
        if (part == 0) tile_out[c] = {vx, vy};
    }
}

// ---------------------------------------------------------------------------
// cols_type1: sum the spread tiles onto one window column, FFT along y (only
// the Q window inputs are non-zero), keep the N centred rows, times d(n2)
// ---------------------------------------------------------------------------
// A block transforms COLS window columns (COLS = 1 or G).  Window cell
// (i1, i2) is the sum of the tile entries listed for it, in list order: 4
// lanes split the list, then a fixed shuffle tree; all threads of the block
// share the cells of its columns, so with COLS = 1 the length of the lists
// (set by the node count, not by N) is spread over a whole block at every
// grid size.  Column c is staged in group c's buffer; group g transforms
// column g % COLS (with COLS = 1 every group runs the same transform, which the
// block's barriers need anyway) and groups g < COLS store.
template <typename R, int LOG, int DIR, int G, int COLS, bool EXACT>
__device__ __forceinline__ void cols_type1_body(const DevPlan& P, int i1_base, cpx<R>* lds_all) {
    using Sh = FftShape<LOG>;
    constexpr int F = Sh::F;
    constexpr int NT = Sh::NT;
    constexpr int BT = NT * G;
    constexpr int L = 4;
    constexpr int LP = lds_group_stride(F);
    static_assert(COLS == 1 || COLS == G, "one column per block or one per group");
    static_assert(BT % L == 0, "the block splits into whole lane groups");
    const int g = threadIdx.x / NT;
    const int tid = threadIdx.x - g * NT;
    cpx<R>* lds = lds_all + g * LP;
    const cpx<R>* tw = static_cast<const cpx<R>*>(P.twr);
    const int q = P.patch;
    // reduced window columns, staged at the start of their groups' FFT buffers
    // (q <= F entries); the FFT's first barrier orders the groups' reads of
    // them before its writes
    const cpx<R>* tiles = static_cast<const cpx<R>*>(P.tiles);
    const int lane = threadIdx.x % L;
    for (int e = threadIdx.x / L; e < COLS * q; e += BT / L) {
        const int c = e / q;
        const int i2 = e - c * q;
        const int i1 = i1_base + c;
        const int cell = (i1 < q ? i1 : 0) * q + i2;
        const int k0 = P.contrib_start[cell], k1 = P.contrib_start[cell + 1];
        R sx = 0, sy = 0, kx = 0, ky = 0;
        // batches of U entries per lane: all index loads, then all value loads,
        // then the sums in list order
        constexpr int U = 8;
        for (int base = k0 + lane; base < k1; base += L * U) {
            int idx[U];
#pragma unroll
            for (int u = 0; u < U; ++u) idx[u] = (base + u * L < k1) ? P.contrib[base + u * L] : -1;
            cpx<R> t[U];
#pragma unroll
            for (int u = 0; u < U; ++u) t[u] = (idx[u] >= 0) ? tiles[idx[u]] : cpx<R>{R(0), R(0)};
#pragma unroll
            for (int u = 0; u < U; ++u) {
                kahan_add(sx, kx, t[u].x);
                kahan_add(sy, ky, t[u].y);
            }
        }
        R vx = sx - kx, vy = sy - ky;
#pragma unroll
        for (int off = L / 2; off > 0; off >>= 1) {
            vx += __shfl_xor(vx, off, L);
            vy += __shfl_xor(vy, off, L);
        }
        if (lane == 0) lds_all[c * LP + i2] = {vx, vy};
    }
    // the deconvolution factors of the stored rows, fetched before the
    // transform (slots outside the crop read the factor of row N/2)
    const int half = EXACT ? F / 4 : (P.n >> 1);
    const double* dy = P.deconv + half;
    double dpre[8];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        if (i < 4 || i >= 12) {
            const int p = tid + NT * i;
            const int o = (i < 4) ? p : p - F;
            const bool inside = (i < 4) ? (p < half) : (p >= F - half);
            dpre[i < 4 ? i : i - 8] = dy[inside ? o : 0];
        }
    }
    __syncthreads();
    const int c = g % COLS;
    const int i1 = i1_base + c;
    const bool active = i1 < q;
    const cpx<R>* staged = lds_all + c * LP;
    cpx<R> v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int i2 = posmod_dev(tid + NT * i - P.patch_lo, F);
        v[i] = (active && i2 < q) ? staged[i2] : cpx<R>{R(0), R(0)};
    }
    fft_reg<R, LOG, DIR>(v, lds, tw, tid);
    if (active && g < COLS) {
        cpx<R>* u = static_cast<cpx<R>*>(P.u) + static_cast<size_t>(half) * q + i1;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int p = tid + NT * i;
            if (i < 4 || i >= 12) {
                const int o = (i < 4) ? p : p - F;     // grid row n2 = o + N/2
                const bool inside = (i < 4) ? (p < half) : (p >= F - half);
                if (inside) {
                    const double d = dpre[i < 4 ? i : i - 8];
                    u[static_cast<ptrdiff_t>(o) * q] = {static_cast<R>(v[i].x * d), static_cast<R>(v[i].y * d)};
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// rows_inverse: Phi row = Re IFFT(S1 + i H) + Im IFFT(S1 + i H) d(n1)
// ---------------------------------------------------------------------------

// For each of the block's G rows the full F-point row spectrum is assembled in
// LDS: the Hermitian extension of the I1 half spectrum (column m of XT, conj at
// F - m) plus i times the Hermitian part H[l] = (U[l] + conj U[-l]) / 2 of the
// type-1 row on the window frequencies.  One inverse FFT then gives I1 in the
// real part and Re(type-1 field) / d(n1) in the imaginary part.  Rows at or
// beyond N (the last block of a grid whose side G does not divide) transform
// zeros and store nothing.
template <typename R, int LOG, int DIR, bool USE_I1, bool USE_I2, int G, bool EXACT>
__device__ __forceinline__ void rows_inverse_body(const DevPlan& P, R* __restrict__ out, int row0,
                                                  cpx<R>* lds_all) {
    using Sh = FftShape<LOG>;
    constexpr int F = Sh::F;
    constexpr int HALF = F / 2;
    constexpr int NT = Sh::NT;
    constexpr int LP = lds_group_stride(F);
    const int n = EXACT ? F / 2 : P.n;
    const int g = threadIdx.x / NT;
    const int tid = threadIdx.x - g * NT;
    cpx<R>* lds = lds_all + g * LP;
    const cpx<R>* tw = static_cast<const cpx<R>*>(P.twr);
    const cpx<R>* xt = static_cast<const cpx<R>*>(P.xt);
    const cpx<R>* u = static_cast<const cpx<R>*>(P.u);
    const int q = P.patch, lo = P.patch_lo;
    // (F/2+1) G entries (column m, row gg), row index fastest; every load is
    // issued unconditionally (clamped index) so that all of them are in flight
    // at once
    constexpr int ITEMS = (HALF + 1) * G;
    constexpr int PASSES = (ITEMS + NT * G - 1) / (NT * G);
#pragma unroll
    for (int k = 0; k < PASSES; ++k) {
        const int idx = threadIdx.x + k * NT * G;
        const int idc = idx < ITEMS ? idx : ITEMS - 1;
        const int gg = idc % G;
        const int m = idc / G;
        const int r = (EXACT || row0 + gg < n) ? row0 + gg : n - 1;   // rows past N read row N - 1, never stored
        cpx<R> x = {R(0), R(0)};
        if constexpr (USE_I1) x = xt[static_cast<size_t>(m) * P.col_stride + r];
        cpx<R> hh = {R(0), R(0)};
        // only frequencies |m| <= Q/2 meet the window (m - lo or -m - lo in
        // [0, Q) mod F); pass k covers m in [k NT, (k+1) NT), so the later
        // passes skip the window loads altogether (a uniform branch)
        if (USE_I2 && k * NT <= (q >> 1)) {
            const int ia = posmod_dev(m - lo, F);
            const int ib = posmod_dev(-m - lo, F);
            const cpx<R>* urow = u + static_cast<size_t>(r) * q;
            const cpx<R> ua0 = urow[ia < q ? ia : q - 1];
            const cpx<R> ub0 = urow[ib < q ? ib : q - 1];
            const cpx<R> ua = (ia < q) ? ua0 : cpx<R>{R(0), R(0)};
            const cpx<R> ub = (ib < q) ? ub0 : cpx<R>{R(0), R(0)};
            hh = {R(0.5) * (ua.x + ub.x), R(0.5) * (ua.y - ub.y)};
        }
        // position m: X + i H;  position F - m: conj X + i conj H (the clamped
        // duplicate of the last entry rewrites the same values)
        cpx<R>* l = lds_all + gg * LP;
        l[lds_pad(m)] = {x.x - hh.y, x.y + hh.x};
        if (m > 0 && m < HALF) l[lds_pad(F - m)] = {x.x + hh.y, -x.y + hh.x};
    }
    // the deconvolution factors of the stored slots, fetched before the
    // transform so that their latency overlaps it (slots outside the crop read
    // the factor of row N/2)
    const int half = EXACT ? F / 4 : (n >> 1);
    const double* dx = P.deconv + half;
    double dpre[8];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        if (i < 4 || i >= 12) {
            const int p = tid + NT * i;
            const int o = (i < 4) ? p : p - F;
            const bool inside = (i < 4) ? (p < half) : (p >= F - half);
            dpre[i < 4 ? i : i - 8] = dx[inside ? o : 0];
        }
    }
    __syncthreads();
    cpx<R> v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = lds[lds_pad(tid + NT * i)];
    fft_reg<R, LOG, DIR>(v, lds, tw, tid);
    if (EXACT || row0 + g < n) {
        R* dst = out + static_cast<size_t>(row0 + g) * n + half;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int p = tid + NT * i;
            if (i < 4 || i >= 12) {
                const int o = (i < 4) ? p : p - F;
                const bool inside = (i < 4) ? (p < half) : (p >= F - half);
                if (inside)
                    dst[o] = static_cast<R>(static_cast<double>(v[i].x) +
                                            static_cast<double>(v[i].y) * dpre[i < 4 ? i : i - 8]);
            }
        }
    }
}

}  // namespace phi

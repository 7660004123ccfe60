// Register-resident Stockham FFT of one power-of-two sequence of length
// F = 2^LOG, computed by a group of NT = F/16 threads that each hold 16 points.
//
// Layout contract: on entry and on exit thread `tid` of the group holds the
// points at positions tid + NT*i, i = 0..15, in v[i].  Stage 0 is radix 16
// with no twiddles; the following stages are radix 16 except a last radix
// 2^(LOG mod 4) stage.  Between stages the points are exchanged through one LDS
// buffer of F complex values (padded every 16 entries); the last stage writes
// its outputs back to registers in the same positions the first stage reads,
// so a forward transform, a pointwise multiply and an inverse transform chain
// without an extra exchange, and zero inputs / unused outputs at positions
// known at compile time are pruned by the compiler.
//
// Stage s of radix R with sub-transform length p (the product of the previous
// radices) and NB = F/R butterflies: butterfly b reads positions b + t NB,
// multiplies input t by W_{pR}^{t k} (k = b mod p), takes a length-R DFT in
// registers, and writes output t to position (b - k) R + k + t p (Stockham
// auto-sort: natural order out, no bit reversal).
//
// Twiddles come from a per-stage table in device memory, rounded once to the
// data precision from FP64 values: stage s (s >= 1) holds W_{p R}^{t k} for
// t = 1..R-1, k = 0..p-1 at index (t-1) p + k, and the stages are stored back
// to back in order.  Forward tables; the inverse takes conjugates.  (FP64
// radix-16 stages read four of a butterfly's powers and multiply out the
// rest; see stage_twiddles.)
//
// DIR = -1: X(k) = sum_j x(j) e^{-2 pi i k j / F} (forward DFT, Sec. 2.2,
// eq. (13)); DIR = +1: the same sum with e^{+...} (eq. (14) times F).  The
// direction is a template parameter so that every sign folds into the code.
#pragma once

#include "device_common.hpp"

namespace phi {

// The 16th roots of unity e^{DIR 2 pi i a / 16}, a = 0..7 (DIR = -1 forward,
// +1 inverse, fixed at compile time).  FP64: correctly rounded constants.
// FP32: cos(pi/8) and sin(pi/8) are taken a few ulps from the true values
// (angle error 7e-8 rad) such that c^2 + s^2 = 1 + 7e-9 instead of the
// correctly rounded pair's 1 - 5.7e-8: every butterfly level then scales the energy of its rotated
// half by a factor much closer to 1, so a long chain of transforms (a time
// stepper) does not lose norm systematically.  (For pi/4 no float pair does
// better than the correctly rounded one, 1 - 3.4e-8.)
template <typename R, int DIR>
__device__ __forceinline__ cpx<R> root16(int a) {
    constexpr double C64[8] = {1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
                               0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613};
    constexpr double S64[8] = {0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613,
                               1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173};
    constexpr float c8 = 0.9238795638084412f, s8 = 0.3826833665370941f;
    constexpr float r4 = 0.70710678118654752440f;
    constexpr float C32[8] = {1.0f, c8, r4, s8, 0.0f, -s8, -r4, -c8};
    constexpr float S32[8] = {0.0f, s8, r4, c8, 1.0f, c8, r4, s8};
    if constexpr (sizeof(R) == 4) return {C32[a], static_cast<float>(DIR) * S32[a]};
    else return {static_cast<R>(C64[a]), static_cast<R>(DIR * S64[a])};
}

// x times DIR i
template <typename R, int DIR>
__device__ __forceinline__ cpx<R> mul_i(cpx<R> a) {
    if constexpr (DIR > 0) return {-a.y, a.x};
    else return {a.y, -a.x};
}

// In-register DFT of length RAD (1, 2, 4, 8; 16 is specialised below) by
// even/odd splitting:
// v[k] <- sum_j v[j] e^{DIR 2 pi i j k / RAD}.
template <int RAD, typename R, int DIR>
struct RegDft {
    __device__ __forceinline__ static void run(cpx<R>* v) {
        constexpr int H = RAD / 2;
        cpx<R> e[H], o[H];
#pragma unroll
        for (int t = 0; t < H; ++t) {
            e[t] = v[2 * t];
            o[t] = v[2 * t + 1];
        }
        RegDft<H, R, DIR>::run(e);
        RegDft<H, R, DIR>::run(o);
#pragma unroll
        for (int k = 0; k < H; ++k) {
            cpx<R> t;
            if (k == 0) {
                t = o[k];
            } else if (4 * k == RAD) {
                t = mul_i<R, DIR>(o[k]);
            } else {
                t = cmul(o[k], root16<R, DIR>(k * (16 / RAD)));
            }
            v[k] = cadd(e[k], t);
            v[k + H] = csub(e[k], t);
        }
    }
};

template <typename R, int DIR>
struct RegDft<1, R, DIR> {
    __device__ __forceinline__ static void run(cpx<R>*) {}
};

// Length-4 DFT in place: 16 real additions, the factor DIR i folded into them.
template <typename R, int DIR>
__device__ __forceinline__ void dft4(cpx<R>& a0, cpx<R>& a1, cpx<R>& a2, cpx<R>& a3) {
    const cpx<R> t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3);
    const cpx<R> t3 = mul_i<R, DIR>(csub(a1, a3));
    a0 = cadd(t0, t2);
    a2 = csub(t0, t2);
    a1 = cadd(t1, t3);
    a3 = csub(t1, t3);
}

// x times e^{DIR 2 pi i a / 16}: the eighth roots of unity (a even) as a
// swap or the sum / difference of the parts times 1/sqrt(2); general angles as
// two products and two fused multiply-adds.
template <typename R, int DIR, int A>
__device__ __forceinline__ cpx<R> rot16(cpx<R> x) {
    constexpr int a = A & 15;
    if constexpr (a == 0) {
        return x;
    } else if constexpr (a == 4) {
        return mul_i<R, DIR>(x);
    } else if constexpr (a == 8) {
        return {-x.x, -x.y};
    } else if constexpr (a == 12) {
        return mul_i<R, -DIR>(x);
    } else if constexpr (a == 2 || a == 6 || a == 10 || a == 14) {
        const R r = root16<R, 1>(2).x;                      // 1/sqrt(2)
        // (x.x + i x.y)(c + i s) with c, s = +-r
        constexpr int cs = (a == 2 || a == 14) ? 1 : -1;      // sign of the cosine
        constexpr int sn = ((a == 2 || a == 6) ? 1 : -1) * DIR; // sign of the sine
        const R re = cs > 0 ? (sn > 0 ? x.x - x.y : x.x + x.y) : (sn > 0 ? -x.x - x.y : -x.x + x.y);
        const R im = cs > 0 ? (sn > 0 ? x.x + x.y : x.y - x.x) : (sn > 0 ? x.x - x.y : -x.x - x.y);
        return {r * re, r * im};
    } else if constexpr (a < 8) {
        return cmul(x, root16<R, DIR>(a));
    } else {
        const cpx<R> w = root16<R, DIR>(a - 8);
        return cmul(x, cpx<R>{-w.x, -w.y});
    }
}

// Length 16 as 4 x 4 (n = 4 n1 + n2, k = k1 + 4 k2): DFT4 over n1 for each n2,
// twiddles W16^{n2 k1}, DFT4 over n2 for each k1.  Of the nine twiddles one is
// a swap (W^4) and four are eighth roots (W^2, W^6), so it takes 128 real
// additions and four general complex products, against ten products in the
// radix-2 splitting.
template <typename R, int DIR>
struct RegDft<16, R, DIR> {
    __device__ __forceinline__ static void run(cpx<R>* v) {
#pragma unroll
        for (int n2 = 0; n2 < 4; ++n2) dft4<R, DIR>(v[n2], v[n2 + 4], v[n2 + 8], v[n2 + 12]);
        // v[n2 + 4 k1] now holds the inner transform y[n2][k1]
        v[5] = rot16<R, DIR, 1>(v[5]);
        v[9] = rot16<R, DIR, 2>(v[9]);
        v[13] = rot16<R, DIR, 3>(v[13]);
        v[6] = rot16<R, DIR, 2>(v[6]);
        v[10] = rot16<R, DIR, 4>(v[10]);
        v[14] = rot16<R, DIR, 6>(v[14]);
        v[7] = rot16<R, DIR, 3>(v[7]);
        v[11] = rot16<R, DIR, 6>(v[11]);
        v[15] = rot16<R, DIR, 9>(v[15]);
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) dft4<R, DIR>(v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]);
        // v[4 k1 + k2] holds X[k1 + 4 k2]: transpose the 4 x 4 register block
        cpx<R> t[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) t[i] = v[i];
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
            for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = t[4 * k1 + k2];
    }
};

template <int LOG>
struct FftShape {
    static constexpr int F = 1 << LOG;
    static constexpr int NT = F / 16;                  // threads per sequence
    static constexpr int S16 = LOG / 4;                // radix-16 stages
    static constexpr int REM = LOG % 4;                // radix 2^REM final stage (0: none)
    static constexpr int NSTAGE = S16 + (REM ? 1 : 0);
    static_assert(LOG >= 4, "FFT length must be at least 16");

    static constexpr int radix(int s) { return (s < S16) ? 16 : (1 << REM); }
    static constexpr int span(int s) {                 // p of stage s
        int p = 1;
        for (int i = 0; i < s; ++i) p *= radix(i);
        return p;
    }
    static constexpr int tw_offset(int s) {            // start of stage s in the table
        int off = 0;
        for (int i = 1; i < s; ++i) off += (radix(i) - 1) * span(i);
        return off;
    }
    static constexpr int tw_size() { return tw_offset(NSTAGE); }
};

// x times the twiddle w (DIR = -1) or its conjugate (DIR = +1); the table holds e^{-i theta}.
template <typename R, int DIR>
__device__ __forceinline__ cpx<R> tw_mul(cpx<R> x, cpx<R> w) {
    if constexpr (DIR < 0) return {x.x * w.x - x.y * w.y, x.x * w.y + x.y * w.x};
    else return {x.x * w.x + x.y * w.y, x.y * w.x - x.x * w.y};
}

// Twiddles of stage S (S >= 1) for this thread: w[c (RAD-1) + t - 1] multiplies
// input t of butterfly c.  At most 15 per stage.  FP64 radix-16 stages load
// W^k, W^2k, W^4k and W^8k and form the other eleven powers by products (at
// most three roundings each, ~1e-16): four loads instead of fifteen, which the
// long FP64 transforms, two waves per SIMD, feel more than the extra products
// (2048^2 FP64 solve 143 -> 136 us).  FP32 keeps the table values (rounded
// once), which its error budget and its norm preservation need.
template <typename R, int LOG, int S>
__device__ __forceinline__ void stage_twiddles(cpx<R> (&w)[16], const cpx<R>* __restrict__ tw, int tid) {
    using Sh = FftShape<LOG>;
    if constexpr (S > 0 && S < Sh::NSTAGE) {
        constexpr int RAD = Sh::radix(S);
        constexpr int P = Sh::span(S);
        constexpr int C = 16 / RAD;
        if constexpr (sizeof(R) == 8 && RAD == 16) {
            const cpx<R>* b = tw + Sh::tw_offset(S) + (tid & (P - 1));
            const cpx<R> w1 = b[0], w2 = b[P], w4 = b[3 * P], w8 = b[7 * P];
            w[0] = w1;
            w[1] = w2;
            w[2] = cmul(w2, w1);
            w[3] = w4;
            w[4] = cmul(w4, w1);
            w[5] = cmul(w4, w2);
            w[6] = cmul(w4, w[2]);
            w[7] = w8;
#pragma unroll
            for (int t = 0; t < 7; ++t) w[8 + t] = cmul(w8, w[t]);
        } else {
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const int k = (tid + Sh::NT * c) & (P - 1);
#pragma unroll
                for (int t = 1; t < RAD; ++t) w[c * (RAD - 1) + t - 1] = tw[Sh::tw_offset(S) + (t - 1) * P + k];
            }
        }
    }
}

// Stage S of the transform.  v holds the thread's 16 points in the register
// layout; stages after the first read their inputs from LDS.  w holds this
// stage's twiddles on entry and the next stage's on exit: they are fetched
// before the exchange so that their latency overlaps the barrier and LDS traffic.
template <typename R, int LOG, int S, int DIR>
__device__ __forceinline__ void fft_stage(cpx<R> (&v)[16], cpx<R> (&w)[16], cpx<R>* lds,
                                          const cpx<R>* __restrict__ tw, int tid) {
    using Sh = FftShape<LOG>;
    constexpr int F = Sh::F;
    constexpr int NT = Sh::NT;
    constexpr int RAD = Sh::radix(S);
    constexpr int P = Sh::span(S);
    constexpr int C = 16 / RAD;          // butterflies per thread (butterfly b reads b + t F/RAD)
    constexpr bool LAST = (S == Sh::NSTAGE - 1);
    if constexpr (S > 0) {
        // inputs of this stage: positions tid + NT i
#pragma unroll
        for (int i = 0; i < 16; ++i) v[i] = lds[lds_pad(tid + NT * i)];
        if constexpr (!LAST) __syncthreads();   // all reads done before this stage overwrites
    }
    cpx<R> x[C][RAD];
#pragma unroll
    for (int c = 0; c < C; ++c) {
#pragma unroll
        for (int t = 0; t < RAD; ++t) {
            x[c][t] = v[c + C * t];
            if constexpr (S > 0) {
                if (t > 0) x[c][t] = tw_mul<R, DIR>(x[c][t], w[c * (RAD - 1) + t - 1]);
            }
        }
    }
    if constexpr (!LAST) stage_twiddles<R, LOG, S + 1>(w, tw, tid);
#pragma unroll
    for (int c = 0; c < C; ++c) RegDft<RAD, R, DIR>::run(x[c]);
    if constexpr (LAST) {
        // output position b + t NB: the same register slot
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
            for (int t = 0; t < RAD; ++t) v[c + C * t] = x[c][t];
    } else {
        // the buffer may still be read by the group's previous use (stage 0)
        if constexpr (S == 0) __syncthreads();
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const int b = tid + NT * c;
            const int k = b & (P - 1);
            const int base = (b - k) * RAD + k;
#pragma unroll
            for (int t = 0; t < RAD; ++t) lds[lds_pad(base + t * P)] = x[c][t];
        }
        __syncthreads();
    }
}

template <typename R, int LOG, int S, int DIR>
__device__ __forceinline__ void fft_stages_from(cpx<R> (&v)[16], cpx<R> (&w)[16], cpx<R>* lds,
                                                const cpx<R>* __restrict__ tw, int tid) {
    if constexpr (S < FftShape<LOG>::NSTAGE) {
        fft_stage<R, LOG, S, DIR>(v, w, lds, tw, tid);
        fft_stages_from<R, LOG, S + 1, DIR>(v, w, lds, tw, tid);
    }
}

// The whole transform.  Every thread of the block must call it (it contains
// block-wide barriers); `lds` is this group's buffer of lds_padded_size(F)
// complex values.  The transform begins with a barrier before its first LDS
// write, so it may follow any earlier reads of the buffer (including another
// transform) directly; it ends without one, so a caller that writes the buffer
// afterwards must synchronise first.
template <typename R, int LOG, int DIR>
__device__ __forceinline__ void fft_reg(cpx<R> (&v)[16], cpx<R>* lds, const cpx<R>* __restrict__ tw, int tid) {
    cpx<R> w[16];
    fft_stages_from<R, LOG, 0, DIR>(v, w, lds, tw, tid);
}

}  // namespace phi

// Power-of-two complex FFT of one sequence held in LDS, computed by a group of
// NT threads with the Stockham auto-sort scheme (radix 16 stages plus one
// radix-2/4/8 stage): each stage reads n/R butterfly inputs at stride n/R,
// applies the twiddles W_{pR}^{t k}, a radix-R DFT in registers, and writes the
// outputs to their sorted positions (j - k) R + k + t p, so the result is in
// natural order with no bit reversal.  The transform is in place in one LDS
// buffer: every thread holds its n/NT values in registers across a barrier.
//
// Twiddles come from two small tables in LDS built from the plan's FP64 values:
// W_n^m = HI[m >> s] * LO[m & (2^s - 1)], two correctly rounded factors, so the
// FP32 path never uses a recurrence or a single-precision sin/cos.
//
// dir = -1: F(k) = sum_j f(j) e^{-2 pi i k j / n} (forward, Sec. 2.2, eq. 13);
// dir = +1: the same sum with e^{+...} (unnormalised inverse, eq. 14 times n).
#pragma once

#include "device_common.hpp"

namespace phi {

// cos / sin of 2 pi a / 16, a = 0..7 (exact constants of the 16th roots of unity).
template <typename R>
__device__ __forceinline__ cpx<R> root16(int a, R dir) {
    constexpr double C[8] = {1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
                             0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613};
    constexpr double S[8] = {0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613,
                             1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173};
    return {static_cast<R>(C[a]), dir * static_cast<R>(S[a])};
}

// In-register DFT of length RAD (2, 4, 8, 16) by even/odd splitting.
template <int RAD, typename R>
struct RegDft {
    __device__ __forceinline__ static void run(cpx<R>* v, R dir) {
        constexpr int H = RAD / 2;
        cpx<R> e[H], o[H];
#pragma unroll
        for (int t = 0; t < H; ++t) {
            e[t] = v[2 * t];
            o[t] = v[2 * t + 1];
        }
        RegDft<H, R>::run(e, dir);
        RegDft<H, R>::run(o, dir);
#pragma unroll
        for (int k = 0; k < H; ++k) {
            cpx<R> t;
            if (k == 0) {
                t = o[k];
            } else if (4 * k == RAD) {
                t = cmul_si(o[k], dir);
            } else {
                t = cmul(o[k], root16<R>(k * (16 / RAD), dir));
            }
            v[k] = cadd(e[k], t);
            v[k + H] = csub(e[k], t);
        }
    }
};

template <typename R>
struct RegDft<1, R> {
    __device__ __forceinline__ static void run(cpx<R>*, R) {}
};

// Twiddle tables in LDS for an FFT of length 2^LOG.
template <typename R, int LOG>
struct TwiddleLds {
    static constexpr int S_LOG = (LOG + 1) / 2;
    static constexpr int N_LO = 1 << S_LOG;
    static constexpr int N_HI = (1 << LOG) >> S_LOG;
    cpx<R> lo[N_LO];
    cpx<R> hi[N_HI];
};

// Fill the tables (forward sign) from the plan's FP64 arrays; the
// caller synchronises before use.
template <typename R, int LOG>
__device__ __forceinline__ void twiddle_fill(TwiddleLds<R, LOG>& tw, const double* lo, const double* hi,
                                             int tid, int nthreads) {
    for (int i = tid; i < TwiddleLds<R, LOG>::N_LO; i += nthreads) tw.lo[i] = load_cpx<R>(lo + 2 * i);
    for (int i = tid; i < TwiddleLds<R, LOG>::N_HI; i += nthreads) tw.hi[i] = load_cpx<R>(hi + 2 * i);
}

template <typename R, int LOG>
__device__ __forceinline__ cpx<R> twiddle(const TwiddleLds<R, LOG>& tw, int m, R dir) {
    constexpr int S = TwiddleLds<R, LOG>::S_LOG;
    cpx<R> w = cmul(tw.hi[m >> S], tw.lo[m & ((1 << S) - 1)]);
    // tables hold e^{-i theta}; dir = +1 needs the conjugate
    w.y = -dir * w.y;
    return w;
}

// One Stockham stage of radix RAD with sub-transform length p.
template <typename R, int LOG, int NT, int RAD>
__device__ __forceinline__ void stockham_stage(cpx<R>* buf, const TwiddleLds<R, LOG>& tw, int p, int tid,
                                               R dir) {
    constexpr int N = 1 << LOG;
    constexpr int NB = N / RAD;                     // butterflies in this stage
    constexpr int PER = (NB + NT - 1) / NT;         // butterflies per thread
    cpx<R> v[PER][RAD];
#pragma unroll
    for (int b = 0; b < PER; ++b) {
        const int j = tid + b * NT;
        if (NB % NT == 0 || j < NB) {
            const int k = j & (p - 1);
            // twiddle exponent step: W_{pR}^{t k} = W_N^{t k N/(pR)}
            const int step = k * (N / (p * RAD));
#pragma unroll
            for (int t = 0; t < RAD; ++t) {
                cpx<R> x = buf[lds_pad(j + t * NB)];
                if (t > 0 && p > 1) x = cmul(x, twiddle<R, LOG>(tw, t * step, dir));
                v[b][t] = x;
            }
            RegDft<RAD, R>::run(v[b], dir);
        }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < PER; ++b) {
        const int j = tid + b * NT;
        if (NB % NT == 0 || j < NB) {
            const int k = j & (p - 1);
            const int base = (j - k) * RAD + k;
#pragma unroll
            for (int t = 0; t < RAD; ++t) buf[lds_pad(base + t * p)] = v[b][t];
        }
    }
    __syncthreads();
}

// Full FFT of length 2^LOG in buf (padded LDS layout).  Must be called by all
// NT threads of the group; begins and ends with the data in LDS, synchronised.
template <typename R, int LOG, int NT>
__device__ __forceinline__ void fft_lds(cpx<R>* buf, const TwiddleLds<R, LOG>& tw, int tid, R dir) {
    constexpr int N16 = LOG / 4;        // radix-16 stages
    constexpr int REM = LOG % 4;        // one final stage of radix 2^REM
    int p = 1;
#pragma unroll
    for (int s = 0; s < N16; ++s) {
        stockham_stage<R, LOG, NT, 16>(buf, tw, p, tid, dir);
        p *= 16;
    }
    if constexpr (REM == 1) stockham_stage<R, LOG, NT, 2>(buf, tw, p, tid, dir);
    if constexpr (REM == 2) stockham_stage<R, LOG, NT, 4>(buf, tw, p, tid, dir);
    if constexpr (REM == 3) stockham_stage<R, LOG, NT, 8>(buf, tw, p, tid, dir);
}

}  // namespace phi

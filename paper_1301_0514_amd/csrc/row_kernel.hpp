// row_kernel.hpp -- the row-pass kernel: one or more rows of length N per
// workgroup, kept in registers, transformed by a Stockham FFT whose stages
// exchange data through LDS, and driven by a RowProgram.
#pragma once

#include "device_common.hpp"
#include "fft_plan.hpp"
#include "lds_layout.hpp"
#include "row_program.h"
#include "transpose_tile.hpp"

#include <type_traits>

namespace scint {

// position of element p in an exchange of the fixed layout
template <int L> __device__ __forceinline__ int lds_index(int p) {
    constexpr int sh = lds_pad_shift<L>();
    return sh > 0 ? p + (p >> sh) : p;
}

// ---------------------------------------------------------------- twiddles
// a[r] *= W^r (r = 1 .. R-1) uses only a few table entries: within a group of
// G (8, 5 or 4) consecutive powers W^1, W^2 (and W^4 for G = 8) are loaded
// and W^3 = W^1 W^2, W^5 = W^1 W^4, W^6 = W^2 W^4, W^7 = W^3 W^4 formed (W^4 =
// W^2 W^2 for G = 5); across groups W^(gG + b) = W^(gG) W^b with W^(gG)
// loaded -- every twiddle within three multiplications of table values.
template <int R> constexpr int twiddle_group() {
    return (R % 8 == 0) ? 8 : (R % 5 == 0) ? 5 : (R % 4 == 0) ? 4 : R;
}
template <int R> constexpr int tw_nbase() {
    constexpr int G = twiddle_group<R>();
    return (G == 8 ? 3 : G == 5 ? 2 : G - 1) + (R / G - 1);
}
// power of W held in base slot b
template <int R> constexpr int tw_base_power(int b) {
    constexpr int G = twiddle_group<R>();
    constexpr int nin = G == 8 ? 3 : G == 5 ? 2 : G - 1;
    if (b < nin) return G == 8 ? (1 << b) : b + 1;
    return (b - nin + 1) * G;
}

// Twiddle cache.  Butterfly j = t + i T of stage s uses W_{Ns R}^{r k},
// k = j mod Ns.  If T is a multiple of Ns, k = t mod Ns for every i (mode 1);
// if Ns is a multiple of T, k = t + (i mod Ns/T) T and W^{r k} =
// W^{r t} W^{r (i mod Ns/T) T}, the second factor a compile-time constant
// (mode 2).  Either way a thread's base twiddles depend on t alone, so each
// workgroup copies them to LDS once per launch; other stages (mode 0) read
// the table in global memory.
template <int L, int V> constexpr int tw_mode(int s) {
    using P = Plan<L, V>;
    const int Ns = stage_ns<L, V>(s);
    if (s == 0 || Ns == 1) return 0;
    if (P::T % Ns == 0) return 1;
    if (Ns % P::T == 0) return 2;
    return 0;
}
template <int L, int V> constexpr int tw_cache_count(int s) {
    const int m = tw_mode<L, V>(s);
    return m == 1 ? stage_ns<L, V>(s) : m == 2 ? Plan<L, V>::T : 0;
}
template <int L, int V> constexpr int tw_nbase_at(int s) {
    constexpr int NS = Plan<L, V>::NS;
    int n = 0;
    for (int q = 0; q < NS; ++q)
        if (q == s) {
            const int R = Plan<L, V>::R[q];
            const int G = (R % 8 == 0) ? 8 : (R % 5 == 0) ? 5 : (R % 4 == 0) ? 4 : R;
            n = (G == 8 ? 3 : G == 5 ? 2 : G - 1) + (R / G - 1);
        }
    return n;
}
template <int L, int V> constexpr int tw_cache_offset(int s) {
    int off = 0;
    for (int q = 1; q < s; ++q) off += tw_cache_count<L, V>(q) * tw_nbase_at<L, V>(q);
    return off;
}
template <int L, int V> constexpr int tw_cache_entries() { return tw_cache_offset<L, V>(Plan<L, V>::NS); }

// exp(-2 pi i r c / M) for r < R, at compile time
template <int R, long long C, long long M> struct TwConst {
    double c[R], s[R];
    constexpr TwConst() : c(), s() {
        for (int r = 0; r < R; ++r) {
            SinCos v = sincos2pi(-(long long)r * C, M);
            c[r] = v.c;
            s[r] = v.s;
        }
    }
};

template <typename Real, int L, int V = 0> struct RowCfg {
    using P = Plan<L, V>;
    static constexpr int T = P::T;
    static constexpr int ELEM = 2 * (int)sizeof(Real);
    // elements of a row's exchange buffer (the largest exchange layout)
    static constexpr int LDS_STRIDE = exch_buffer_length<L, V>(ELEM);
    static constexpr int B_THREADS = T >= 256 ? 1 : 256 / T;
    static constexpr int B_LDS = (P::NS > 1) ? ((65536 / (LDS_STRIDE * ELEM)) > 0 ? 65536 / (LDS_STRIDE * ELEM) : 1)
                                             : B_THREADS;
    static constexpr int B = B_THREADS < B_LDS ? B_THREADS : B_LDS;  // rows per workgroup
    static constexpr int THREADS = T * B;
    // LDS: the FFT exchange buffers, then the twiddle cache when it fits (two
    // workgroups per CU kept where the rows allowed two), or at least one
    // double per thread for the row reductions.
    static constexpr int FFT_LDS_BYTES = (P::NS > 1) ? B * LDS_STRIDE * ELEM : 0;
    static constexpr int TWC_BYTES = tw_cache_entries<L, V>() * ELEM;
    static constexpr bool TWC_ON =
        TWC_BYTES > 0 && (FFT_LDS_BYTES <= 80 * 1024 ? FFT_LDS_BYTES + TWC_BYTES <= 80 * 1024
                                                     : FFT_LDS_BYTES + TWC_BYTES <= 160 * 1024);
    static constexpr int RED_LDS_BYTES = THREADS * 8;
    static constexpr int USED_BYTES = FFT_LDS_BYTES + (TWC_ON ? TWC_BYTES : 0);
    static constexpr int LDS_BYTES = USED_BYTES > RED_LDS_BYTES ? USED_BYTES : RED_LDS_BYTES;
    // lower bound on the occupancy the register allocator must keep: two
    // waves per SIMD (up to 256 VGPRs), which the heaviest programs need
    // without spilling; lighter programs use fewer registers anyway.  Rows of
    // 10000 and more in 8-wave workgroups whose LDS lets two share a CU ask
    // for four (up to 128 VGPRs), so that the registers let them too.
#ifndef SCINT_WAVES_PER_EU
#define SCINT_WAVES_PER_EU 2
#endif
    static constexpr int WAVES_WG = (THREADS + 63) / 64;
    static constexpr int WAVES_PER_EU =
        (L >= 10000 && WAVES_WG == 8 && 2 * LDS_BYTES <= 160 * 1024 && SCINT_WAVES_PER_EU < 4) ? 4
                                                                                                 : SCINT_WAVES_PER_EU;
    // Mixed-radix rows of 10000 and more: each FFT stage (and each loop
    // iteration) sees an opaque copy of the thread index, so that the
    // per-element LDS addresses, which the padding makes nonlinear in the
    // element index, are formed where they are used.  Otherwise the compiler
    // shares them between the forward and inverse transforms and across the
    // wavelength loop, and under the 128 VGPRs of the 1000-thread plans (or
    // of two 500-thread workgroups per CU at 10000) keeps them in scratch:
    // up to 668 bytes per thread at 20000, reloaded right before the LDS
    // writes.  The power-of-two rows keep them in registers (a few programs
    // spill 12-72 bytes): forming them per stage there adds about 10 % to the
    // VALU instructions of the instruction-bound 8192 passes, and made the
    // 8192 smear 7 % slower.
#ifndef SCINT_REMAT_MIN_L
#define SCINT_REMAT_MIN_L 10000
#endif
#ifndef SCINT_REMAT_POW2
#define SCINT_REMAT_POW2 0
#endif
    static constexpr bool REMAT_T = L >= SCINT_REMAT_MIN_L && (SCINT_REMAT_POW2 || (L & (L - 1)) != 0);
};

// ---------------------------------------------------------------- FFT
// the group powers p[b] = W^b (b < G) from the base values (slots as in
// tw_base_power), and the twiddle of power r
template <typename Real, int R> struct TwGroup {
    static constexpr int G = twiddle_group<R>();
    static constexpr int NIN = G == 8 ? 3 : G == 5 ? 2 : G - 1;
    cpx<Real> p[G];
    cpx<Real> base[R / G];
    __device__ __forceinline__ void build(const cpx<Real> *bv) {
        p[0] = {(Real)1, (Real)0};
        if constexpr (G == 8) {
            p[1] = bv[0];
            p[2] = bv[1];
            p[4] = bv[2];
            p[3] = cmul(p[1], p[2]);
            p[5] = cmul(p[1], p[4]);
            p[6] = cmul(p[2], p[4]);
            p[7] = cmul(p[3], p[4]);
        } else if constexpr (G == 5) {
            p[1] = bv[0];
            p[2] = bv[1];
            p[3] = cmul(p[1], p[2]);
            p[4] = cmul(p[2], p[2]);
        } else {
#pragma unroll
            for (int b = 1; b < G; ++b) p[b] = bv[b - 1];
        }
        base[0] = {(Real)1, (Real)0};
#pragma unroll
        for (int g = 1; g < R / G; ++g) base[g] = bv[NIN + g - 1];
    }
    __device__ __forceinline__ cpx<Real> w(int r) const {
        const int g = r / G, b = r % G;
        return g == 0 ? p[b] : (b == 0 ? base[g] : cmul(base[g], p[b]));
    }
};

// a[r] *= W^r (r >= 1) with the base values bv[] of the butterfly's k; for
// mode 2 butterflies past the first block of T, also by the constant
// W_M^{r c} (M = Ns R, c = (i mod Ns/T) T)
template <typename Real, int R, long long C, long long M>
__device__ __forceinline__ void apply_twiddles(cpx<Real> (&a)[R], const TwGroup<Real, R> &tg) {
    if constexpr (C == 0) {
#pragma unroll
        for (int r = 1; r < R; ++r) a[r] = cmul(a[r], tg.w(r));
    } else {
        constexpr TwConst<R, C, M> K{};
#pragma unroll
        for (int r = 1; r < R; ++r) a[r] = cmul(a[r], cmul(tg.w(r), cpx<Real>{(Real)K.c[r], (Real)K.s[r]}));
    }
}

template <typename Real, int R> __device__ __forceinline__ void load_bases(cpx<Real> *bv, const cpx<Real> *w) {
#pragma unroll
    for (int b = 0; b < tw_nbase<R>(); ++b) bv[b] = w[tw_base_power<R>(b)];
}

template <typename Real, int L, int V, int s, int i = 0>
__device__ __forceinline__ void stage_butterflies(cpx<Real> (&v)[(Plan<L, V>::E)], cpx<Real> *lds, int t,
                                                  const cpx<Real> *__restrict__ tw, const cpx<Real> *twc,
                                                  TwGroup<Real, Plan<L, V>::R[s]> &tg);

template <typename Real, int L, int V, int s>
__device__ __forceinline__ void fft_stage(cpx<Real> (&v)[(Plan<L, V>::E)], cpx<Real> *lds, int t,
                                          const cpx<Real> *__restrict__ tw, const cpx<Real> *twc) {
    using P = Plan<L, V>;
    constexpr int E = P::E, T = P::T, R = P::R[s];
    constexpr int Ns = stage_ns<L, V>(s);
    constexpr int mode = tw_mode<L, V>(s);
    constexpr bool last = (s == P::NS - 1);
    // t as seen by this stage's butterflies (see RowCfg::REMAT_T)
    int ts = t;
    if constexpr (RowCfg<Real, L, V>::REMAT_T) asm volatile("" : "+v"(ts));
    TwGroup<Real, R> tg;
    if constexpr (mode != 0 && RowCfg<Real, L, V>::TWC_ON) {
        // the thread's base twiddles, once for all its butterflies of the stage
        cpx<Real> bv[tw_nbase<R>()];
        const cpx<Real> *src = twc + tw_cache_offset<L, V>(s) + (mode == 1 ? ts % Ns : ts) * tw_nbase<R>();
#pragma unroll
        for (int b = 0; b < tw_nbase<R>(); ++b) bv[b] = src[b];
        tg.build(bv);
    }
    stage_butterflies<Real, L, V, s, 0>(v, lds, ts, tw, twc, tg);
    if constexpr (!last) {
        __syncthreads();
        constexpr ExchLayout lay = exch_layout<L, V>(s, 2 * (int)sizeof(Real));
        if constexpr (lay.linear) {
            // f(t + m T) = f(t) + m (T + T / P): one address, then offsets
            constexpr int step = T + (lay.P > 0 ? T / lay.P : 0);
            const int q = lay.P > 0 ? ts + (int)((unsigned)ts / (unsigned)lay.P) : ts;
#pragma unroll
            for (int m = 0; m < E; ++m) v[m] = lds[q + m * step];
        } else {
#pragma unroll
            for (int m = 0; m < E; ++m) v[m] = lds[lds_index<L>(ts + m * T)];
        }
        __syncthreads();
        fft_stage<Real, L, V, s + 1>(v, lds, t, tw, twc);
    }
}

template <typename Real, int L, int V, int s, int i>
__device__ __forceinline__ void stage_butterflies(cpx<Real> (&v)[(Plan<L, V>::E)], cpx<Real> *lds, int t,
                                                  const cpx<Real> *__restrict__ tw, const cpx<Real> *twc,
                                                  TwGroup<Real, Plan<L, V>::R[s]> &tg) {
    using P = Plan<L, V>;
    constexpr int E = P::E, T = P::T, R = P::R[s], Q = E / R;
    constexpr int Ns = stage_ns<L, V>(s);
    constexpr int mode = tw_mode<L, V>(s);
    constexpr bool last = (s == P::NS - 1);
    if constexpr (i < Q) {
        const int j = t + i * T;
        const int k = (Ns == 1) ? 0 : (j % Ns);
        cpx<Real> a[R];
#pragma unroll
        for (int r = 0; r < R; ++r) a[r] = v[i + r * Q];
        if constexpr (Ns > 1) {
            if constexpr (mode != 0 && RowCfg<Real, L, V>::TWC_ON) {
                constexpr long long C = (mode == 2) ? (long long)(i % (Ns / T)) * T : 0;
                apply_twiddles<Real, R, C, (long long)Ns * R>(a, tg);
            } else {
                // keep the compiler from hoisting twiddle loads out of loops
                // over wavelengths (they would stay live in registers)
                asm volatile("" ::: "memory");
                cpx<Real> bv[tw_nbase<R>()];
                load_bases<Real, R>(bv, tw + twiddle_offset<L, V>(s) + k * R);
                tg.build(bv);
                apply_twiddles<Real, R, 0, 1>(a, tg);
            }
        }
        Dft<R, -1, Real>::run(a);
        if constexpr (last) {
#pragma unroll
            for (int r = 0; r < R; ++r) v[i + r * Q] = a[r];
        } else {
            const int base = (j - k) * R + k;
            constexpr ExchLayout lay = exch_layout<L, V>(s, 2 * (int)sizeof(Real));
            if constexpr (lay.linear) {
                // f(base + r Ns) = f(base) + r (Ns + Ns / P) if P divides Ns,
                // f(base) + r Ns if the butterfly's outputs share one period
                constexpr int step = Ns + ((lay.P > 0 && Ns % lay.P == 0) ? Ns / lay.P : 0);
                const int q = lay.P > 0 ? base + (int)((unsigned)base / (unsigned)lay.P) : base;
#pragma unroll
                for (int r = 0; r < R; ++r) lds[q + r * step] = a[r];
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r) lds[lds_index<L>(base + r * Ns)] = a[r];
            }
        }
        stage_butterflies<Real, L, V, s, i + 1>(v, lds, t, tw, twc, tg);
    }
}

// Copies each workgroup's base twiddles to the LDS cache (before the first
// FFT; the caller synchronises).
template <typename Real, int L, int V, int s = 1>
__device__ __forceinline__ void fill_tw_cache(cpx<Real> *twc, const cpx<Real> *__restrict__ tw, int tid, int nthr) {
    if constexpr (s < Plan<L, V>::NS) {
        constexpr int mode = tw_mode<L, V>(s);
        if constexpr (mode != 0) {
            constexpr int R = Plan<L, V>::R[s], nb = tw_nbase<R>(), cnt = tw_cache_count<L, V>(s);
            cpx<Real> *dst = twc + tw_cache_offset<L, V>(s);
            const cpx<Real> *src = tw + twiddle_offset<L, V>(s);
            for (int e = tid; e < cnt * nb; e += nthr) {
                const int idx = e / nb, b = e - idx * nb;
                dst[e] = src[idx * R + tw_base_power<R>(b)];
            }
        }
        fill_tw_cache<Real, L, V, s + 1>(twc, tw, tid, nthr);
    }
}

// Forward DFT of the register row (natural order in, natural order out).
template <typename Real, int L, int V>
__device__ __forceinline__ void fft_forward(cpx<Real> (&v)[(Plan<L, V>::E)], cpx<Real> *lds, int t,
                                            const cpx<Real> *__restrict__ tw, const cpx<Real> *twc) {
    fft_stage<Real, L, V, 0>(v, lds, t, tw, twc);
}

// ---------------------------------------------------------------- pointwise
// exp(2 pi i turns) with the argument reduced to [-1/2, 1/2] in FP64 and the
// sine/cosine evaluated in the working precision.
template <typename Real> __device__ __forceinline__ cpx<Real> expi_turns(double turns);
template <> __device__ __forceinline__ cpx<float> expi_turns<float>(double turns) {
    const double f = turns - rint(turns);
#ifndef SCINT_FAST_SINCOS
#define SCINT_FAST_SINCOS 1
#endif
#if SCINT_FAST_SINCOS
    // hardware sine/cosine of 2 pi x (x in turns, |x| <= 1/2; absolute error
    // about 1.2e-7 measured on gfx950, the same order as FP32 rounding)
    const float x = (float)f;
    return {__builtin_amdgcn_cosf(x), __builtin_amdgcn_sinf(x)};
#else
    float s, c;
    sincospif((float)(2.0 * f), &s, &c);
    return {c, s};
#endif
}
template <> __device__ __forceinline__ cpx<double> expi_turns<double>(double turns) {
    const double f = turns - rint(turns);
    double s, c;
    sincospi(2.0 * f, &s, &c);
    return {c, s};
}

// Random phase spectrum coefficient at Fourier pixel (kx, ky) of realisation r.
template <typename Real>
__device__ __forceinline__ cpx<Real> spectrum_coeff(int kx, int ky, int N, uint32_t r,
                                                    const RowProgram &p);

template <>
__device__ __forceinline__ cpx<float> spectrum_coeff<float>(int kx, int ky, int N, uint32_t r,
                                                            const RowProgram &p) {
    const U32x4 w = philox4x32_10(U32x4{(uint32_t)kx, (uint32_t)ky, r, 0u}, p.seed_lo, p.seed_hi);
    // the uniforms ((x_hi 2^32 + x_lo) >> 11) + 1/2) 2^-53 of the FP64 path,
    // formed in FP32 as (x_hi + x_lo 2^-32) 2^-32 + 2^-54: within an ulp of
    // the FP64 value rounded to FP32, and never zero (the smallest is 2^-54)
    const float u1 = fmaf((float)w.x1, 0x1.0p-64f, fmaf((float)w.x0, 0x1.0p-32f, 0x1.0p-54f));
    const float u2 = fmaf((float)w.x3, 0x1.0p-64f, fmaf((float)w.x2, 0x1.0p-32f, 0x1.0p-54f));
    // hardware transcendentals, their arguments in range by construction:
    // -2 ln u1 = -2 ln 2 log2 u1 (u1 >= 2^-54, a normal float); the angle
    // 2 pi (u2 - rint(u2)) as the turns the hardware sine and cosine take
    const float rad = sqrtf(-1.38629436111989061f * __builtin_amdgcn_logf(u1));
    const float turn = u2 - rintf(u2);
    const float sn = __builtin_amdgcn_sinf(turn), cs = __builtin_amdgcn_cosf(turn);
    const int fx = kx < N / 2 ? kx : kx - N;
    const int fy = ky < N / 2 ? ky : ky - N;
    const uint32_t k2 = (uint32_t)(fx * fx) + (uint32_t)(fy * fy);
    // DC, and the lowest modes when the screen pass adds them in FP64
    const int K = p.low_k;
    if (k2 == 0u || (abs(fx) <= K && abs(fy) <= K)) return {0.0f, 0.0f};
    // amp = amp0 k2^(-beta/4): log2 of the mantissa in FP32, the product with
    // -beta/4 in FP64, exp2 of the fractional part in FP32.
    int ex;
    const float mant = frexpf((float)k2, &ex);  // in [1/2, 1)
    const double y = p.neg_beta_4 * ((double)ex + (double)__builtin_amdgcn_logf(mant));
    const double n = floor(y);
    const float amp =
        ldexpf((float)p.amp0 * __builtin_amdgcn_exp2f((float)(y - n)), (int)n) * 0.70710678118654752f;
    return {amp * rad * cs, amp * rad * sn};
}

template <>
__device__ __forceinline__ cpx<double> spectrum_coeff<double>(int kx, int ky, int N, uint32_t r,
                                                              const RowProgram &p) {
    const double2 c = spectrum_coeff_f64(kx, ky, N, r, p.seed_lo, p.seed_hi, p.amp0, p.neg_beta_4);
    return {c.x, c.y};
}

template <typename Real> __device__ __forceinline__ Real sqrt2_of() { return (Real)1.41421356237309504880; }

// ---------------------------------------------------------------- kernel
// A row program's op codes are a compile-time list (so each program is
// straight-line code with exact register liveness); its operands (pointers,
// strides, scales) come at run time in the RowProgram, op[i] matching code i.
template <int... C> struct OpList {
    static constexpr int code[] = {C...};
    static constexpr int n = sizeof...(C);
};

template <class Ops> constexpr int find_endloop(int i) {
    for (int j = i; j < Ops::n; ++j)
        if (Ops::code[j] == ROP_ENDLOOP) return j;
    return Ops::n;
}

// two-lane vector of Real, the unit of the streaming complex loads and stores
template <typename Real> using Real2 = Real __attribute__((ext_vector_type(2)));

template <typename Real, int L, int V> struct RowState {
    static constexpr int E = Plan<L, V>::E;
    cpx<Real> v[E];
    Real acc[E];
    Real keep[E];
    cpx<Real> keepc[E];
    const RowProgram *prog;
    cpx<Real> *lds;
    const cpx<Real> *tw;
    const cpx<Real> *twc;  // twiddle cache in LDS (or NULL)
    double *red;
    int t, tid, g, batch, row, it, it0, it1;  // it0, it1: this workgroup's range of loop iterations
    bool valid;
};

// FP32 screens, second pass (rows y, after the inverse DFT along x): the
// screen is sqrt(2) Re v (the high modes, from the FP32 transforms) plus the
// lowest modes synthesised in FP64,
//   phi_low(x, y) = Re sum_{k=0}^{K} G_y[k] exp(2 pi i k x / N),
// G_y (one row of RowProgram::low_tab, K + 1 complex doubles) folding the
// negative kx' onto the positive ones.  The thread's elements are
// x = t + m T with T/N = 1/E, so exp(2 pi i k x / N) = W^k c_m^k with
// W = exp(2 pi i t / N) and c_m^k = exp(2 pi i m k / E) a compile-time
// constant: the thread forms D[k] = G_y[k] W^k once, and element m is
// P - Q with P = sum_k Re D[k] cos(2 pi m k / E), Q = sum_k Im D[k]
// sin(2 pi m k / E); element E - m is P + Q (same cosines, opposite sines).
// Each sum is split over even and odd k: at E/2 - m the cosines and sines
// take the factors (-1)^k and -(-1)^k, so the same four partial sums give
// elements E/2 - m and E/2 + m too, and a thread sums for m <= E/4 only.
// The result is
// kept as the pair v = (hi, lo), hi = phi rounded to FP32 and lo the FP32
// remainder, so that the stored screen is phi correctly rounded and the phase
// factor can take phi to FP64 accuracy (RF_HILO).
template <int L, int V, int E = Plan<L, V>::E>
__device__ __forceinline__ void add_low_modes(cpx<float> *v, const void *low_tab, int grow, int t) {
    constexpr int K = low_modes_k_of(L);
    static_assert(E % 2 == 0, "elements per thread must be even");
    // the row's coefficients are the same for all its threads: read through
    // the constant address space, so that a workgroup of one row keeps them
    // in scalar registers (the table is written by an earlier launch)
    using ConstRow = const __attribute__((address_space(4))) double *;
    if constexpr (RowCfg<float, L, V>::B == 1) grow = __builtin_amdgcn_readfirstlane(grow);
    const ConstRow Gc = (ConstRow)(static_cast<const double *>(low_tab) + (int64_t)grow * (2 * (K + 1)));
    const double sw = sinpi(2.0 * (double)t / (double)L), cw = cospi(2.0 * (double)t / (double)L);
    double dr[K + 1], di[K + 1];
    double pr = 1.0, pim = 0.0;  // W^k
#pragma unroll
    for (int k = 0; k <= K; ++k) {
        const double gr = Gc[2 * k], gi = Gc[2 * k + 1];
        dr[k] = fma(gr, pr, -gi * pim);
        di[k] = fma(gr, pim, gi * pr);
        const double npr = fma(pr, cw, -pim * sw);
        pim = fma(pr, sw, pim * cw);
        pr = npr;
    }
    constexpr RootTable<E, 1> C{};  // cos, sin of 2 pi e / E
    constexpr double kSqrt2 = 1.41421356237309504880;
    // phi at element j from the sums of its P and Q: P - Q, and P + Q at E - j
    auto put = [&](int j, double P, double Q) {
        const double phi = fma(kSqrt2, (double)v[j].re, P - Q);
        const float hi = (float)phi;
        v[j] = {hi, (float)(phi - (double)hi)};
        if (j != 0 && j != E / 2) {
            const double phi2 = fma(kSqrt2, (double)v[E - j].re, P + Q);
            const float hi2 = (float)phi2;
            v[E - j] = {hi2, (float)(phi2 - (double)hi2)};
        }
    };
#pragma unroll
    for (int m = 0; m <= E / 4; ++m) {
        double Pk[2] = {0.0, 0.0}, Qk[2] = {0.0, 0.0};  // over even and odd k
#pragma unroll
        for (int k = 0; k <= K; ++k) {
            // exact 0 and +-1 factors as adds (IEEE forbids folding x * 0)
            double &P = Pk[k & 1], &Q = Qk[k & 1];
            const int e = (m * k) % E;
            if (e == 0) {
                P += dr[k];
            } else if (2 * e == E) {
                P -= dr[k];
            } else if (4 * e == E) {
                Q += di[k];
            } else if (4 * e == 3 * E) {
                Q -= di[k];
            } else {
                P = fma(dr[k], C.c[e], P);
                Q = fma(di[k], C.s[e], Q);
            }
        }
        put(m, Pk[0] + Pk[1], Qk[0] + Qk[1]);
        if (E / 2 - m != m) put(E / 2 - m, Pk[0] - Pk[1], Qk[1] - Qk[0]);
    }
}

template <typename Real, int L, int V, int CODE>
__device__ __forceinline__ void exec_op(RowState<Real, L, V> &st, const RowOp &op) {
    constexpr int E = Plan<L, V>::E, T = Plan<L, V>::T;
    auto &v = st.v;
    // Rows past the end of the batch (st.valid false) are given batch 0,
    // row 0, so their loads stay inside the operands and need no predicate
    // (a per-element guard serialises the loads); only stores are guarded.
    const bool valid = st.valid;
    const int64_t off = (int64_t)st.batch * op.batch_stride + (int64_t)st.it * op.iter_stride +
                        (int64_t)st.row * op.row_stride + st.t;
    const double s = (op.flags & RF_ITER_SCALE) ? st.prog->scale[st.it] : op.param;
    if constexpr (CODE == ROP_LOAD_C) {
        // complex rows are read once per pass: streaming (nontemporal) loads
        const cpx<Real> *src = static_cast<const cpx<Real> *>(op.ptr) + off;
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const Real2<Real> x = __builtin_nontemporal_load(reinterpret_cast<const Real2<Real> *>(src + m * T));
            v[m] = {x.x, x.y};
        }
    } else if constexpr (CODE == ROP_LOAD_R) {
        const Real *src = static_cast<const Real *>(op.ptr) + off;
        if (op.flags & RF_PAIR) {  // two real rows as one complex row
            const Real *src2 = static_cast<const Real *>(op.ptr2) + off;
#pragma unroll
            for (int m = 0; m < E; ++m) v[m] = {src[m * T], src2[m * T]};
        } else {
#pragma unroll
            for (int m = 0; m < E; ++m) v[m] = {src[m * T], (Real)0};
        }
    } else if constexpr (CODE == ROP_LOAD_PHASE) {
        const Real *src = static_cast<const Real *>(op.ptr) + off;
        const double sturn = s * (0.5 / kPi);
#pragma unroll
        for (int m = 0; m < E; ++m) v[m] = expi_turns<Real>(sturn * (double)src[m * T]);
    } else if constexpr (CODE == ROP_NOISE) {
        const uint32_t r = (uint32_t)st.prog->r0 + (uint32_t)st.batch;
#pragma unroll
        for (int m = 0; m < E; ++m) v[m] = spectrum_coeff<Real>(st.row, st.t + m * T, L, r, *st.prog);
    } else if constexpr (CODE == ROP_NOISE_SWAP) {
        const uint32_t r = (uint32_t)st.prog->r0 + (uint32_t)st.batch;
#pragma unroll
        for (int m = 0; m < E; ++m) v[m] = spectrum_coeff<Real>(st.t + m * T, st.row, L, r, *st.prog);
    } else if constexpr (CODE == ROP_KEEP_R) {
        const Real *src = static_cast<const Real *>(op.ptr) + off;
#pragma unroll
        for (int m = 0; m < E; ++m) st.keep[m] = src[m * T];
    } else if constexpr (CODE == ROP_EXP_KEEP) {
        const double sturn = s * (0.5 / kPi);
#pragma unroll
        for (int m = 0; m < E; ++m) v[m] = expi_turns<Real>(sturn * (double)st.keep[m]);
    } else if constexpr (CODE == ROP_FFT_FWD) {
        fft_forward<Real, L, V>(v, st.lds, st.t, st.tw, st.twc);
    } else if constexpr (CODE == ROP_FFT_INV) {
        // IDFT(v) = conj(DFT(conj(v)))
#pragma unroll
        for (int m = 0; m < E; ++m) v[m].im = -v[m].im;
        fft_forward<Real, L, V>(v, st.lds, st.t, st.tw, st.twc);
#pragma unroll
        for (int m = 0; m < E; ++m) v[m].im = -v[m].im;
    } else if constexpr (CODE == ROP_MUL_TAB) {
        const cpx<Real> *tab = static_cast<const cpx<Real> *>(op.ptr) + off;
        if (op.flags & RF_CONJ) {
#pragma unroll
            for (int m = 0; m < E; ++m) v[m] = cmulc(v[m], tab[m * T]);
        } else {
#pragma unroll
            for (int m = 0; m < E; ++m) v[m] = cmul(v[m], tab[m * T]);
        }
    } else if constexpr (CODE == ROP_MUL_RTAB2D) {
        // element e = t + m T lies in the lower half for m < E/2 and mirrors
        // to N - e = (E - m) T - t for m >= E/2 (E even)
        static_assert(E % 2 == 0, "elements per thread must be even");
        const int r = st.row <= L / 2 ? st.row : L - st.row;
        const Real *tab = static_cast<const Real *>(op.ptr) + (int64_t)st.it * op.iter_stride +
                          (int64_t)r * op.row_stride;
#pragma unroll
        for (int m = 0; m < E; ++m)
            v[m] = cscale(v[m], m < E / 2 ? tab[st.t + m * T] : tab[(E - m) * T - st.t]);
    } else if constexpr (CODE == ROP_MUL_RLOAD) {
        const Real *src = static_cast<const Real *>(op.ptr) + off;
        const Real sc = (Real)op.param;
#pragma unroll
        for (int m = 0; m < E; ++m) v[m] = cscale(v[m], sc * src[m * T]);
    } else if constexpr (CODE == ROP_SQRT2RE) {
        // FP32 screens always take their lowest modes from the FP64 table
        // (the host builds it for every FP32 screen pass)
        if constexpr (std::is_same<Real, float>::value) {
            add_low_modes<L, V>(v, st.prog->low_tab, st.batch * L + st.row, st.t);  // < 2^30 rows
        } else {
#pragma unroll
            for (int m = 0; m < E; ++m) v[m] = {sqrt2_of<Real>() * v[m].re, (Real)0};
        }
    } else if constexpr (CODE == ROP_EXP_RE) {
        // FP32: the phase is the (hi, lo) pair of ROP_SQRT2RE, summed in FP64
        const double sturn = s * (0.5 / kPi);
        if constexpr (std::is_same<Real, float>::value) {
#pragma unroll
            for (int m = 0; m < E; ++m) v[m] = expi_turns<Real>(sturn * ((double)v[m].re + (double)v[m].im));
        } else {
#pragma unroll
            for (int m = 0; m < E; ++m) v[m] = expi_turns<Real>(sturn * (double)v[m].re);
        }
    } else if constexpr (CODE == ROP_MUL_ROWTAB) {
        const cpx<Real> a = static_cast<const cpx<Real> *>(op.ptr)[(int64_t)st.it * op.iter_stride + st.row];
#pragma unroll
        for (int m = 0; m < E; ++m) v[m] = cmul(v[m], a);
    } else if constexpr (CODE == ROP_STORE_C) {
        if (valid && op.ptr != nullptr) {
            // written once, read by a later pass: streaming (nontemporal) stores
            cpx<Real> *dst = static_cast<cpx<Real> *>(const_cast<void *>(op.ptr)) + off;
#pragma unroll
            for (int m = 0; m < E; ++m) {
                Real2<Real> x;
                x.x = v[m].re;
                x.y = v[m].im;
                __builtin_nontemporal_store(x, reinterpret_cast<Real2<Real> *>(dst + m * T));
            }
        }
    } else if constexpr (CODE == ROP_STORE_R) {
        if (valid && op.ptr != nullptr) {
            Real *dst = static_cast<Real *>(const_cast<void *>(op.ptr)) + off;
            const Real sc = (Real)op.param;
#pragma unroll
            for (int m = 0; m < E; ++m) dst[m * T] = sc * v[m].re;
            if (op.flags & RF_PAIR) {  // the imaginary part to the second row
                Real *dst2 = static_cast<Real *>(op.ptr2) + off;
#pragma unroll
                for (int m = 0; m < E; ++m) dst2[m * T] = sc * v[m].im;
            }
        }
    } else if constexpr (CODE == ROP_ACC_ABS2) {
        const Real w = (Real)((op.flags & RF_ITER_WEIGHT) ? st.prog->weight[st.it] : op.param);
#pragma unroll
        for (int m = 0; m < E; ++m) st.acc[m] += w * (v[m].re * v[m].re + v[m].im * v[m].im);
    } else if constexpr (CODE == ROP_ACC_ABS2U) {
#pragma unroll
        for (int m = 0; m < E; ++m) st.acc[m] = fma(v[m].im, v[m].im, fma(v[m].re, v[m].re, st.acc[m]));
    } else if constexpr (CODE == ROP_STORE_ACC) {
        if (valid) {
            Real *dst = static_cast<Real *>(const_cast<void *>(op.ptr)) + off;
            if (op.flags & RF_ADD) {
#pragma unroll
                for (int m = 0; m < E; ++m) dst[m * T] += st.acc[m];
            } else {
#pragma unroll
                for (int m = 0; m < E; ++m) dst[m * T] = st.acc[m];
            }
        }
    } else if constexpr (CODE == ROP_SAVE) {
#pragma unroll
        for (int m = 0; m < E; ++m) st.keepc[m] = v[m];
    } else if constexpr (CODE == ROP_RESTORE) {
#pragma unroll
        for (int m = 0; m < E; ++m) v[m] = st.keepc[m];
    } else if constexpr (CODE == ROP_GRAD_PHI) {
        const Real *src = static_cast<const Real *>(op.ptr) + off;
        const double sturn = s * (0.5 / kPi);
        const Real sc = (Real)s;
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const cpx<Real> u = expi_turns<Real>(sturn * (double)src[m * T]);
            v[m] = {sc * (v[m].im * u.re - v[m].re * u.im), (Real)0};  // s Im(v conj(u))
        }
    } else if constexpr (CODE == ROP_DOT_R) {
        // per-row sum of src[e] Re v[e] in FP64 in a fixed order: registers,
        // then a tree over the row's threads through LDS
        const Real *src = static_cast<const Real *>(op.ptr) + off;
        double part = 0.0;
#pragma unroll
        for (int m = 0; m < E; ++m) part += (double)src[m * T] * (double)v[m].re;
        double *red = st.red;
        __syncthreads();
        red[st.tid] = part;
        __syncthreads();
        for (int width = 1; width < T; width *= 2) {
            if ((st.t % (2 * width)) == 0 && st.t + width < T) red[st.tid] += red[st.tid + width];
            __syncthreads();
        }
        if (st.t == 0 && valid) static_cast<double *>(op.ptr2)[st.g] = red[st.tid];
        __syncthreads();
    } else if constexpr (CODE == ROP_SIDE_T) {
        // the side transposes run in workgroups of their own (row_kernel)
    } else {
        static_assert(CODE == ROP_END, "unknown row op");
    }
}

template <typename Real, int L, int V, class Ops, int I, int End>
__device__ __forceinline__ void run_ops(RowState<Real, L, V> &st) {
    if constexpr (I < End) {
        constexpr int c = Ops::code[I];
        if constexpr (c == ROP_LOOP) {
            constexpr int e = find_endloop<Ops>(I);
#pragma clang loop unroll(disable)
            for (st.it = st.it0; st.it < st.it1; ++st.it) {
                // (RowCfg::REMAT_T: addresses formed again per iteration)
                if constexpr (RowCfg<Real, L, V>::REMAT_T) asm volatile("" : "+v"(st.t));
                run_ops<Real, L, V, Ops, I + 1, e>(st);
            }
            st.it = 0;
            run_ops<Real, L, V, Ops, e + 1, End>(st);
        } else {
            exec_op<Real, L, V, c>(st, st.prog->op[I]);
            run_ops<Real, L, V, Ops, I + 1, End>(st);
        }
    }
}

template <class Ops> constexpr bool has_side() { return Ops::n > 0 && Ops::code[0] == ROP_SIDE_T; }

// Whether a program's loop iterations may be split between two workgroups
// (RowProgram::iter_split): one loop, nothing after it, and inside it only
// per-iteration loads, transforms, table products and stores.
template <class Ops> constexpr bool iter_splittable() {
    int i = has_side<Ops>() ? 1 : 0;
    if (i >= Ops::n || Ops::code[i] != ROP_LOOP) return false;
    for (++i; i < Ops::n && Ops::code[i] != ROP_ENDLOOP; ++i) {
        const int c = Ops::code[i];
        if (c != ROP_LOAD_PHASE && c != ROP_LOAD_C && c != ROP_FFT_FWD && c != ROP_FFT_INV && c != ROP_MUL_TAB &&
            c != ROP_STORE_C)
            return false;
    }
    return i == Ops::n - 1;
}

// LDS of a row kernel: the row pass's, or the transpose tile's if larger
// (programs with side transposes)
template <typename Real, int L, int V, class Ops> constexpr int row_kernel_lds() {
    constexpr int a = RowCfg<Real, L, V>::LDS_BYTES, b = (int)sizeof(TransposeTile<cpx<float>>);
    return has_side<Ops>() && a < b ? b : a;
}

// The side transposes of one transpose workgroup (number sb of the launch):
// its units_per_block consecutive units of [u0, u1), one after the other.
// Their data is touched once, so it is streamed with nontemporal accesses
// and leaves the cached tables and phase rows of the row workgroups alone.
template <int NT>
__device__ __forceinline__ void side_transposes(const RowSide &sd, int N, int sb, unsigned char *lds, int tid) {
    const int nx = transpose_units_x(N), ny = transpose_units_y(N);
    const int64_t per = (int64_t)nx * ny, nn = (int64_t)N * N;
    int64_t u = sd.u0 + (int64_t)sb * sd.units_per_block;
    const int64_t end = min(u + (int64_t)sd.units_per_block, sd.u1);
    auto &tile = *reinterpret_cast<TransposeTile<cpx<float>> *>(lds);
    const cpx<float> *in = static_cast<const cpx<float> *>(sd.in);
    cpx<float> *out = static_cast<cpx<float> *>(sd.out);
    for (; u < end; ++u) {
        const int64_t z = u / per;
        const int rem = (int)(u - z * per);
        const int uy = rem / nx, ux = rem - uy * nx;
        transpose_unit<cpx<float>, NT, true>(in + z * nn, out + z * nn, N, ux, uy, tile, tid);
        __syncthreads();  // the tile is reused by the next unit
    }
}

template <typename Real, int L, int V, class Ops>
__global__ __launch_bounds__((RowCfg<Real, L, V>::THREADS))
__attribute__((amdgpu_waves_per_eu(RowCfg<Real, L, V>::WAVES_PER_EU))) void row_kernel(const RowProgram prog,
                                                                           const cpx<Real> *__restrict__ tw) {
    using Cfg = RowCfg<Real, L, V>;
    constexpr int E = Plan<L, V>::E, T = Plan<L, V>::T, B = Cfg::B;
    __shared__ __align__(16) unsigned char lds_raw[row_kernel_lds<Real, L, V, Ops>()];
    int rb = blockIdx.x;  // row workgroup number
    if constexpr (has_side<Ops>()) {
        // groups of fft_blocks row workgroups followed by side_blocks
        // transpose workgroups (uniform per workgroup, so the early returns
        // come before any barrier)
        static_assert(std::is_same<Real, float>::value, "side transposes are complex64 only");
        const RowSide &sd = prog.side;
        const int G = sd.fft_blocks + sd.side_blocks;
        const int grp = blockIdx.x / G, r = blockIdx.x - grp * G;
        if (r >= sd.fft_blocks) {
            side_transposes<Cfg::THREADS>(sd, prog.N, grp * sd.side_blocks + (r - sd.fft_blocks), lds_raw,
                                          threadIdx.x);
            return;
        }
        rb = grp * sd.fft_blocks + r;
    }
    int it0 = 0, it1 = prog.n_iter;
    if constexpr (iter_splittable<Ops>()) {
        if (prog.iter_split == 2) {
            // row workgroups q and q + 8 of each 16 share row workgroup
            // 8 (q / 16) + q % 8
            const int half = (rb >> 3) & 1;
            rb = ((rb >> 4) << 3) | (rb & 7);
            const int h = (prog.n_iter + 1) / 2;
            it0 = half ? h : 0;
            it1 = half ? prog.n_iter : h;
        }
    }
    if constexpr (has_side<Ops>()) {
        if ((int64_t)rb * B >= prog.total_rows) return;
    }
    RowState<Real, L, V> st;
    st.prog = &prog;
    st.tid = threadIdx.x;
    const int bsub = st.tid / T;
    st.t = st.tid - bsub * T;
    st.g = rb * B + bsub;  // global row over the batch
    st.valid = st.g < prog.total_rows;
    st.batch = st.valid ? st.g / L : 0;
    st.row = st.valid ? st.g - st.batch * L : 0;
    st.lds = reinterpret_cast<cpx<Real> *>(lds_raw) + bsub * Cfg::LDS_STRIDE;
    st.red = reinterpret_cast<double *>(lds_raw);
    st.tw = tw;
    st.twc = nullptr;
    if constexpr (Cfg::TWC_ON) {
        cpx<Real> *twc = reinterpret_cast<cpx<Real> *>(lds_raw + Cfg::FFT_LDS_BYTES);
        fill_tw_cache<Real, L, V>(twc, tw, st.tid, Cfg::THREADS);
        __syncthreads();
        st.twc = twc;
    }
    st.it = 0;
    st.it0 = it0;
    st.it1 = it1;
#pragma unroll
    for (int m = 0; m < E; ++m) {
        st.v[m] = {(Real)0, (Real)0};
        st.acc[m] = (Real)0;
    }
    run_ops<Real, L, V, Ops, 0, Ops::n>(st);
}

// The row programs used by the library.  Each name lists its op codes; the
// host fills the operands of op[i] for code i.
using ProgNoise = OpList<ROP_NOISE, ROP_FFT_INV, ROP_STORE_C>;
// the noise pass carrying the transpose of an earlier batch's output (RowSide)
using ProgNoiseT = OpList<ROP_SIDE_T, ROP_NOISE, ROP_FFT_INV, ROP_STORE_C>;
// the same along kx (rows ky), for screens made transposed
using ProgNoiseSwap = OpList<ROP_NOISE_SWAP, ROP_FFT_INV, ROP_STORE_C>;
using ProgNoiseSwapT = OpList<ROP_SIDE_T, ROP_NOISE_SWAP, ROP_FFT_INV, ROP_STORE_C>;
using ProgScreen = OpList<ROP_LOAD_C, ROP_FFT_INV, ROP_SQRT2RE, ROP_STORE_R>;
using ProgScreenProp = OpList<ROP_LOAD_C, ROP_FFT_INV, ROP_SQRT2RE, ROP_STORE_R, ROP_EXP_RE, ROP_FFT_FWD,
                              ROP_MUL_TAB, ROP_FFT_INV, ROP_STORE_C>;
// (the phase is re-read for every wavelength: keeping it in registers
// costs more in occupancy than the cached re-read)
using ProgPhaseProp = OpList<ROP_LOOP, ROP_LOAD_PHASE, ROP_FFT_FWD, ROP_MUL_TAB, ROP_FFT_INV, ROP_STORE_C,
                             ROP_ENDLOOP>;
// (the weights of a co-addition ride in the chirp tables, so the sum of
// |.|^2 takes no product by them)
using ProgPropIntensity = OpList<ROP_LOOP, ROP_LOAD_C, ROP_FFT_FWD, ROP_MUL_TAB, ROP_FFT_INV, ROP_ACC_ABS2U,
                                 ROP_ENDLOOP, ROP_STORE_ACC>;
// the two propagation passes carrying transposes of other data (RowSide)
using ProgPhasePropT = OpList<ROP_SIDE_T, ROP_LOOP, ROP_LOAD_PHASE, ROP_FFT_FWD, ROP_MUL_TAB, ROP_FFT_INV,
                              ROP_STORE_C, ROP_ENDLOOP>;
using ProgPropIntensityT = OpList<ROP_SIDE_T, ROP_LOOP, ROP_LOAD_C, ROP_FFT_FWD, ROP_MUL_TAB, ROP_FFT_INV,
                                  ROP_ACC_ABS2U, ROP_ENDLOOP, ROP_STORE_ACC>;
using ProgRealFwd = OpList<ROP_LOAD_R, ROP_FFT_FWD, ROP_STORE_C>;
using ProgFwdRe = OpList<ROP_LOAD_C, ROP_FFT_FWD, ROP_STORE_R>;
using ProgSmearMid = OpList<ROP_LOAD_C, ROP_FFT_FWD, ROP_SAVE, ROP_LOOP, ROP_RESTORE, ROP_MUL_RTAB2D,
                            ROP_FFT_INV, ROP_STORE_C, ROP_ENDLOOP>;
using ProgInvRe = OpList<ROP_LOAD_C, ROP_FFT_INV, ROP_STORE_R>;
// the three smear passes carrying transposes of other data (RowSide)
using ProgRealFwdT = OpList<ROP_SIDE_T, ROP_LOAD_R, ROP_FFT_FWD, ROP_STORE_C>;
using ProgSmearMidT = OpList<ROP_SIDE_T, ROP_LOAD_C, ROP_FFT_FWD, ROP_SAVE, ROP_LOOP, ROP_RESTORE, ROP_MUL_RTAB2D,
                             ROP_FFT_INV, ROP_STORE_C, ROP_ENDLOOP>;
using ProgInvReT = OpList<ROP_SIDE_T, ROP_LOAD_C, ROP_FFT_INV, ROP_STORE_R>;
using ProgVjpY = OpList<ROP_LOAD_C, ROP_FFT_FWD, ROP_MUL_TAB, ROP_FFT_INV, ROP_MUL_RLOAD, ROP_FFT_FWD,
                        ROP_MUL_TAB, ROP_FFT_INV, ROP_STORE_C>;
using ProgVjpX = OpList<ROP_LOAD_C, ROP_FFT_FWD, ROP_MUL_TAB, ROP_FFT_INV, ROP_GRAD_PHI, ROP_STORE_R,
                        ROP_DOT_R>;
// the second propagation pass keeping the field A as the adjoint's
// checkpoint beside |A|^2, and the adjoint's first pass starting from it
using ProgPropField = OpList<ROP_LOAD_C, ROP_FFT_FWD, ROP_MUL_TAB, ROP_FFT_INV, ROP_STORE_C, ROP_ACC_ABS2U,
                             ROP_STORE_ACC>;
using ProgVjpYField = OpList<ROP_LOAD_C, ROP_MUL_RLOAD, ROP_FFT_FWD, ROP_MUL_TAB, ROP_FFT_INV, ROP_STORE_C>;
// aperture mode: windowed, chirped exp(i s phi) -> DFT along the row; then
// DFT along the other axis and |.|^2
using ProgApertureX = OpList<ROP_LOAD_PHASE, ROP_MUL_TAB, ROP_MUL_ROWTAB, ROP_FFT_FWD, ROP_STORE_C>;
using ProgAbs2 = OpList<ROP_LOAD_C, ROP_FFT_FWD, ROP_ACC_ABS2, ROP_STORE_ACC>;

}  // namespace scint

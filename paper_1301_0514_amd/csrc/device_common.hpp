// device_common.hpp -- complex arithmetic, compile-time trigonometry, the
// in-register radix butterflies and the Philox4x32-10 counter generator used
// by the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace scint {

template <typename Real> struct alignas(2 * sizeof(Real)) cpx {
    Real re, im;
};

template <typename Real> __device__ __forceinline__ cpx<Real> cadd(cpx<Real> a, cpx<Real> b) {
    return {a.re + b.re, a.im + b.im};
}
template <typename Real> __device__ __forceinline__ cpx<Real> csub(cpx<Real> a, cpx<Real> b) {
    return {a.re - b.re, a.im - b.im};
}
template <typename Real> __device__ __forceinline__ cpx<Real> cmul(cpx<Real> a, cpx<Real> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// a * conj(b)
template <typename Real> __device__ __forceinline__ cpx<Real> cmulc(cpx<Real> a, cpx<Real> b) {
    return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}
template <typename Real> __device__ __forceinline__ cpx<Real> cscale(cpx<Real> a, Real s) {
    return {a.re * s, a.im * s};
}
// multiply by S*i (S = +1 or -1)
template <int S, typename Real> __device__ __forceinline__ cpx<Real> mul_si(cpx<Real> a) {
    if constexpr (S > 0) return {-a.im, a.re};
    else return {a.im, -a.re};
}

// ---------------------------------------------------------------------------
// Compile-time cos/sin of 2 pi n / d.  Exact rational octant reduction to an
// angle of at most pi/4, then Taylor series in double (error below 1 ulp).
// ---------------------------------------------------------------------------
constexpr double kPi = 3.141592653589793238462643383279502884;

constexpr double taylor_sin(double x) {
    double term = x, sum = x, x2 = x * x;
    for (int k = 1; k < 14; ++k) {
        term *= -x2 / ((2.0 * k) * (2.0 * k + 1.0));
        sum += term;
    }
    return sum;
}
constexpr double taylor_cos(double x) {
    double term = 1.0, sum = 1.0, x2 = x * x;
    for (int k = 1; k < 14; ++k) {
        term *= -x2 / ((2.0 * k - 1.0) * (2.0 * k));
        sum += term;
    }
    return sum;
}

struct SinCos {
    double c, s;
};

// cos and sin of 2 pi n/d for integers (any sign of n), d > 0.
constexpr SinCos sincos2pi(long long n, long long d) {
    long long m = n % d;
    if (m < 0) m += d;
    // angle = 2 pi m/d, m/d in [0,1)
    double sign_s = 1.0;
    long long num = m, den = d;
    if (2 * num > den) {  // r > 1/2: r -> 1 - r, sin flips
        num = den - num;
        sign_s = -1.0;
    }
    // now r = num/den in [0, 1/2]
    double sign_c = 1.0;
    if (4 * num > den) {  // r > 1/4: r -> 1/2 - r, cos flips
        num = den - 2 * num;
        den = 2 * den;
        sign_c = -1.0;
    }
    // r in [0, 1/4]
    bool swap = false;
    if (8 * num > den) {  // r > 1/8: r -> 1/4 - r, swap sin and cos
        num = den - 4 * num;
        den = 4 * den;
        swap = true;
    }
    double x = 2.0 * kPi * (double)num / (double)den;
    double c = taylor_cos(x), s = taylor_sin(x);
    if (swap) {
        double t = c;
        c = s;
        s = t;
    }
    return SinCos{sign_c * c, sign_s * s};
}

// Table of W_R^{e} = exp(S 2 pi i e / R), e in [0, R), built at compile time.
template <int R, int S> struct RootTable {
    double c[R], s[R];
    constexpr RootTable() : c(), s() {
        for (int e = 0; e < R; ++e) {
            SinCos v = sincos2pi((long long)S * e, R);
            c[e] = v.c;
            s[e] = v.s;
        }
    }
};

// ---------------------------------------------------------------------------
// In-register DFT of size R:  a[k] <- sum_n a[n] exp(S 2 pi i n k / R).
// Base radices 2, 4, 5.  An even R >= 8 is split R = (R/2) x 2 by decimation
// in time: two half-size DFTs of the even and odd elements, then R/2 radix-2
// butterflies whose compile-time twiddle multiplies one input, which a
// butterfly takes in six fused multiply-adds (below) instead of a complex
// product and four additions.
// ---------------------------------------------------------------------------
#ifndef SCINT_DFT_DIT2
#define SCINT_DFT_DIT2 1
#endif
template <int R> constexpr int split_factor() {
    if constexpr (SCINT_DFT_DIT2 && R % 2 == 0 && R >= 8) return R / 2;
    else if constexpr (R == 32) return 4;
    else if constexpr (R % 4 == 0 && R != 8) return 4;
    else if constexpr (R % 2 == 0) return 2;
    else return 5;
}

template <typename Real> __device__ __forceinline__ Real fmar(Real a, Real b, Real c) {
    if constexpr (sizeof(Real) == 4) return __builtin_fmaf(a, b, c);
    else return __builtin_fma(a, b, c);
}

// (a, b) <- (a + w b, a - w b) for a constant w = c + i s (Linzer & Feig):
// w b = c (b + i (s/c) b) when |c| >= |s|, else s ((c/s) b + i b), so that
// the scaled product takes two fused multiply-adds and each output two more,
// with the ratio at most 1 in magnitude.
template <typename Real> __device__ __forceinline__ void bfly_const(cpx<Real> &a, cpx<Real> &b, double c, double s) {
    Real vr, vi, g;
    if (c * c >= s * s) {
        const Real t = (Real)(s / c);
        g = (Real)c;
        vr = fmar(-t, b.im, b.re);
        vi = fmar(t, b.re, b.im);
    } else {
        const Real u = (Real)(c / s);
        g = (Real)s;
        vr = fmar(u, b.re, -b.im);
        vi = fmar(u, b.im, b.re);
    }
    const cpx<Real> x0 = {fmar(g, vr, a.re), fmar(g, vi, a.im)};
    const cpx<Real> x1 = {fmar(-g, vr, a.re), fmar(-g, vi, a.im)};
    a = x0;
    b = x1;
}

template <int R, int S, typename Real> struct Dft;

template <int S, typename Real> struct Dft<1, S, Real> {
    static __device__ __forceinline__ void run(cpx<Real>*) {}
};

template <int S, typename Real> struct Dft<2, S, Real> {
    static __device__ __forceinline__ void run(cpx<Real>* a) {
        cpx<Real> t = a[0];
        a[0] = cadd(t, a[1]);
        a[1] = csub(t, a[1]);
    }
};

template <int S, typename Real> struct Dft<4, S, Real> {
    static __device__ __forceinline__ void run(cpx<Real>* a) {
        cpx<Real> s02 = cadd(a[0], a[2]), d02 = csub(a[0], a[2]);
        cpx<Real> s13 = cadd(a[1], a[3]), d13 = mul_si<S>(csub(a[1], a[3]));
        a[0] = cadd(s02, s13);
        a[2] = csub(s02, s13);
        a[1] = cadd(d02, d13);
        a[3] = csub(d02, d13);
    }
};

template <int S, typename Real> struct Dft<5, S, Real> {
    static __device__ __forceinline__ void run(cpx<Real>* a) {
        constexpr SinCos w1 = sincos2pi(1, 5), w2 = sincos2pi(2, 5);
        const Real c1 = (Real)w1.c, c2 = (Real)w2.c;
        const Real s1 = (Real)(S * w1.s), s2 = (Real)(S * w2.s);
        cpx<Real> b1 = cadd(a[1], a[4]), b4 = csub(a[1], a[4]);
        cpx<Real> b2 = cadd(a[2], a[3]), b3 = csub(a[2], a[3]);
        cpx<Real> x0 = a[0];
        a[0] = cadd(x0, cadd(b1, b2));
        // real-coefficient parts
        cpx<Real> p1 = {x0.re + c1 * b1.re + c2 * b2.re, x0.im + c1 * b1.im + c2 * b2.im};
        cpx<Real> p2 = {x0.re + c2 * b1.re + c1 * b2.re, x0.im + c2 * b1.im + c1 * b2.im};
        // i * (s1 b4 + s2 b3) and i * (s2 b4 - s1 b3)
        Real q1re = s1 * b4.re + s2 * b3.re, q1im = s1 * b4.im + s2 * b3.im;
        Real q2re = s2 * b4.re - s1 * b3.re, q2im = s2 * b4.im - s1 * b3.im;
        a[1] = {p1.re - q1im, p1.im + q1re};
        a[4] = {p1.re + q1im, p1.im - q1re};
        a[2] = {p2.re - q2im, p2.im + q2re};
        a[3] = {p2.re + q2im, p2.im - q2re};
    }
};

template <int R, int S, typename Real> struct Dft {
    static constexpr int R1 = split_factor<R>();
    static constexpr int R2 = R / R1;
    static __device__ __forceinline__ void run(cpx<Real>* a) {
        constexpr RootTable<R, S> W{};
        if constexpr (R2 == 2) {
            // decimation in time: X[k] = E[k] + W^k O[k], X[k + R/2] = E[k] - W^k O[k]
            cpx<Real> e[R1], o[R1];
#pragma unroll
            for (int n = 0; n < R1; ++n) {
                e[n] = a[2 * n];
                o[n] = a[2 * n + 1];
            }
            Dft<R1, S, Real>::run(e);
            Dft<R1, S, Real>::run(o);
#pragma unroll
            for (int k = 0; k < R1; ++k) {
                if (k == 0) {
                    a[k] = cadd(e[k], o[k]);
                    a[k + R1] = csub(e[k], o[k]);
                } else if (4 * k == R) {
                    const cpx<Real> t = mul_si<S>(o[k]);
                    a[k] = cadd(e[k], t);
                    a[k + R1] = csub(e[k], t);
                } else {
                    bfly_const(e[k], o[k], W.c[k], W.s[k]);
                    a[k] = e[k];
                    a[k + R1] = o[k];
                }
            }
            return;
        }
        cpx<Real> y[R];
#pragma unroll
        for (int n2 = 0; n2 < R2; ++n2) {
            cpx<Real> b[R1];
#pragma unroll
            for (int n1 = 0; n1 < R1; ++n1) b[n1] = a[R2 * n1 + n2];
            Dft<R1, S, Real>::run(b);
#pragma unroll
            for (int k1 = 0; k1 < R1; ++k1) {
                // W^e is 1, S i, -1 or -S i for e = 0, R/4, R/2, 3R/4: a swap
                // and sign changes (a multiply by an exact 0 or 1 is not
                // folded away under IEEE rules); other e a complex multiply
                const int e = (n2 * k1) % R;
                if (e == 0) {
                    y[n2 * R1 + k1] = b[k1];
                } else if (4 * e == R) {
                    y[n2 * R1 + k1] = mul_si<S>(b[k1]);
                } else if (2 * e == R) {
                    y[n2 * R1 + k1] = {-b[k1].re, -b[k1].im};
                } else if (4 * e == 3 * R) {
                    y[n2 * R1 + k1] = mul_si<-S>(b[k1]);
                } else {
                    cpx<Real> w = {(Real)W.c[e], (Real)W.s[e]};
                    y[n2 * R1 + k1] = cmul(b[k1], w);
                }
            }
        }
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) {
            cpx<Real> c[R2];
#pragma unroll
            for (int n2 = 0; n2 < R2; ++n2) c[n2] = y[n2 * R1 + k1];
            Dft<R2, S, Real>::run(c);
#pragma unroll
            for (int k2 = 0; k2 < R2; ++k2) a[k1 + R1 * k2] = c[k2];
        }
    }
};

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11).
// ---------------------------------------------------------------------------
struct U32x4 {
    uint32_t x0, x1, x2, x3;
};

// a ^ b ^ k with the key k uniform over the wave (held in a scalar
// register): one three-input logic instruction (truth table 0x96, the
// three-way exclusive or), which the compiler does not form from the two
// exclusive ors by itself
__device__ __forceinline__ uint32_t xor3_key(uint32_t a, uint32_t b, uint32_t k) {
#ifndef SCINT_PHILOX_BITOP3
#define SCINT_PHILOX_BITOP3 1
#endif
#if SCINT_PHILOX_BITOP3
    uint32_t r;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "s"(k));
    return r;
#else
    return a ^ b ^ k;
#endif
}

// The keys k0, k1 must be the same for every lane of the wave (they are the
// seed's two halves plus round constants at every call site).
__device__ __forceinline__ U32x4 philox4x32_10(U32x4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        // each 32 x 32 -> 64-bit product as one full-width multiply (one
        // v_mad_u64_u32) rather than separate high and low halves
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x0, p1 = (uint64_t)0xCD9E8D57u * c.x2;
        if (round < 2) {
            // the first rounds still mix words that are uniform in some
            // callers (a row's kx, the realisation), which the compiler folds
            // into scalar instructions
            c = U32x4{(uint32_t)(p1 >> 32) ^ c.x1 ^ k0, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ c.x3 ^ k1, (uint32_t)p0};
        } else {
            c = U32x4{xor3_key((uint32_t)(p1 >> 32), c.x1, k0), (uint32_t)p1,
                      xor3_key((uint32_t)(p0 >> 32), c.x3, k1), (uint32_t)p0};
        }
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// Random phase spectrum coefficient in FP64 at Fourier pixel (kx, ky) (FFT
// indices in [0, N)) of realisation r (Sect. 3.1, Eqs. spectre and
// densite): two 53-bit uniforms from one Philox block, Box-Muller, times
// amp0 |k'|^(-beta/2) / sqrt(2), with amp0 = sqrt(C_beta R^(2-beta))
// N^(beta/2) / N; zero at k = 0.
__device__ __forceinline__ double2 spectrum_coeff_f64(int kx, int ky, int N, uint32_t r, uint32_t seed_lo,
                                                      uint32_t seed_hi, double amp0, double neg_beta_4) {
    const U32x4 w = philox4x32_10(U32x4{(uint32_t)kx, (uint32_t)ky, r, 0u}, seed_lo, seed_hi);
    const uint64_t a = ((uint64_t)w.x0 << 32) | w.x1;
    const uint64_t b = ((uint64_t)w.x2 << 32) | w.x3;
    const double u1 = ((double)(a >> 11) + 0.5) * 0x1.0p-53;
    const double u2 = ((double)(b >> 11) + 0.5) * 0x1.0p-53;
    const double rad = sqrt(-2.0 * log(u1));
    double sn, cs;
    sincospi(2.0 * (u2 - rint(u2)), &sn, &cs);
    const int fx = kx < N / 2 ? kx : kx - N;
    const int fy = ky < N / 2 ? ky : ky - N;
    const double k2 = (double)fx * fx + (double)fy * fy;
    if (k2 == 0.0) return make_double2(0.0, 0.0);
    const double amp = amp0 * pow(k2, neg_beta_4) * 0.70710678118654752440;
    return make_double2(amp * rad * cs, amp * rad * sn);
}


}  // namespace scint

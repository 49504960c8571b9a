// fft_plan.hpp -- compile-time Stockham plans for the 1-D transforms along a
// row of the N x N grid.  Included by the kernels (which unroll the stages)
// and by the host (which builds the per-stage twiddle tables from the same
// description).
//
// A length-L transform is done by T = L/E threads; each thread keeps E
// elements in registers, namely x[t + m T] for m in [0, E).  Stage s has radix
// R_s (R_s divides E, so each thread does E/R_s butterflies of it), and Ns is
// the product of the radices of the earlier stages.  Butterfly j of stage s
// takes x[j + r L/R_s] (r < R_s), multiplies by W_{Ns R_s}^{r (j mod Ns)},
// does an R_s-point DFT and writes to (j - j mod Ns) R_s + j mod Ns + r Ns:
// the self-sorting (Stockham) order, so the result ends in natural order with
// every thread again holding x[t + m T].
#pragma once

namespace scint {

// Plan<L, V>: variant V of the plan for length L.  Variant 0 exists for every
// supported size; the large FP32 sizes have alternatives that the run-time
// tuner times on first use.
template <int L, int V = 0> struct Plan;  // only the sizes below exist

constexpr bool plan_ok(int L, int E, const int *R, int ns) {
    int prod = 1;
    for (int s = 0; s < ns; ++s) {
        if (R[s] < 2 || E % R[s] != 0) return false;
        prod *= R[s];
    }
    return prod == L && L % E == 0 && L / E <= 1024;
}

#define SCINT_PLAN_V(L_, V_, E_, ...)                                           \
    template <> struct Plan<L_, V_> {                                           \
        static constexpr int L = L_;                                            \
        static constexpr int E = E_;                                            \
        static constexpr int R[] = {__VA_ARGS__};                               \
        static constexpr int NS = sizeof(R) / sizeof(int);                      \
        static constexpr int T = L_ / E_;                                       \
        static_assert(plan_ok(L_, E_, R, NS),                                   \
                      "radices must multiply to L and each divide E");          \
    };
#define SCINT_PLAN(L_, E_, ...) SCINT_PLAN_V(L_, 0, E_, __VA_ARGS__)
// expands a size list given through another macro
#define SCINT_PLAN_EXPAND(...) SCINT_PLAN(__VA_ARGS__)

// powers of two
SCINT_PLAN(16, 16, 16)
SCINT_PLAN(32, 8, 8, 4)
SCINT_PLAN(64, 8, 8, 8)
SCINT_PLAN(128, 16, 16, 8)
SCINT_PLAN(256, 16, 16, 16)
SCINT_PLAN(512, 8, 8, 8, 8)
SCINT_PLAN(1024, 16, 16, 16, 4)
SCINT_PLAN(2048, 16, 16, 16, 8)
SCINT_PLAN(4096, 32, 32, 8, 16)
SCINT_PLAN(8192, 32, 32, 8, 32)
SCINT_PLAN(16384, 32, 32, 32, 16)
// 2^a 5^b
SCINT_PLAN(40, 20, 4, 10)
SCINT_PLAN(80, 20, 4, 20)
SCINT_PLAN(100, 10, 10, 10)
SCINT_PLAN(160, 20, 4, 4, 10)
SCINT_PLAN(200, 20, 20, 10)
SCINT_PLAN(320, 20, 4, 4, 20)
SCINT_PLAN(400, 20, 20, 20)
SCINT_PLAN(640, 20, 4, 4, 4, 10)
SCINT_PLAN(1000, 10, 10, 10, 10)
SCINT_PLAN(1280, 20, 4, 4, 4, 20)
SCINT_PLAN(2000, 20, 20, 10, 10)
SCINT_PLAN(2560, 20, 4, 4, 4, 4, 10)
SCINT_PLAN(4000, 20, 20, 20, 10)
SCINT_PLAN(5000, 10, 10, 10, 10, 5)
SCINT_PLAN(8000, 20, 20, 20, 20)
SCINT_PLAN(10000, 10, 10, 10, 10, 10)
// FP32 only: a row of 16000 or 20000 complex64 fills most of the LDS
SCINT_PLAN(16000, 40, 40, 40, 10)
SCINT_PLAN(20000, 40, 40, 10, 10, 5)

// alternatives timed by the tuner (FP32)
SCINT_PLAN_V(2048, 1, 16, 16, 8, 16)
SCINT_PLAN_V(4096, 1, 16, 16, 16, 16)
SCINT_PLAN_V(4096, 2, 32, 32, 16, 8)
SCINT_PLAN_V(8192, 1, 16, 16, 8, 8, 8)
SCINT_PLAN_V(8192, 2, 32, 32, 32, 8)
SCINT_PLAN_V(10000, 1, 20, 20, 20, 5, 5)
SCINT_PLAN_V(16384, 1, 32, 16, 32, 32)
SCINT_PLAN_V(16384, 2, 32, 32, 16, 32)
SCINT_PLAN_V(16000, 1, 20, 20, 20, 20, 2)
SCINT_PLAN_V(20000, 1, 20, 20, 20, 10, 5)

#undef SCINT_PLAN_EXPAND
#undef SCINT_PLAN
#undef SCINT_PLAN_V

// Number of plan variants of length L (FP32; FP64 uses variant 0 only).
constexpr int plan_variants(int L) {
    return (L == 4096 || L == 8192 || L == 16384) ? 3
           : (L == 2048 || L == 10000 || L == 16000 || L == 20000) ? 2
                                                                    : 1;
}

// X(L, V) for every FP32 variant beyond 0
#define SCINT_VARIANTS_F32(X) \
    X(2048, 1) X(4096, 1) X(4096, 2) X(8192, 1) X(8192, 2) X(10000, 1) X(16000, 1) X(16384, 1) X(16384, 2) X(20000, 1)

// Sizes in ascending order, per precision (FP64 stops at 8192 because a
// 10000-point complex128 row does not fit in the 160 KB of LDS; FP32 stops at
// 20000, whose complex64 row nearly fills it).
#define SCINT_SIZES_F64(X)                                                      \
    X(16) X(32) X(40) X(64) X(80) X(100) X(128) X(160) X(200) X(256) X(320)     \
    X(400) X(512) X(640) X(1000) X(1024) X(1280) X(2000) X(2048) X(2560)        \
    X(4000) X(4096) X(5000) X(8000) X(8192)
#define SCINT_SIZES_F32(X) SCINT_SIZES_F64(X) X(10000) X(16000) X(16384) X(20000)

// Number of entries of the per-stage twiddle tables of a plan: stage s >= 1
// holds W_{Ns R}^{r k} for k < Ns and r < R, i.e. Ns R entries.
template <int L, int V = 0> constexpr int twiddle_count() {
    using P = Plan<L, V>;
    int n = 0, ns = 1;
    for (int s = 0; s < P::NS; ++s) {
        if (s > 0) n += ns * P::R[s];
        ns *= P::R[s];
    }
    return n;
}

// Offset of stage s's table inside the concatenated twiddle array.
template <int L, int V = 0> constexpr int twiddle_offset(int stage) {
    using P = Plan<L, V>;
    int n = 0, ns = 1;
    for (int s = 0; s < stage; ++s) {
        if (s > 0) n += ns * P::R[s];
        ns *= P::R[s];
    }
    return n;
}

template <int L, int V = 0> constexpr int stage_ns(int stage) {
    int ns = 1;
    for (int s = 0; s < stage; ++s) ns *= Plan<L, V>::R[s];
    return ns;
}

}  // namespace scint

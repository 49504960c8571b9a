// twiddles.cpp -- host construction of the per-stage twiddle tables of the
// Stockham plans, evaluated in extended precision and rounded once by the
// caller to the working precision.
#include <cmath>
#include <cstddef>

#include "fft_plan.hpp"
#include "row_launch.h"

namespace scint {

// exp(-2 pi i m / M) with exact integer reduction of m modulo M and an octant
// reduction of the angle, in long double.
static void root_ld(long long m, long long M, long double &c, long double &s) {
    m %= M;
    if (m < 0) m += M;
    long long num = m, den = M;
    long double sign_s = 1.0L, sign_c = 1.0L;
    if (2 * num > den) {
        num = den - num;
        sign_s = -1.0L;
    }
    if (4 * num > den) {
        num = den - 2 * num;
        den *= 2;
        sign_c = -1.0L;
    }
    bool swap = false;
    if (8 * num > den) {
        num = den - 4 * num;
        den *= 4;
        swap = true;
    }
    const long double pi = 3.141592653589793238462643383279502884L;
    const long double x = 2.0L * pi * (long double)num / (long double)den;
    long double cc = cosl(x), ss = sinl(x);
    if (swap) {
        long double t = cc;
        cc = ss;
        ss = t;
    }
    c = sign_c * cc;
    s = -sign_s * ss;  // forward transform: exp(-i angle)
}

template <int L, int V> static void fill(double *out) {
    using P = Plan<L, V>;
    long long ns = 1;
    size_t idx = 0;
    for (int st = 0; st < P::NS; ++st) {
        const long long R = P::R[st];
        if (st > 0) {
            for (long long k = 0; k < ns; ++k)
                for (long long r = 0; r < R; ++r) {
                    long double c, s;
                    root_ld(r * k, ns * R, c, s);
                    out[2 * idx] = (double)c;
                    out[2 * idx + 1] = (double)s;
                    ++idx;
                }
        }
        ns *= R;
    }
}

int twiddle_entries(int L, int V) {
#define SCINT_VCASE(LL, VV) \
    if (L == LL && V == VV) return twiddle_count<LL, VV>();
    SCINT_VARIANTS_F32(SCINT_VCASE)
#undef SCINT_VCASE
    if (V != 0) return 0;
#define SCINT_CASE(LL) \
    case LL:           \
        return twiddle_count<LL, 0>();
    switch (L) {
        SCINT_SIZES_F32(SCINT_CASE)
    default:
        return 0;
    }
#undef SCINT_CASE
}

template <int L, int V> static int stages(TwiddleStages *d) {
    using P = Plan<L, V>;
    d->n = 0;
    int ns = 1;
    for (int st = 0; st < P::NS; ++st) {
        if (st > 0) {
            d->ns[d->n] = ns;
            d->R[d->n] = P::R[st];
            d->off[d->n] = twiddle_offset<L, V>(st);
            ++d->n;
        }
        ns *= P::R[st];
    }
    d->total = twiddle_count<L, V>();
    return d->n;
}

bool twiddle_stages(int L, int V, TwiddleStages *d) {
#define SCINT_VCASE(LL, VV)                  \
    if (L == LL && V == VV) {                \
        stages<LL, VV>(d);                   \
        return true;                         \
    }
    SCINT_VARIANTS_F32(SCINT_VCASE)
#undef SCINT_VCASE
    if (V != 0) return false;
#define SCINT_CASE(LL)      \
    case LL:                \
        stages<LL, 0>(d);   \
        return true;
    switch (L) {
        SCINT_SIZES_F32(SCINT_CASE)
    default:
        return false;
    }
#undef SCINT_CASE
}

bool build_twiddles(int L, int V, double *out) {
#define SCINT_VCASE(LL, VV)     \
    if (L == LL && V == VV) {   \
        fill<LL, VV>(out);      \
        return true;            \
    }
    SCINT_VARIANTS_F32(SCINT_VCASE)
#undef SCINT_VCASE
    if (V != 0) return false;
#define SCINT_CASE(LL)     \
    case LL:               \
        fill<LL, 0>(out);  \
        return true;
    switch (L) {
        SCINT_SIZES_F32(SCINT_CASE)
    default:
        return false;
    }
#undef SCINT_CASE
}

}  // namespace scint

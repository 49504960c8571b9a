// lds_layout.hpp -- where the row FFT's LDS exchanges put each element.
//
// Stage s of a plan writes its butterfly outputs to the Stockham positions
// p = B + r Ns (B = (j - k) R + k, k = j mod Ns, r < R) and stage s + 1 reads
// p = t + m T (m < E).  Exchange s stores element p at f_s(p):
//  * a linear layout f(p) = p + p / P (P = 0: f(p) = p) with a padding period
//    P that keeps both sides affine in r and m -- P divides Ns, or Ns R
//    divides P (then B and B + (R - 1) Ns lie in one period), and P divides T
//    -- so that a thread forms one address per butterfly and one per read
//    sweep, the rest being immediate offsets;
//  * otherwise the fixed layout p + (p >> sh), whose addresses are formed
//    element by element.
// The period is chosen at compile time per exchange: the fewest LDS bank
// conflicts of a wave's writes and reads (64 banks of 4 bytes assumed; a
// half wave's elements counted per bank group), at no more LDS than the fixed
// layout, preferring its period 2^sh, then no padding, then the longest
// period; the fixed layout only where every linear one conflicts more.
// Host-compilable (constexpr only), so that the choice can be listed and
// tested on the CPU.
#pragma once

#include "fft_plan.hpp"

namespace scint {

// LDS layout of a row in the fixed scheme: one padding slot every 32
// elements breaks the power-of-two strides of the Stockham writes across
// banks.  A row whose padded length would not fit the 160 KB of LDS (20000
// complex64), or would just miss the 80 KB that lets two workgroups share a
// CU (10000), takes one slot every 64 elements.
#ifndef SCINT_LDS_PAD_SHIFT
#define SCINT_LDS_PAD_SHIFT 5
#endif
constexpr int kLdsPadShift = SCINT_LDS_PAD_SHIFT;
template <int L> constexpr int lds_pad_shift() {
    if (kLdsPadShift <= 0 || kLdsPadShift >= 6) return kLdsPadShift;
    const int b = (L + (L >> kLdsPadShift)) * 8, b6 = (L + (L >> 6)) * 8;
    return (b > 160 * 1024 || (b > 80 * 1024 && b6 <= 80 * 1024)) ? 6 : kLdsPadShift;
}
template <int L> constexpr int fixed_layout_length() {
    return lds_pad_shift<L>() > 0 ? L + (L >> lds_pad_shift<L>()) : L;
}

struct ExchLayout {
    bool linear;  // false: p + (p >> sh)
    int P;        // linear: p + p / P (0: p)
    int length;   // elements the exchange occupies
};

constexpr int layout_at(const ExchLayout &lay, int sh, int p) {
    return lay.linear ? (lay.P > 0 ? p + p / lay.P : p) : (sh > 0 ? p + (p >> sh) : p);
}

// Bank-conflict degree of one wave's access: the largest number of lanes of
// a half wave whose elements fall in the same group of banks (elements of
// elem_bytes, 64 banks of 4 bytes).
template <int N> constexpr int conflict_degree(const int (&addr)[N], int n, int elem_bytes) {
    const int groups = 256 / elem_bytes;
    int worst = 0;
    for (int h = 0; h < n; h += 32) {
        int cnt[64] = {};
        for (int i = h; i < n && i < h + 32; ++i) {
            const int g = addr[i] % groups;
            if (++cnt[g] > worst) worst = cnt[g];
        }
    }
    return worst;
}

template <int L, int V> constexpr int exch_conflicts(const ExchLayout &lay, int s, int elem_bytes) {
    using P = Plan<L, V>;
    const int T = P::T, R = P::R[s], Ns = stage_ns<L, V>(s), sh = lds_pad_shift<L>();
    const int n = T < 64 ? T : 64;
    int worst = 0;
    int a[64] = {};
    for (int r = 0; r < 2 && r < R; ++r) {  // writes of butterflies j = t, outputs r
        for (int t = 0; t < n; ++t) {
            const int k = t % Ns;
            a[t] = layout_at(lay, sh, (t - k) * R + k + r * Ns);
        }
        const int c = conflict_degree(a, n, elem_bytes);
        if (c > worst) worst = c;
    }
    for (int t = 0; t < n; ++t) a[t] = layout_at(lay, sh, t);  // reads, m = 0
    const int c = conflict_degree(a, n, elem_bytes);
    return c > worst ? c : worst;
}

template <int L, int V> constexpr bool linear_ok(int s, int Pd) {
    using P = Plan<L, V>;
    const int T = P::T, R = P::R[s], Ns = stage_ns<L, V>(s);
    if (Pd == 0) return true;
    return (Ns % Pd == 0 || Pd % (Ns * R) == 0) && T % Pd == 0;
}

// The layout of exchange s (0 <= s < NS - 1) for elements of elem_bytes.
template <int L, int V> constexpr ExchLayout exch_layout(int s, int elem_bytes) {
    using P = Plan<L, V>;
    const int T = P::T, sh = lds_pad_shift<L>(), limit = fixed_layout_length<L>();
    ExchLayout best{false, 0, limit};
    int best_c = exch_conflicts<L, V>(best, s, elem_bytes);
    bool have_linear = false;
    auto consider = [&](int Pd) {
        if (!linear_ok<L, V>(s, Pd)) return;
        const int len = Pd > 0 ? L + L / Pd : L;
        if (len > limit) return;
        const ExchLayout cand{true, Pd, len};
        const int c = exch_conflicts<L, V>(cand, s, elem_bytes);
        if (c < best_c || (c == best_c && !have_linear)) {
            best = cand;
            best_c = c;
            have_linear = true;
        }
    };
    if (sh > 0) consider(1 << sh);
    consider(0);
    for (int Pd = T; Pd >= 2; --Pd)
        if (T % Pd == 0) consider(Pd);
    return best;
}

// Elements a row's exchange buffer takes: the largest exchange layout.
template <int L, int V> constexpr int exch_buffer_length(int elem_bytes) {
    int len = L;
    for (int s = 0; s + 1 < Plan<L, V>::NS; ++s) {
        const int l = exch_layout<L, V>(s, elem_bytes).length;
        if (l > len) len = l;
    }
    return len;
}

}  // namespace scint

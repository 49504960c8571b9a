// Host check of the row FFT's LDS exchange layouts (lds_layout.hpp), built
// and run by tests/test_lds_layout.py: for every plan and exchange, the
// layout maps the L elements to distinct slots inside the row's buffer, and
// where it is linear, the per-butterfly and per-sweep addresses the kernel
// forms (one address plus a constant step) equal the layout of each element.
#include <cstdio>
#include <vector>

#include "lds_layout.hpp"

using namespace scint;

static int failures = 0;

template <int L, int V> static void check(int eb) {
    using P = Plan<L, V>;
    const int T = P::T, E = P::E, sh = lds_pad_shift<L>(), buf = exch_buffer_length<L, V>(eb);
    for (int s = 0; s + 1 < P::NS; ++s) {
        const ExchLayout lay = exch_layout<L, V>(s, eb);
        const int R = P::R[s], Ns = stage_ns<L, V>(s);
        std::vector<char> used(buf, 0);
        for (int p = 0; p < L; ++p) {
            const int a = layout_at(lay, sh, p);
            if (a < 0 || a >= buf || used[a]) {
                std::printf("FAIL L=%d V=%d eb=%d s=%d: element %d at %d (buffer %d)\n", L, V, eb, s, p, a, buf);
                ++failures;
                return;
            }
            used[a] = 1;
        }
        if (!lay.linear) continue;
        const int wstep = Ns + ((lay.P > 0 && Ns % lay.P == 0) ? Ns / lay.P : 0);
        for (int j = 0; j < L / R; ++j) {
            const int k = j % Ns, base = (j - k) * R + k;
            const int q = lay.P > 0 ? base + base / lay.P : base;
            for (int r = 0; r < R; ++r)
                if (q + r * wstep != layout_at(lay, sh, base + r * Ns)) {
                    std::printf("FAIL L=%d V=%d eb=%d s=%d: write j=%d r=%d\n", L, V, eb, s, j, r);
                    ++failures;
                    return;
                }
        }
        const int rstep = T + (lay.P > 0 ? T / lay.P : 0);
        for (int t = 0; t < T; ++t) {
            const int q = lay.P > 0 ? t + t / lay.P : t;
            for (int m = 0; m < E; ++m)
                if (q + m * rstep != layout_at(lay, sh, t + m * T)) {
                    std::printf("FAIL L=%d V=%d eb=%d s=%d: read t=%d m=%d\n", L, V, eb, s, t, m);
                    ++failures;
                    return;
                }
        }
    }
    std::printf("ok L=%d V=%d eb=%d buffer=%d\n", L, V, eb, buf);
}

int main() {
#define SCINT_F64_CASE(LL) check<LL, 0>(16);
    SCINT_SIZES_F64(SCINT_F64_CASE)
#define SCINT_F32_CASE(LL) check<LL, 0>(8);
    SCINT_SIZES_F32(SCINT_F32_CASE)
#define SCINT_V_CASE(LL, VV) check<LL, VV>(8);
    SCINT_VARIANTS_F32(SCINT_V_CASE)
    std::printf("%d failures\n", failures);
    return failures ? 1 : 0;
}

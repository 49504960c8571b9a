// row_inst.hip -- explicit instances of the row-pass kernel for one precision
// and one program, selected at compile time by SCINT_REAL and SCINT_PROG
// (the build compiles this file once per pair).
#include "row_kernel.hpp"
#include "row_launch.h"

#ifndef SCINT_REAL
#error "SCINT_REAL (float or double) must be defined"
#endif
#ifndef SCINT_PROG
#error "SCINT_PROG (a program name such as ProgNoise) must be defined"
#endif

#define SCINT_CAT2(a, b) a##b
#define SCINT_CAT(a, b) SCINT_CAT2(a, b)

namespace scint {

template <int L, int V>
static hipError_t launch_one(const RowProgram &prog, const void *tw, hipStream_t stream) {
    using Cfg = RowCfg<SCINT_REAL, L, V>;
    RowProgram p = prog;
    // two workgroups per row only where the program allows it, the loop has
    // two or more iterations and the row workgroups come in whole eights
    const int row_wgs = (prog.total_rows + Cfg::B - 1) / Cfg::B;
    p.iter_split = (prog.iter_split == 2 && iter_splittable<SCINT_PROG>() && prog.n_iter >= 2 && row_wgs % 8 == 0)
                       ? 2 : 1;
    const int rows_blocks = row_wgs * p.iter_split;
    if constexpr (has_side<SCINT_PROG>()) {
        // groups of fft_blocks row workgroups and side_blocks transpose
        // workgroups; the units are spread evenly over the latter
        RowSide &sd = p.side;
        const int64_t units = sd.u1 - sd.u0;
        if (sd.fft_blocks < 1 || sd.side_blocks < 1 || units < 1 || sd.u0 < 0 || !sd.in || !sd.out)
            return hipErrorInvalidValue;
        sd.groups = (rows_blocks + sd.fft_blocks - 1) / sd.fft_blocks;
        const int64_t nside = (int64_t)sd.groups * sd.side_blocks;
        const int64_t per = (units + nside - 1) / nside;
        if (per > (1 << 30) || (int64_t)sd.groups * (sd.fft_blocks + sd.side_blocks) > (1ll << 31) - 1)
            return hipErrorInvalidValue;
        sd.units_per_block = (int32_t)per;
        const int grid = sd.groups * (sd.fft_blocks + sd.side_blocks);
        hipLaunchKernelGGL((row_kernel<SCINT_REAL, L, V, SCINT_PROG>), dim3(grid), dim3(Cfg::THREADS), 0, stream, p,
                           static_cast<const cpx<SCINT_REAL> *>(tw));
    } else {
        hipLaunchKernelGGL((row_kernel<SCINT_REAL, L, V, SCINT_PROG>), dim3(rows_blocks), dim3(Cfg::THREADS), 0,
                           stream, p, static_cast<const cpx<SCINT_REAL> *>(tw));
    }
    return hipGetLastError();
}

template <>
hipError_t launch_row<SCINT_REAL, SCINT_CAT(SCINT_PROG, Tag)>(int L, int V, const RowProgram &prog, const void *tw,
                                                               hipStream_t stream) {
#define SCINT_CASE(LL) \
    case LL:           \
        if (V == 0) return launch_one<LL, 0>(prog, tw, stream); \
        break;
#define SCINT_VCASE(LL, VV) \
    if (L == LL && V == VV) return launch_one<LL, VV>(prog, tw, stream);
#if !SCINT_IS_F64
    SCINT_VARIANTS_F32(SCINT_VCASE)
#endif
    switch (L) {
#if SCINT_IS_F64
        SCINT_SIZES_F64(SCINT_CASE)
#else
        SCINT_SIZES_F32(SCINT_CASE)
#endif
    default:
        break;
    }
    return hipErrorInvalidValue;
#undef SCINT_CASE
#undef SCINT_VCASE
}

}  // namespace scint

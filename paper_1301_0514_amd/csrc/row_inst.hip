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
    const int grid = (prog.total_rows + Cfg::B - 1) / Cfg::B;
    hipLaunchKernelGGL((row_kernel<SCINT_REAL, L, V, SCINT_PROG>), dim3(grid), dim3(Cfg::THREADS), 0, stream,
                       prog, static_cast<const cpx<SCINT_REAL> *>(tw));
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

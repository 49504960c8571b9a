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

template <int L>
static hipError_t launch_one(const RowProgram &prog, const void *tw, hipStream_t stream) {
    using Cfg = RowCfg<SCINT_REAL, L>;
    const int grid = (prog.total_rows + Cfg::B - 1) / Cfg::B;
    hipLaunchKernelGGL((row_kernel<SCINT_REAL, L, SCINT_PROG>), dim3(grid), dim3(Cfg::THREADS), 0, stream,
                       prog, static_cast<const cpx<SCINT_REAL> *>(tw));
    return hipGetLastError();
}

template <>
hipError_t launch_row<SCINT_REAL, SCINT_CAT(SCINT_PROG, Tag)>(int L, const RowProgram &prog, const void *tw,
                                                               hipStream_t stream) {
#define SCINT_CASE(LL) \
    case LL:           \
        return launch_one<LL>(prog, tw, stream);
    switch (L) {
#if SCINT_IS_F64
        SCINT_SIZES_F64(SCINT_CASE)
#else
        SCINT_SIZES_F32(SCINT_CASE)
#endif
    default:
        return hipErrorInvalidValue;
    }
#undef SCINT_CASE
}

}  // namespace scint

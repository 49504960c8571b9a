// row_launch.h -- host-side launchers of the row-pass kernels, one per
// (precision, program), each dispatching on the row length at run time.
#pragma once

#include <hip/hip_runtime.h>

#include "row_program.h"

namespace scint {

struct ProgNoiseTag;
struct ProgNoiseSwapTag;
struct ProgScreenTag;
struct ProgScreenPropTag;
struct ProgPhasePropTag;
struct ProgPropIntensityTag;
struct ProgRealFwdTag;
struct ProgFwdReTag;
struct ProgSmearMidTag;
struct ProgInvReTag;
struct ProgVjpYTag;
struct ProgPropFieldTag;
struct ProgVjpYFieldTag;
struct ProgVjpXTag;
struct ProgApertureXTag;
struct ProgAbs2Tag;
struct ProgNoiseTTag;          // complex64 only
struct ProgNoiseSwapTTag;      // complex64 only
struct ProgPhasePropTTag;     // complex64 only
struct ProgPropIntensityTTag;  // complex64 only
struct ProgRealFwdTTag;        // complex64 only
struct ProgSmearMidTTag;       // complex64 only
struct ProgInvReTTag;          // complex64 only

// Launches program Tag on total_rows rows of length L (the grid size N) with
// plan variant V; tw is the device twiddle table of that plan in the same
// precision.  Returns hipErrorInvalidValue for an unsupported (L, V).  For
// programs with side transposes the launcher sizes the grid from
// prog.side.fft_blocks and side_blocks and fills groups and units_per_block.
template <typename Real, class Tag>
hipError_t launch_row(int L, int V, const RowProgram &prog, const void *tw, hipStream_t stream);

// Number of twiddle entries of plan (L, V) (0 if unsupported), and a builder
// that fills them: W_{Ns R}^{r k} = exp(-2 pi i r k / (Ns R)) for every stage
// s >= 1, k < Ns, r < R, evaluated in extended precision.
int twiddle_entries(int L, int V);
bool build_twiddles(int L, int V, double *out_ri /* 2 * twiddle_entries(L, V) */);

// The same tables described by their stages (for a device-side build): for
// each stage s >= 1 of plan (L, V), the span ns of the earlier stages, its
// radix R and the offset of its ns R entries; total entries in `total`.
struct TwiddleStages {
    int n;
    int ns[8], R[8], off[8];
    int total;
};
bool twiddle_stages(int L, int V, TwiddleStages *d);

}  // namespace scint

// row_program.h -- the small program a row-pass kernel executes.  Plain data,
// shared by the host (which builds programs) and the kernels (which run them).
//
// A row pass gives each row of a batch of N x N arrays to T = N/E threads that
// keep the row in registers (element e = t + m T in register m).  The program
// is a list of operations applied to that register row: loads (complex, real,
// exp(i s phi), or the random phase spectrum), forward and inverse FFTs along
// the row, pointwise multiplies (Fresnel chirp, disk spectrum, gradient),
// and stores.  An optional loop repeats a range of operations n_iter times
// (over wavelengths or source radii) with per-iteration pointer offsets,
// phase scales and weights.
#pragma once

#include <stdint.h>

namespace scint {

enum RowOpCode : int32_t {
    ROP_END = 0,
    ROP_LOAD_C,      // v = src[e]                      (complex)
    ROP_LOAD_R,      // v = (src[e], 0)                 (real)
    ROP_LOAD_PHASE,  // v = exp(i s src[e])             (real phase; s = phase scale)
    ROP_NOISE,       // v = random phase spectrum, row = kx, element = ky
    ROP_KEEP_R,      // keep = src[e]                   (real, kept for ROP_EXP_KEEP)
    ROP_EXP_KEEP,    // v = exp(i s keep)
    ROP_FFT_FWD,     // v = DFT(v)   (kernel exp(-2 pi i e k / N))
    ROP_FFT_INV,     // v = IDFT(v)  (kernel exp(+2 pi i e k / N), unnormalised)
    ROP_MUL_TAB,     // v *= tab[e]  (complex table along the row; flag 1: conjugate)
    ROP_MUL_RTAB2D,  // v *= tab[min(row, N - row)][min(e, N - e)]: the quarter 0..N/2 x 0..N/2 of a real
                     //   table even in both signed indices (row_stride N/2 + 1; no batch offset)
    ROP_MUL_RLOAD,   // v *= param * src[e]  (real array)
    ROP_SQRT2RE,     // v = (sqrt(2) Re v, 0); FP32: v = (hi, lo) of sqrt(2) Re v
                     //   plus the FP64 low modes of the row (low_tab)
    ROP_EXP_RE,      // v = exp(i s Re v); FP32: exp(i s (Re v + Im v)), the sum in FP64
    ROP_STORE_C,     // dst[e] = v
    ROP_STORE_R,     // dst[e] = param * Re v
    ROP_ACC_ABS2,    // acc += w |v|^2
    ROP_STORE_ACC,   // dst[e] = acc   (flag 1: dst[e] += acc)
    ROP_SAVE,        // keepc = v
    ROP_RESTORE,     // v = keepc
    ROP_GRAD_PHI,    // v = (s Im(v conj(exp(i s src[e]))), 0)   (src = phi)
    ROP_DOT_R,       // ptr2[global row] = sum_e src[e] Re v   (double)
    ROP_LOOP,        // start of the repeated range
    ROP_ENDLOOP,     // end of the repeated range
    ROP_MUL_ROWTAB,  // v *= tab[row]  (complex, one factor per row)
    ROP_SIDE_T,      // first op only: the launch also runs the transposes of RowProgram::side
    ROP_ACC_ABS2U,   // acc[e] += |v|^2, no weight (two fused multiply-adds per element)
    ROP_NOISE_SWAP,  // ROP_NOISE with row = ky, element = kx (screens made transposed)
};

// Flag bits
enum : int32_t {
    RF_CONJ = 1,       // ROP_MUL_TAB: multiply by the conjugate
    RF_ADD = 1,        // ROP_STORE_ACC: accumulate into dst
    RF_ITER_SCALE = 2, // phase scale s = scale[it] (else param)
    RF_ITER_WEIGHT = 4, // ROP_ACC_ABS2: w = weight[it] (else param)
    RF_PAIR = 8         // ROP_LOAD_R: v = (src[e], ptr2[e]); ROP_STORE_R: dst[e] = Re, ptr2[e] = Im
};

// Address of element e of row `row` of batch b at loop iteration it:
//   ptr + b * batch_stride + it * iter_stride + row * row_stride + e
// (strides in elements of the operand's type).
struct RowOp {
    int32_t code;
    int32_t flags;
    int64_t batch_stride;
    int64_t iter_stride;
    int64_t row_stride;
    const void *ptr;
    void *ptr2;      // ROP_DOT_R: double destination, one value per global row
    double param;
};

constexpr int kRowMaxOps = 20;
constexpr int kRowMaxIter = 64;

// Half-width of the square of lowest Fourier modes, |kx'|, |ky'| <= K, that
// the FP32 screens synthesise in FP64 (the FP32 transforms carry the rest):
// 16, or N/2 - 1 on grids too small for it (the Nyquist row and column stay
// with the transforms).
constexpr int32_t low_modes_k_of(int N) { return N / 2 - 1 < 16 ? N / 2 - 1 : 16; }

// Transposes a row pass carries as extra workgroups of its own launch
// (programs whose first op is ROP_SIDE_T; complex64 only): units [u0, u1) of
// the N x N matrices at `in`, written transposed to the same place in `out`.
// Unit u is matrix u / (ux uy), then row band, then column band, with
// ux x uy units of 64 rows by 128 columns per matrix (transpose_tile.hpp).
// The grid is made of `groups` groups, each of fft_blocks row workgroups
// followed by side_blocks transpose workgroups that take units_per_block
// consecutive units each; the launcher fills groups and units_per_block.
// The row pass and the transposes must not touch each other's data.
struct RowSide {
    const void *in;
    void *out;
    int64_t u0, u1;
    int32_t fft_blocks, side_blocks;
    int32_t groups, units_per_block;
};

struct RowProgram {
    RowOp op[kRowMaxOps];
    RowSide side;
    int32_t n_iter;      // iterations of the loop range (>= 1)
    int32_t N;           // row length (= grid size)
    int32_t total_rows;  // batch * N
    int32_t r0;          // realisation of batch 0 (ROP_NOISE)
    uint32_t seed_lo, seed_hi;
    double amp0;         // sqrt(C_beta R^(2-beta)) N^(beta/2) / N   (ROP_NOISE)
    double neg_beta_4;   // -beta/4                                 (ROP_NOISE)
    double scale[kRowMaxIter];
    double weight[kRowMaxIter];
    // 1, or 2: each row is taken by two workgroups, 8 apart in launch order
    // (one XCD, dispatched together), the first doing the loop's first
    // ceil(n_iter/2) iterations and the second the rest, so that per-row
    // operands re-read in every iteration are fetched by both from one L2.
    // Only for programs whose iterations are independent; the launcher
    // falls back to 1 where it does not apply (the results are the same).
    int32_t iter_split;
    // FP32 screens: ROP_NOISE leaves out the Fourier modes with |kx'|,
    // |ky'| <= low_k (low_modes_k_of(N); 0 in every other program and in
    // FP64), and ROP_SQRT2RE adds them back in FP64 from low_tab, the table
    // [batch][N][low_modes_k_of(N) + 1] of complex doubles G with
    // phi_low(x, y) = Re sum_k G[b][y][k] exp(2 pi i k x / N) (required by
    // every FP32 program that contains ROP_SQRT2RE).
    int32_t low_k;
    const void *low_tab;
};

// Feature sets: which register arrays beyond the row itself a kernel keeps.
enum RowFeature : int { RFEAT_PLAIN = 0, RFEAT_KEEP = 1, RFEAT_ACC = 2, RFEAT_KEEPC = 4 };

}  // namespace scint

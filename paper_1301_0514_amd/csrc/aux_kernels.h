// aux_kernels.h -- launchers of the non-FFT kernels: batched transposes,
// chirp tables, disk images, reductions and the L2 loss.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace scint {

// out[b][x][y] = in[b][y][x] for b < nbatch; elem_bytes in {4, 8, 16}.
hipError_t launch_transpose(const void *in, void *out, int N, int64_t nbatch, int elem_bytes,
                            hipStream_t stream);

// tab[j][k] = scale amp[j] exp(-2 pi i a[j] k'^2), k' the signed frequency
// of k, for j < n (n <= 64); a[j] = pi rho_j^2 / N^2 (turns per k'^2); amp
// NULL means amp[j] = 1.  The turn count is formed and reduced in FP64 and
// the sine/cosine taken in FP64.
hipError_t launch_chirp_tables(void *tab, int N, const double *a, int n, double scale, bool f64,
                               hipStream_t stream, const double *amp = nullptr);

// The twiddle table of an FFT plan built on the device: entry off[s] + k R[s]
// + r = exp(-2 pi i r k / (ns[s] R[s])) for the stages described (n <= 8,
// `total` entries), the product r k reduced modulo ns R in integers and the
// sine/cosine taken in FP64, rounded once to the working precision.
hipError_t launch_twiddle_table(void *tab, int n_stages, const int *ns, const int *R, const int *off, int total,
                                bool f64, hipStream_t stream);

// img[y][x] = value if dx^2 + dy^2 <= r2 (minimum-image offsets of pixel
// (x, y) from the origin), else 0.
hipError_t launch_disk_image(void *img, int N, double r2, double value, bool f64, hipStream_t stream);

// partials[b * nblk + blk] = sum over block blk's share of batch b of
// (x - center[b])^power  (center may be NULL = 0; power 1 or 2), FP64.
hipError_t launch_block_sums(const void *x, int64_t n_per_batch, int nbatch, const double *center,
                             int power, int nblk, bool f64, double *partials, hipStream_t stream);

// As launch_block_sums over a w x h region of each batch member: rows of
// w elements, row_stride apart, starting at x + b * batch_stride.
hipError_t launch_region_sums(const void *x, int64_t batch_stride, int64_t w, int64_t h, int64_t row_stride,
                              int nbatch, const double *center, int power, int nblk, bool f64, double *partials,
                              hipStream_t stream);

// tab[j] = SF(j + 1/2) exp(i (2 pi a (j - N/2)^2 + pi j)), j < N, with SF the
// raised-sine window over Lm pixels at each border (Lm = 0: SF = 1); the
// phase is formed and reduced in FP64 turns, the sine/cosine taken in FP64.
hipError_t launch_aperture_table(void *tab, int N, double a, double Lm, bool f64, hipStream_t stream);

// Light curves: lines of 4 doubles (x0, y0, dx, dy) in pixels, passed by
// value kLinesPerLaunch at a time; out[b][l][k] = the pattern b sampled at
// (x0 + k dx, y0 + k dy) (mode 0 nearest pixel, 1 bilinear, periodic);
// stats[2 (b n_lines + l) + {0, 1}] = mean and population variance (FP64) if
// stats != NULL.
constexpr int kLinesPerLaunch = 64;
struct LineSet {
    double p[kLinesPerLaunch][4];
};
hipError_t launch_light_curves(const void *I, int N, int nbatch, const double *lines, int n_lines, int n_samples,
                               int mode, bool f64, void *out, double *stats, hipStream_t stream);

// Ring sums of a power map P [nbatch][N][N] (real): S[b][k] = mean of P over
// the pixels whose signed frequency |k'| rounds to k, k = 0 .. N/2, in FP64;
// count[k] = their number (if count != NULL).
hipError_t launch_ring_sums(const void *P, int N, int nbatch, bool f64, double *S, double *count, hipStream_t stream);

// D(r) = 2 (xi(0) - xi(r)) from ring spectra S [nbatch][N/2 + 1] (pixel units,
// the J0 sum of Eq. crec) at n_r radii (pixels; by value, kRadiiPerLaunch at a
// time) into D [nbatch][n_r], and R_diff^rec (D = 1) into rdiff [nbatch] if
// rdiff != NULL (NaN if not bracketed in [1e-3, N/2]).
constexpr int kRadiiPerLaunch = 64;
struct RadiusSet {
    double r[kRadiiPerLaunch];
};
hipError_t launch_hankel(const double *S, int N, int nbatch, const double *radii, int n_r, double *D, double *rdiff,
                         hipStream_t stream);

// The lowest Fourier modes of FP32 screens, synthesised in FP64 (Sect. 3.1):
// for realisations r0 + b, b < nbatch, with W = 2K + 1,
//   C[b][i][j] = c(kx' = i - K, ky' = j - K), the FP64 spectrum coefficient
//                (Philox counter (kx, ky, r, 0), key (seed_lo, seed_hi)),
//   G[b][y][k] = sqrt(2) (B(k) + conj(B(-k))) for 1 <= k <= K, sqrt(2) B(0)
//                for k = 0, B(kx') = sum_{|ky'| <= K} c(kx', ky') exp(2 pi i ky' y / N),
// so that sqrt(2) Re of their part of the inverse DFT is
// Re sum_k G[b][y][k] exp(2 pi i k x / N).  With swap the roles of x and y
// (kx' and ky') are exchanged: G[b][x][k] for screens kept transposed,
// [b][x][y].  C is scratch (nbatch W^2 complex doubles); G is
// [nbatch][N][K + 1] complex doubles.  K < N/2.
hipError_t launch_low_modes(void *C, void *G, int N, int K, int nbatch, uint32_t r0, uint32_t seed_lo,
                            uint32_t seed_hi, double amp0, double neg_beta_4, hipStream_t stream, bool swap = false);

// out[b] = scale * sum_blk partials[b * nblk + blk], fixed-order tree.
hipError_t launch_finalize_sums(const double *partials, int nblk, int nbatch, double scale, double *out,
                                hipStream_t stream);

// grad[i] = 2 (I[i] - It[i]) (if grad != NULL); partials as launch_block_sums
// of (I - It)^2.
hipError_t launch_l2_loss(const void *I, const void *It, void *grad, int64_t n_per_batch, int nbatch,
                          int nblk, bool f64, double *partials, hipStream_t stream);

}  // namespace scint

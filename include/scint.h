/*
 * scint.h -- C ABI of the MI355X (gfx950) phase-screen + Fresnel propagation
 * library (libscint.so).
 *
 * The operations follow Habibi, Moniez, Ansari & Rahvar, "Simulation of
 * optical interstellar scintillation" (A&A 2013, arXiv:1301.0514).  Citations
 * name the section and equation of that paper.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Grids are square, N x N pixels of side `delta` (Sect. 3.1).  Supported N
 *    are listed by ps_supported_size(); every other N returns PS_E_SIZE.
 *  - Arrays are device memory owned by the caller, contiguous, row-major
 *    [batch][N][N] with y (row) slow and x fast, 16-byte aligned (else
 *    PS_E_PARAM).  Real arrays hold float (dtype PS_F32) or double (PS_F64).
 *    The library never frees caller memory.
 *  - delta, lambda, z, r_diff and source radii share one length unit of the
 *    caller's choice.  The Fresnel radius is R_F = sqrt(lambda z / 2 pi)
 *    (Sect. 2, Eq. Rfresnel); the screen-observer distance z is the effective
 *    distance of the footnote to Eq. Rfresnel when the source is not far.
 *  - Work is enqueued asynchronously on `hip_stream` (a hipStream_t; NULL is
 *    the null stream); the caller synchronises.  Entry points returning host
 *    scalars (m_out, loss_out, phi_dot_grad_out) synchronise the stream first.
 *  - The library keeps a per-device cache of FFT twiddle tables, disk spectra
 *    and a per-stream workspace; the first call of a given shape allocates it
 *    (hipMalloc), later calls of that shape or smaller allocate nothing.  Calls
 *    that overlap on the same stream are ordered by the stream; calls on two
 *    streams use two workspaces.  ps_release_cache() frees everything.
 *  - Graph capture: a call made while hip_stream is being captured into a
 *    HIP graph returns PS_E_CAPTURE, before enqueuing anything, if it would
 *    have to allocate (a first use of a size, radius set or larger batch on
 *    that stream), tune an FFT plan, copy tables from the host or synchronise
 *    (entry points returning host values).  Make the same call once before
 *    the capture, or call ps_tune_plans(); the captured call then enqueues
 *    kernels only.
 *  - Every entry point returns a ps_status.  Arguments are validated before
 *    anything is launched; on error nothing is written and ps_last_error()
 *    returns a message (thread-local).  PS_E_DEVICE reports a failing HIP call.
 *  - All arithmetic of the FP32 path is in FP32, with FFT twiddles and chirp
 *    tables computed in FP64 and rounded once, and the phase arguments of
 *    exp(i s phi) reduced modulo 2 pi in FP64 before the FP32 sine/cosine.
 */
#ifndef SCINT_H
#define SCINT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { PS_F32 = 0, PS_F64 = 1 } ps_dtype;

typedef enum {
    PS_OK = 0,
    PS_E_NULL = -1,          /* a required pointer is NULL                      */
    PS_E_SIZE = -2,          /* N (or a count) unsupported / too large          */
    PS_E_PARAM = -3,         /* a physical parameter is non-finite or out of range */
    PS_E_DTYPE = -4,         /* dtype is not PS_F32 or PS_F64                   */
    PS_E_ALLOC = -5,         /* device memory for the workspace or cache failed */
    PS_E_DEVICE = -6,        /* a HIP call or kernel launch failed              */
    PS_E_ALIAS = -7,         /* output overlaps an input where that is not allowed */
    PS_E_UNIMPLEMENTED = -8, /* combination the library does not provide       */
    PS_E_CAPTURE = -9        /* would allocate or synchronise during graph capture */
} ps_status;

/* 1 if N is supported for dtype, else 0.  The FP32 set is
 * {16,32,...,16384} (powers of two) and {40,80,100,160,200,320,400,640,1000,
 * 1280,2000,2560,4000,5000,8000,10000} (2^a 5^b); the FP64 set is the same
 * up to 8192.  */
int ps_supported_size(int N, int dtype);

/* Number of supported sizes for dtype, and the i-th of them (ascending). */
int ps_num_supported_sizes(int dtype);
int ps_supported_size_at(int dtype, int i);

/*
 * ps_generate -- random phase screens (Sect. 3.1, Eqs. spectre and densite).
 *
 * For realisation r = first_realisation + b (b = 0..n_real-1) and every Fourier
 * pixel k = (kx, ky) of the FFT grid (kx, ky in [0, N), signed frequency
 * k' = k for k < N/2 else k - N):
 *   counter = (kx, ky, r, 0), key = (seed mod 2^32, seed >> 32);
 *   (w0..w3) = Philox4x32-10(counter, key);
 *   u1 = ((((w0 << 32) | w1) >> 11) + 1/2) 2^-53, u2 likewise from (w2, w3);
 *   g = sqrt(-2 ln u1) (cos 2 pi u2 + i sin 2 pi u2);
 *   c[k] = sqrt(S(q)) / N * g / sqrt(2),  q = |k'| / N cycles per pixel,
 *   with S(q) = R^2 / (2 (2 pi)^(beta-1) f(beta)) (R q)^(-beta),
 *   f(beta) = 2^-beta beta Gamma(-beta/2) / Gamma(beta/2), R = r_diff/delta;
 *   c[0] = 0.
 * The screen is phi[m] = sqrt(2) Re sum_k c[k] exp(+2 pi i k.m / N) (radians).
 * The "Gaussian of width L_x L_y S" of the paper is read as variance L_x L_y S
 * per part, so that <|F_phi|^2> = L_x L_y S (Eq. densite) with c = F_phi/L^2.
 *
 *   N, delta          grid size and pixel side (delta > 0)
 *   r_diff            diffraction radius R_diff (> 0), where D_phi = 1 (Eq. dphi)
 *   beta              spectral exponent, 2 < beta < 4 (11/3 = Kolmogorov)
 *   seed, first_realisation, n_real   noise stream selection (n_real >= 1)
 *   phi_out           device [n_real][N][N] real (dtype)
 * A warning (ps_last_warning) is set when delta >= r_diff/2, the sampling
 * criterion of Sect. 3.2.2.
 * In FP32 from N = 2048 a batch is split into up to four jobs of consecutive
 * realisations whose noise passes carry the previous job's transpose as
 * extra workgroups (SCINT_SCREEN_JOBS=<n> in the environment sets the
 * number, 1 turns the split off); every value is the same bit for bit.
 */
int ps_generate(int N, double delta, double r_diff, double beta, uint64_t seed,
                uint32_t first_realisation, int n_real, int dtype, void *phi_out,
                void *hip_stream);

/*
 * fresnel_propagate -- point-source illumination pattern (Sect. 2, Eq. hxy).
 *
 * For each of the n screens phi (radians, scaled by phase_scale s):
 *   U = exp(i s phi);  A = N^-2 IDFT[ H(k) DFT[U](k) ];  I = |A|^2,
 *   H(k) = H1(kx') H1(ky'),  H1(k') = exp(-i 2 pi^2 rho^2 k'^2 / N^2),
 *   rho = R_F / delta = sqrt(lambda z / 2 pi) / delta,
 * which is the Fresnel-Huygens integral of Eq. hxy on the periodic screen,
 * normalised so that a uniform screen gives I = 1 (so <I> = 1).  At
 * N = 2 pi rho^2 it equals the direct sum of Eq. hxy and the one-FFT form of
 * Sect. 3.2 (Eqs. intens, Gxy).  phase_scale = lambda_ref / lambda re-uses a
 * screen given at lambda_ref (phi scales as 1/lambda, Sect. 2, Eq. phiNl).
 *
 *   phi       device [n][N][N] real (input, not modified)
 *   I_out     device [n][N][N] real; must not overlap phi (PS_E_ALIAS)
 * In FP32 from N = 2048 up with n >= 2 the screens run as the pipelined jobs
 * of illumination_polychromatic (one wavelength), with the same result.
 */
int fresnel_propagate(int N, double delta, double lambda, double z, const void *phi,
                      double phase_scale, int n, int dtype, void *I_out, void *hip_stream);

/*
 * fresnel_propagate_noalloc -- fresnel_propagate for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, result and errors as
 * fresnel_propagate, computed by the same kernels in the plain order (x pass,
 * transpose, y pass, transpose) with FFT plan 0 and its twiddle table built on
 * the device, so FP32 results agree with fresnel_propagate to FP32 rounding.
 * Its intermediates live in one static device array per GPU of 65 MiB
 * (68157440 bytes), held from the library's load until the process ends; a
 * call needs 16 N^2 n bytes (FP32; 32 N^2 n in FP64) plus its tables there
 * and returns PS_E_SIZE, writing nothing, when that exceeds the array (FP32:
 * up to n = 1 at N = 2048, n = 4 at 1024; FP64: n = 2 at 1024).  The call
 * enqueues kernels only: no hipMalloc, hipFree, host copy or
 * synchronisation, no plan tuning and no cached tables; the first call on a
 * device resolves the array's device address (hipGetSymbolAddress).  Every
 * call on one GPU uses the same array: calls that overlap in time on one GPU
 * (on different streams, or from several threads) race and corrupt each
 * other's results, so serialise them, e.g. on one stream.
 */
int fresnel_propagate_noalloc(int N, double delta, double lambda, double z, const void *phi,
                              double phase_scale, int n, int dtype, void *I_out, void *hip_stream);

/*
 * fresnel_propagate_field -- fresnel_propagate that also keeps the complex
 * field A = N^-2 IDFT[H DFT[U]] of each screen as the checkpoint of its
 * adjoint (fresnel_propagate_vjp's `field`), in the layout of the second
 * 1-D pass: field_out[b][x][y] (x slow, y fast; interleaved re, im), so
 * that I[b][y][x] = |field_out[b][x][y]|^2.  Same kernels and result as the
 * plain (single-job) order of fresnel_propagate.
 *   field_out  device [n][N][N] complex (2 n N^2 reals); must not overlap
 *              phi or I_out (PS_E_ALIAS)
 */
int fresnel_propagate_field(int N, double delta, double lambda, double z, const void *phi,
                            double phase_scale, int n, int dtype, void *I_out, void *field_out,
                            void *hip_stream);

/*
 * ps_screen_fresnel -- ps_generate followed by fresnel_propagate with s = 1,
 * fused so that the screen need not go through device memory.
 *   phi_out    optional device [n_real][N][N] real copy of the screen, or NULL
 *   I_out      device [n_real][N][N] real
 *   field_out  optional device [n_real][N][N] complex checkpoint of the field
 *              for fresnel_propagate_vjp (layout of fresnel_propagate_field),
 *              or NULL
 * The FP32 screen's lowest Fourier modes (|kx'|, |ky'| <= 16) are synthesised
 * in FP64 and the phase of exp(i phi) is formed from the screen to FP64
 * accuracy; phi_out holds the screen rounded once to FP32.  With phi_out and
 * field_out both NULL the screen is made transposed and the two propagation
 * passes run in the other order (no final transpose): the same pattern up to
 * the rounding of the differently ordered transforms, not bit for bit the
 * one a call that also returns the screen gives.
 */
int ps_screen_fresnel(int N, double delta, double r_diff, double beta, uint64_t seed,
                      uint32_t first_realisation, int n_real, double lambda, double z,
                      int dtype, void *phi_out, void *I_out, void *field_out, void *hip_stream);

/*
 * illumination_polychromatic -- co-added pattern over a passband
 * (Sect. 3.2.4).  The same screen phi_ref, given at lambda_ref, is seen at each
 * lambda_j with phase scale s_j = lambda_ref / lambda_j (Eq. phiNl) and
 * Fresnel radius sqrt(lambda_j z / 2 pi) (Eq. Rfresnel):
 *   I = sum_j w_j I_j / sum_j w_j.
 *   lambdas, weights   host arrays of n_lambda entries; weights may be NULL
 *                      (equal weights); weights >= 0 with a positive sum
 *   n_lambda           1 .. 4096
 *   phi_ref   device [n_real][N][N] real;  I_out device [n_real][N][N] real
 * Work is split into jobs of up to 64 wavelengths and as many realisations as
 * the workspace budget allows (ps_set_workspace_budget).  In FP32 from
 * N = 2048 up the jobs are pipelined (work that fits one job is split into
 * two, by realisations or else by wavelengths): the transpose between the
 * two 1-D passes of one job runs inside the launches of the neighbouring
 * jobs' passes, which takes twice the workspace of the plain loop and gives
 * the same result bit for bit for the same job split (environment
 * SCINT_PIPELINE=0 turns it off).  The pipelined first passes give each row
 * two workgroups, each taking half of the job's wavelengths (same result;
 * SCINT_ITER_SPLIT=1 keeps one).
 */
int illumination_polychromatic(int N, double delta, double z, const void *phi_ref,
                               double lambda_ref, const double *lambdas,
                               const double *weights, int n_lambda, int n_real, int dtype,
                               void *I_out, void *hip_stream);

/*
 * source_smear -- extended source (Sect. 3.2.3, Eq. iprh): circular
 * convolution of each pattern with a uniform disk of projected radius R_s,
 *   I_ext[m] = sum_d P[d] I[m - d],  P[d] = 1/n_R if |d| <= R_s/delta else 0,
 * |d| the minimum-image distance between pixel centres on the periodic grid,
 * n_R the number of such pixels (so R_s < delta gives the identity and the
 * mean is preserved).  Computed by FFT multiplication.
 *   I_in      device [n_real][N][N] real
 *   radii     host array of n_r radii R_s >= 0 (length unit of delta), n_r <= 64
 *   I_out     device [n_real][n_r][N][N] real; may equal I_in only if n_r == 1
 */
int source_smear(int N, double delta, const void *I_in, const double *radii, int n_r,
                 int n_real, int dtype, void *I_out, void *hip_stream);

/*
 * fresnel_propagate_vjp -- adjoint of fresnel_propagate (vector-Jacobian
 * product) for a loss L(I) whose gradient dL/dI is grad_I:
 *   g_A = 2 grad_I A;  g_U = N^-2 IDFT[ conj(H) DFT[g_A] ];
 *   dL/dphi = s Im(g_U conj(U)).
 * The forward field A is taken from the checkpoint `field` when given (four
 * 1-D FFT passes per point), else recomputed from phi (eight).
 *   phi, grad_I        device [n][N][N] real
 *   field              optional device [n][N][N] complex, the checkpoint
 *                      written by fresnel_propagate_field or
 *                      ps_screen_fresnel for the same phi, lambda, z and s;
 *                      NULL to recompute
 *   grad_phi_out       device [n][N][N] real; must not overlap phi, grad_I or field
 *   phi_dot_grad_out   optional host array of n doubles: sum_m phi dL/dphi
 *                      per screen (FP64), from which
 *                      dL/dlog R_diff = ((2 - beta)/2) phi_dot_grad, since the
 *                      screen scales as R_diff^((2-beta)/2) for fixed noise.
 */
int fresnel_propagate_vjp(int N, double delta, double lambda, double z, const void *phi,
                          double phase_scale, const void *grad_I, const void *field, int n,
                          int dtype, void *grad_phi_out, double *phi_dot_grad_out,
                          void *hip_stream);

/*
 * fresnel_aperture -- the paper's own numerics for a bounded screen
 * (Sect. 3.2, Eqs. intens and Gxy, with the screen regularisation of
 * Sect. 3.2.1): one 2-D DFT of the windowed, chirped screen read out on the
 * observer grid.  For each of the n screens phi (radians, scaled by s):
 *   G[y][x] = SF(x) SF(y) exp(i (s phi[y][x] + ((x - N/2)^2 + (y - N/2)^2) / (2 rho^2))),
 *   I[my][mx] = |DFT[G](ky, kx)|^2 / (2 pi rho^2)^2,  k = m - N/2 (mod N),
 * with rho = R_F / delta = sqrt(lambda z / 2 pi) / delta.  Screen pixel j
 * has the coordinate (j - N/2) delta; observer pixel m has the coordinate
 * (m - N/2) lambda z / (N delta): the observer pixel is lambda z / (N delta)
 * and observer pixel N/2 faces screen pixel N/2.  SF is the raised-sine
 * window of the paper over a margin L_m = margin_rf R_F at each border
 * (the paper uses margin_rf = 10; 0 = no window), evaluated at the pixel
 * centres, (j + 1/2) delta from the border.  The 2-D prefactor 1/(2 pi R_F^2)
 * is applied to the field, so an unbounded uniform screen gives I = 1.  At
 * N delta^2 = lambda z (Sect. 3.4) and margin_rf = 0 the result equals
 * fresnel_propagate pixel by pixel.
 *   phi        device [n][N][N] real (input, not modified)
 *   margin_rf  L_m / R_F >= 0, with 2 L_m <= N delta (else PS_E_PARAM)
 *   I_out      device [n][N][N] real; must not overlap phi (PS_E_ALIAS)
 * N delta^2 > lambda z is rejected (PS_E_PARAM): the chirp would be sampled
 * below two points per period at the screen border (the aliasing criterion
 * of Sect. 3.2.2) and would fold light from there onto the observer grid.
 */
int fresnel_aperture(int N, double delta, double lambda, double z, const void *phi,
                     double phase_scale, double margin_rf, int n, int dtype, void *I_out,
                     void *hip_stream);

/*
 * ps_aperture_geometry -- the observer grid of fresnel_aperture and its
 * fiducial zone (Sect. 3.2.1): observer_pixel = lambda z / (N delta) (length
 * unit of delta), and fiducial_margin = the number of observer pixels to
 * exclude at each border: the dark rim outside the screen's shadow,
 * N (1 - delta / observer_pixel) / 2 (zero at N delta^2 = lambda z), plus
 * (R_ref / 2 + r_s) / observer_pixel, rounded up; R_ref = lambda z / r_diff
 * (= 2 pi R_F^2 / R_diff, the refractive scale) and r_s the projected source
 * radius (0 for a point source; the extended-source zone adds R_s).  Host
 * arithmetic only.  A warning is set when the zone is empty
 * (2 fiducial_margin >= N); fiducial_margin is capped at N.
 */
int ps_aperture_geometry(int N, double delta, double lambda, double z, double r_diff,
                         double r_s, double *observer_pixel, int *fiducial_margin);

/*
 * ps_modulation_index -- m = sigma_I / mean(I) per pattern (Sect. 4),
 * population sigma over all N^2 pixels, FP64 accumulation in a fixed order
 * (bitwise reproducible).
 *   I       device [n][N][N] real
 *   m_out   host array of n doubles;  mean_out optional host array of n doubles
 */
int ps_modulation_index(int N, const void *I, int n, int dtype, double *m_out,
                        double *mean_out, void *hip_stream);

/*
 * ps_modulation_index_region -- m and the mean as ps_modulation_index, over
 * the w x h rectangle whose first pixel is (x0, y0) in each pattern: the
 * statistics inside a fiducial zone (Sect. 3.2.1, Sect. 4).  The rectangle
 * must be non-empty and inside the image (PS_E_PARAM).
 *   I       device [n][N][N] real
 *   m_out   host array of n doubles;  mean_out optional host array of n doubles
 */
int ps_modulation_index_region(int N, const void *I, int n, int x0, int y0, int w, int h,
                               int dtype, double *m_out, double *mean_out, void *hip_stream);

/*
 * ps_structure_function -- the check of a generated screen by its recomputed
 * structure function (Sect. 3.1.1, Eq. crec).  For each of the n screens:
 *   S_rec(q_b) = <|F_phi|^2>_ring / (L_x L_y) = delta^2 <|DFT phi|^2>_ring / N^2,
 * averaged over the Fourier pixels whose signed frequency |k'| (components
 * in [-N/2, N/2)) rounds to b, q_b = b / (N delta), b = 0 .. N/2;
 *   xi(r) = sum_{b=1}^{N/2} 2 pi q_b S_rec(q_b) J0(2 pi q_b r) dq, dq = 1/(N delta)
 * (the paper's limits q_min = 1/(N delta), q_max = 1/(2 delta)),
 *   D_rec(r) = 2 (xi(0) - xi(r)),
 * and R_diff^rec, the r with D_rec(r) = 1 (bisection between 1e-3 and N/2
 * pixels; NaN and a warning if not bracketed).  FP64 ring sums and Hankel
 * sums (J0 by its power series below 14 and Hankel's expansion above).
 *   phi        device [n][N][N] real (radians; input, not modified)
 *   radii      host array of n_r radii >= 0 (length unit of delta), n_r >= 0
 *   S_out      optional host [n][N/2 + 1]: S_rec in (length unit)^2 rad^2
 *   D_out      host [n][n_r] (required when n_r > 0): D_rec at the radii
 *   rdiff_out  optional host [n]: R_diff^rec (length unit of delta)
 * Synchronises with the stream.
 */
int ps_structure_function(int N, double delta, const void *phi, int n, const double *radii,
                          int n_r, int dtype, double *S_out, double *D_out, double *rdiff_out,
                          void *hip_stream);

/*
 * ps_light_curves -- light curves as a telescope sweeping the pattern sees
 * them (Sect. 3.3): each pattern is sampled along straight lines at a
 * constant speed.  Pixel (ix, iy) sits at the point (ix, iy) in pixel units;
 * sample k of line l lies at (x0 + k dx, y0 + k dy) with
 * lines[4 l .. 4 l + 3] = (x0, y0, dx, dy), wrapped onto the periodic
 * pattern.  mode 0 takes the nearest pixel (ties round up), mode 1
 * interpolates bilinearly between the four surrounding pixels (FP64
 * weights).  (dx, dy) is the relative transverse velocity times the sampling
 * interval, in pixels.
 *   I           device [n][N][N] real
 *   lines       host array of 4 n_lines finite doubles (n_lines >= 1)
 *   curves_out  device [n][n_lines][n_samples] real; must not overlap I
 *   m_out       optional host array of n n_lines doubles: sigma/mean of each
 *               curve (population sigma, FP64, Sect. 4); the call then
 *               synchronises with the stream
 */
int ps_light_curves(int N, const void *I, int n, const double *lines, int n_lines,
                    int n_samples, int mode, int dtype, void *curves_out, double *m_out,
                    void *hip_stream);

/*
 * ps_m_theory -- expected modulation index of an extended source in the
 * strong, quenched regime for Kolmogorov turbulence (Sect. 4.1, Eq. xparam,
 * after Narayan 1992): m = (R_diff/R_F)^(1/3) (R_ref / (2 pi R_s))^(7/6),
 * R_ref = 2 pi R_F^2 / R_diff, with R_s the projected source radius (all in
 * one length unit, > 0).  Host arithmetic only; a warning is set outside the
 * regime R_s/R_F > R_F/R_diff > 1 where the relation holds.
 */
int ps_m_theory(double r_diff, double r_f, double r_s, double *m_out);

/*
 * ps_l2_loss -- L = sum_m (I - I_target)^2 per pattern and its gradient
 * dL/dI = 2 (I - I_target).
 *   grad_out   optional device [n][N][N] real
 *   loss_out   optional host array of n doubles (FP64 accumulation)
 */
int ps_l2_loss(int N, const void *I, const void *I_target, int n, int dtype,
               void *grad_out, double *loss_out, void *hip_stream);

/*
 * FFT plan variants and the plan tuner.  The large FP32 sizes (2048, 4096,
 * 8192, 10000, 16384) have several compiled Stockham plans (radix orders and
 * elements per thread).  The first FP32 call of such a size on a device times
 * each plan on a propagation row pass of 32 wavelength iterations over
 * scratch data (hipMalloc of about 200 MB, a private stream, synchronised)
 * and keeps the fastest; it keeps
 * plan 0 unless another is faster by more than 3%.  Different plans round
 * differently (within FP32 rounding), so pin a plan for bitwise-reproducible
 * results across processes: environment SCINT_PLAN_VARIANT=<v> or
 * ps_set_plan_variant.  FP64 always uses plan 0.
 *   ps_num_plan_variants  number of plans of N for dtype (0 if unsupported)
 *   ps_plan_variant       plan in use (tuning it now if not yet chosen);
 *                         ms_out, optional host array of
 *                         ps_num_plan_variants(N, dtype) floats, receives the
 *                         tuner's times (-1 where not timed)
 *   ps_set_plan_variant   pins plan `variant`, or -1 to return to tuning
 *   ps_tune_plans         chooses the plan of N (tuning it if needed) and
 *                         builds its twiddle table on the current device,
 *                         synchronously on the null stream, so that no later
 *                         call of size N tunes or builds tables: call it
 *                         before capturing a graph that uses size N
 */
int ps_num_plan_variants(int N, int dtype);
int ps_plan_variant(int N, int dtype, int *variant_out, float *ms_out);
int ps_set_plan_variant(int N, int dtype, int variant);
int ps_tune_plans(int N, int dtype);

/*
 * ps_set_workspace_budget -- upper bound, in bytes, on the workspace that
 * later calls on the current device plan for; whole-batch work is split into
 * chunks that fit it (the chunking can change FP32 rounding of sums over
 * wavelength chunks).  0 restores the default: a quarter of the free device
 * memory at the next call, at most 32 GiB.  Values below 64 MiB are rejected
 * (PS_E_PARAM).  A single grid that needs more than the budget still gets
 * the memory it needs.
 */
int ps_set_workspace_budget(size_t bytes);

/*
 * ps_plan_polychromatic -- how illumination_polychromatic would split a call
 * of these sizes under a workspace budget of budget_bytes (host arithmetic
 * only: no device call, callable without a GPU).  Any output pointer may be
 * NULL.
 *   pipelined        1 if the jobs are pipelined (transposes inside the
 *                    passes), 0 for the plain loop
 *   n_jobs           number of jobs (pipelined) or chunks (plain loop)
 *   lambdas_per_job  wavelengths per job (<= 64)
 *   real_per_job     realisations per job
 *   workspace_bytes  workspace the call asks for
 * Errors as for illumination_polychromatic's sizes; budget_bytes must be > 0.
 */
int ps_plan_polychromatic(int N, int n_real, int n_lambda, int dtype, size_t budget_bytes, int *pipelined,
                          int *n_jobs, int *lambdas_per_job, int *real_per_job, size_t *workspace_bytes);

/*
 * Kernel timing (instrumentation).  While enabled, every kernel the library
 * launches is bracketed by two HIP events recorded on the stream it runs on,
 * and per kernel name the library accumulates the event-measured duration,
 * the launch count, and per launch:
 *   bytes           algorithmic bytes: each array the method reads or writes
 *                   in that pass, once (complex elements count 2 reals; an
 *                   array re-read on every loop iteration at the same
 *                   address, such as the phase screen re-read for each
 *                   wavelength, once; the 1-D chirp tables not at all; the
 *                   transposes between the two 1-D passes of a 2-D transform
 *                   zero, since the method's one exchange per transform is
 *                   the first pass's write and the second pass's read);
 *   schedule_bytes  the operand bytes of the launch as scheduled: every
 *                   access of the kernel's operations, loop re-reads
 *                   included, plus 16 bytes per element of the transposes a
 *                   row pass carries or 2 x element size per element of a
 *                   transpose kernel;
 *   flops           algorithmic floating-point operations (5 N log2 N per
 *                   length-N complex DFT, 6 per complex multiply, 2 per
 *                   real-by-complex multiply, 5 per weighted |A|^2
 *                   accumulation; sine, cosine and the noise generator not
 *                   counted).
 *   ps_timing_enable(1) clears the totals and starts recording; (0) stops.
 *   ps_timing_count() waits for the recorded events and returns the number
 *   of distinct kernel names; ps_timing_entry(i, ...) returns the i-th
 *   (name copied into name_buf, NUL-terminated, at most buf_len bytes).
 */
int ps_timing_enable(int on);
int ps_timing_count(void);
int ps_timing_entry(int i, char *name_buf, int buf_len, double *total_ms, long long *launches,
                    double *bytes, double *schedule_bytes, double *flops);

/* Message for the last non-OK status of this thread ("" if none). */
const char *ps_last_error(void);
/* Message for the last warning of this thread ("" if none); cleared by every call. */
const char *ps_last_warning(void);
/* Free every cached table and workspace on every device.  Not to be called
 * while work that uses them is in flight. */
int ps_release_cache(void);
/* Library version (major * 10000 + minor * 100 + patch). */
int ps_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SCINT_H */

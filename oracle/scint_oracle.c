/*
 * scint_oracle.c -- plain FP64 CPU reference for the phase-screen + Fresnel
 * propagation method of Habibi, Moniez, Ansari & Rahvar, "Simulation of
 * optical interstellar scintillation" (A&A 2013, arXiv:1301.0514).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code, header, table or
 * constant generator with the GPU library: it has its own Philox generator,
 * its own mixed-radix DFT and its own argument reductions.
 *
 * Everything is in pixel units unless stated otherwise (pixel side = 1),
 * double precision, row-major [y][x] arrays with x fastest.
 *
 * Status of the pins (the tests under tests/ hold them):
 *   Philox4x32-10 / 4x64-10  : known-answer vectors and numpy's Philox
 *   own DFT                  : numpy.fft and direct O(n^2) sums
 *   spectrum normalisation   : continuous D(R_diff)=1 and closed forms of f(beta)
 *   screen                   : discrete expectation of D(r) and the paper's
 *                              540 km figure (Sect. 3.1.1)
 *   propagation              : direct O(N^4) Fresnel sum at N = 2 pi rho^2,
 *                              uniform screen, phase ramp, Parseval, phase
 *                              grating (Jacobi-Anger), Talbot, weak regime
 *   polychromatic, smear     : reductions, direct convolution, invariants
 *   adjoint                  : dot-product test and finite differences
 *   aperture mode            : direct O(N^4) Fresnel sum with the window,
 *                              the periodic form at N = 2 pi rho^2 without
 *                              it, the window's closed-form values, Parseval,
 *                              and the paper's < 1 % flatness for a uniform
 *                              screen
 *   structure-function check : a single Fourier mode against its closed form
 *                              through the ring average and J0, the
 *                              theoretical spectrum's R_diff^rec against a
 *                              quadrature of the continuous integral, the
 *                              paper's 540 km
 *   light curves, m theory   : axis-aligned lines equal pattern rows and
 *                              columns, bilinear sampling is exact on linear
 *                              fields and equals the pixels at integer points;
 *                              the paper's numeric form of Eq. xparam
 *   Propagation at a general rho (N != 2 pi rho^2) beyond the closed forms
 *   above is "parity unpinned" as physics; its algebra is pinned by the DFT.
 */
#define _DEFAULT_SOURCE /* j0 (Bessel function of the first kind) from libm */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define ORACLE_PI 3.14159265358979323846264338327950288

/* ------------------------------------------------------------------------ */
/* Counter-based Philox generators (Salmon, Moraes, Dror & Shaw, SC'11).    */
/* One round multiplies words 0 and 2 by the round multipliers, takes the    */
/* high and low halves of the double-width products, xors the high halves    */
/* with the other two words and the key, and permutes; the key is bumped by  */
/* the Weyl constants between rounds.  Ten rounds.                           */
/* ------------------------------------------------------------------------ */

void oracle_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2],
                          uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        if (round < 9) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

void oracle_philox4x64_10(const uint64_t ctr_in[4], const uint64_t key_in[2],
                          uint64_t out[4])
{
    uint64_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        unsigned __int128 p0 = (unsigned __int128)0xD2E7470EE14C6C93ull * c0;
        unsigned __int128 p1 = (unsigned __int128)0xCA5A826395121157ull * c2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t n0 = hi1 ^ c1 ^ k0;
        uint64_t n1 = lo1;
        uint64_t n2 = hi0 ^ c3 ^ k1;
        uint64_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        if (round < 9) {
            k0 += 0x9E3779B97F4A7C15ull;
            k1 += 0xBB67AE8584CAA73Bull;
        }
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Two uniforms in (0,1) from the four 32-bit words: each pair forms a 64-bit
 * integer, its top 53 bits plus one half is scaled by 2^-53 (exact in FP64). */
static void uniforms_from_words(const uint32_t w[4], double *u1, double *u2)
{
    uint64_t a = ((uint64_t)w[0] << 32) | (uint64_t)w[1];
    uint64_t b = ((uint64_t)w[2] << 32) | (uint64_t)w[3];
    *u1 = ((double)(a >> 11) + 0.5) * 0x1.0p-53;
    *u2 = ((double)(b >> 11) + 0.5) * 0x1.0p-53;
}

/* Complex standard normal g = g_re + i g_im (each part of unit variance) for
 * the spectral pixel (kx, ky) of realisation r (Sect. 3.1: one random complex
 * number per Fourier pixel; Box-Muller from the two uniforms). */
static void normal_pair(uint64_t seed, uint32_t r, int kx, int ky,
                        double *g_re, double *g_im)
{
    uint32_t ctr[4] = {(uint32_t)kx, (uint32_t)ky, r, 0u};
    uint32_t key[2] = {(uint32_t)(seed & 0xFFFFFFFFull), (uint32_t)(seed >> 32)};
    uint32_t w[4];
    oracle_philox4x32_10(ctr, key, w);
    double u1, u2;
    uniforms_from_words(w, &u1, &u2);
    double rad = sqrt(-2.0 * log(u1));
    *g_re = rad * cos(2.0 * ORACLE_PI * u2);
    *g_im = rad * sin(2.0 * ORACLE_PI * u2);
}

/* g[ky][kx][2] for one realisation. */
void oracle_normals(int N, uint64_t seed, uint32_t r, double *g)
{
#pragma omp parallel for schedule(static)
    for (int ky = 0; ky < N; ++ky)
        for (int kx = 0; kx < N; ++kx) {
            double *o = g + 2 * ((size_t)ky * N + kx);
            normal_pair(seed, r, kx, ky, &o[0], &o[1]);
        }
}

/* ------------------------------------------------------------------------ */
/* Own DFT: recursive decimation in time by the smallest prime factor.      */
/* out[k] = sum_j in[j] exp(sign * 2 pi i j k / n), unnormalised.            */
/* ------------------------------------------------------------------------ */

static int smallest_factor(int n)
{
    if (n % 2 == 0) return 2;
    for (int p = 3; p * p <= n; p += 2)
        if (n % p == 0) return p;
    return n;
}

/* root[m] = exp(sign 2 pi i m / root_n), m in [0, root_n). */
static cplx *make_roots(int root_n, int sign)
{
    cplx *root = (cplx *)malloc(sizeof(cplx) * (size_t)root_n);
    for (int m = 0; m < root_n; ++m) {
        double ang = 2.0 * ORACLE_PI * (double)m / (double)root_n;
        root[m] = cos(ang) + (double)sign * sin(ang) * I;
    }
    return root;
}

/* DFT of length n of in[0], in[stride], ..., written contiguously to out.
 * 'root' holds the root_n-th roots; n divides root_n. */
static void dft_rec(int n, const cplx *in, size_t stride, cplx *out,
                    const cplx *root, int root_n)
{
    if (n == 1) { out[0] = in[0]; return; }
    int p = smallest_factor(n);
    int m = n / p;
    /* sub-transforms of the p decimated sequences */
    for (int q = 0; q < p; ++q)
        dft_rec(m, in + (size_t)q * stride, stride * (size_t)p, out + (size_t)q * m,
                root, root_n);
    /* combine: X[k1 + m k2] = sum_q W_n^{q (k1 + m k2)} Y_q[k1] */
    int step = root_n / n; /* W_n^e = root[e * step] */
    cplx ybuf[64], xbuf[64];
    cplx *yv = p <= 64 ? ybuf : (cplx *)malloc(sizeof(cplx) * (size_t)p);
    cplx *xv = p <= 64 ? xbuf : (cplx *)malloc(sizeof(cplx) * (size_t)p);
    for (int k1 = 0; k1 < m; ++k1) {
        for (int q = 0; q < p; ++q) yv[q] = out[(size_t)q * m + k1];
        for (int k2 = 0; k2 < p; ++k2) {
            long k = (long)k1 + (long)m * k2;
            cplx acc = 0.0;
            for (int q = 0; q < p; ++q) {
                long e = ((long)q * k) % n;
                acc += root[e * step] * yv[q];
            }
            xv[k2] = acc;
        }
        for (int k2 = 0; k2 < p; ++k2) out[(size_t)k2 * m + k1] = xv[k2];
    }
    if (xv != xbuf) free(xv);
    if (yv != ybuf) free(yv);
}

/* 1-D DFT, unnormalised; sign = -1 forward, +1 backward. */
void oracle_dft1(int n, const double *in_ri, double *out_ri, int sign)
{
    const cplx *in = (const cplx *)in_ri;
    cplx *out = (cplx *)out_ri;
    cplx *root = make_roots(n, sign);
    dft_rec(n, in, 1, out, root, n);
    free(root);
}

/* In-place unnormalised 2-D DFT of an N x N complex array. */
static void dft2_inplace(int N, cplx *a, int sign)
{
    cplx *root = make_roots(N, sign);
#pragma omp parallel
    {
        cplx *buf_in = (cplx *)malloc(sizeof(cplx) * (size_t)N);
        cplx *buf_out = (cplx *)malloc(sizeof(cplx) * (size_t)N);
        /* rows (transform along x) */
#pragma omp for schedule(static)
        for (int y = 0; y < N; ++y) {
            cplx *row = a + (size_t)y * N;
            memcpy(buf_in, row, sizeof(cplx) * (size_t)N);
            dft_rec(N, buf_in, 1, row, root, N);
        }
        /* columns (transform along y) */
#pragma omp for schedule(static)
        for (int x = 0; x < N; ++x) {
            for (int y = 0; y < N; ++y) buf_in[y] = a[(size_t)y * N + x];
            dft_rec(N, buf_in, 1, buf_out, root, N);
            for (int y = 0; y < N; ++y) a[(size_t)y * N + x] = buf_out[y];
        }
        free(buf_in);
        free(buf_out);
    }
    free(root);
}

void oracle_dft2(int N, double *a_ri, int sign)
{
    dft2_inplace(N, (cplx *)a_ri, sign);
}

/* ------------------------------------------------------------------------ */
/* Phase spectrum (Sect. 2, Eq. spectre):                                    */
/*   S(q) = R^2 / (2 (2 pi)^(beta-1) f(beta)) (R q)^(-beta),                 */
/*   f(beta) = 2^(-beta) beta Gamma(-beta/2) / Gamma(beta/2).                */
/* ------------------------------------------------------------------------ */

double oracle_f_beta(double beta)
{
    return pow(2.0, -beta) * beta * tgamma(-beta / 2.0) / tgamma(beta / 2.0);
}

double oracle_spectrum(double q, double R, double beta)
{
    double f = oracle_f_beta(beta);
    return R * R / (2.0 * pow(2.0 * ORACLE_PI, beta - 1.0) * f) * pow(R * q, -beta);
}

static int signed_freq(int k, int N) { return k < N / 2 ? k : k - N; }

/* Filtered spectrum of one realisation (Sect. 3.1, Eq. densite):
 * c[ky][kx] = F_phi / (L_x L_y) with F_phi = (f_Re + i f_Im)/sqrt(2) and
 * Var f = L_x L_y S(q) (the "width" read as the variance); L = N pixels, so
 * c = sqrt(S(q)/N^2) (g_re + i g_im)/sqrt(2).  The DC pixel is zero (the
 * lowest sampled frequency is 1/(N pixel), Sect. 3.1.1). */
void oracle_spectrum_coeffs(int N, double R, double beta, uint64_t seed, uint32_t r,
                            double *c_ri)
{
    cplx *c = (cplx *)c_ri;
#pragma omp parallel for schedule(static)
    for (int ky = 0; ky < N; ++ky)
        for (int kx = 0; kx < N; ++kx) {
            size_t idx = (size_t)ky * N + kx;
            if (kx == 0 && ky == 0) { c[idx] = 0.0; continue; }
            double fx = signed_freq(kx, N), fy = signed_freq(ky, N);
            double q = sqrt(fx * fx + fy * fy) / (double)N;
            double S = oracle_spectrum(q, R, beta);
            double g_re, g_im;
            normal_pair(seed, r, kx, ky, &g_re, &g_im);
            double amp = sqrt(S) / (double)N;
            c[idx] = amp * (g_re + g_im * I) / sqrt(2.0);
        }
}

/* Phase screen (Sect. 3.1): inverse Fourier transform of the random phase
 * spectrum, phi = sqrt(2) Re(sum_k c[k] exp(+2 pi i k.m/N)). */
void oracle_screen(int N, double R, double beta, uint64_t seed, uint32_t r, double *phi)
{
    cplx *c = (cplx *)malloc(sizeof(cplx) * (size_t)N * N);
    oracle_spectrum_coeffs(N, R, beta, seed, r, (double *)c);
    dft2_inplace(N, c, +1);
    size_t NN = (size_t)N * N;
#pragma omp parallel for schedule(static)
    for (size_t i = 0; i < NN; ++i) phi[i] = sqrt(2.0) * creal(c[i]);
    free(c);
}

/* ------------------------------------------------------------------------ */
/* Fresnel propagation on the periodic screen (Sect. 2, Eq. hxy).           */
/*   U = exp(i s phi); A = N^-2 IDFT[ H(k) DFT[U] ];  I = |A|^2             */
/*   H(k) = H1(kx') H1(ky'),  H1(k') = exp(-i 2 pi^2 rho^2 k'^2 / N^2),      */
/* the transfer function of the paper's kernel exp(+i |x0-x1|^2 / 2 R_F^2)  */
/* normalised so that a uniform screen gives I = 1.                         */
/* Phase arguments are reduced modulo 2 pi in FP64 before cos/sin.          */
/* ------------------------------------------------------------------------ */

static cplx expi_turns(double t) /* exp(2 pi i t) with t reduced to [-1/2, 1/2] */
{
    double f = t - nearbyint(t);
    double a = 2.0 * ORACLE_PI * f;
    return cos(a) + sin(a) * I;
}

static cplx chirp1(int k, int N, double rho)
{
    /* theta = 2 pi^2 rho^2 k'^2 / N^2 = 2 pi * (pi rho^2 k'^2 / N^2) */
    double kk = (double)signed_freq(k, N);
    double turns = ORACLE_PI * rho * rho / ((double)N * (double)N) * (kk * kk);
    return conj(expi_turns(turns));
}

double oracle_fresnel_radius_px(double delta, double lambda, double z)
{
    /* R_F = sqrt(lambda z / 2 pi) (Sect. 2, Eq. Rfresnel), in pixels */
    return sqrt(lambda * z / (2.0 * ORACLE_PI)) / delta;
}

/* Field A after propagation, for phase scale s and Fresnel radius rho (px).
 * conj_chirp != 0 applies conj(H) (the adjoint's transfer function). */
static void propagate_field(int N, double rho, cplx *a, int conj_chirp)
{
    dft2_inplace(N, a, -1);
    cplx *h = (cplx *)malloc(sizeof(cplx) * (size_t)N);
    for (int k = 0; k < N; ++k) h[k] = conj_chirp ? conj(chirp1(k, N, rho)) : chirp1(k, N, rho);
    double norm = 1.0 / ((double)N * (double)N);
#pragma omp parallel for schedule(static)
    for (int ky = 0; ky < N; ++ky)
        for (int kx = 0; kx < N; ++kx)
            a[(size_t)ky * N + kx] *= h[kx] * h[ky] * norm;
    free(h);
    dft2_inplace(N, a, +1);
}

void oracle_propagate(int N, double rho, double s, const double *phi, double *I_out,
                      double *A_ri /* optional */)
{
    size_t NN = (size_t)N * N;
    cplx *a = (cplx *)malloc(sizeof(cplx) * NN);
#pragma omp parallel for schedule(static)
    for (size_t i = 0; i < NN; ++i) a[i] = expi_turns(s * phi[i] / (2.0 * ORACLE_PI));
    propagate_field(N, rho, a, 0);
#pragma omp parallel for schedule(static)
    for (size_t i = 0; i < NN; ++i) I_out[i] = creal(a[i]) * creal(a[i]) + cimag(a[i]) * cimag(a[i]);
    if (A_ri) memcpy(A_ri, a, sizeof(cplx) * NN);
    free(a);
}

/* One-dimensional counterpart along a line of N pixels: a = N^-1 IDFT[H1  */
/* DFT exp(i s phi)].  For a separable screen phi(x, y) = f(x) + g(y) the     */
/* 2-D field of oracle_propagate is the outer product a_g(y) a_f(x), since   */
/* both the DFT and H = H1(kx) H1(ky) factorise.                             */
void oracle_propagate_line(int N, double rho, double s, const double *phi, double *a_ri)
{
    cplx *a = (cplx *)malloc(sizeof(cplx) * (size_t)N);
    cplx *b = (cplx *)malloc(sizeof(cplx) * (size_t)N);
    for (int x = 0; x < N; ++x) a[x] = expi_turns(s * phi[x] / (2.0 * ORACLE_PI));
    cplx *fwd = make_roots(N, -1), *inv = make_roots(N, +1);
    dft_rec(N, a, 1, b, fwd, N);
    for (int k = 0; k < N; ++k) b[k] *= chirp1(k, N, rho) / (double)N;
    dft_rec(N, b, 1, a, inv, N);
    free(fwd);
    free(inv);
    memcpy(a_ri, a, sizeof(cplx) * (size_t)N);
    free(b);
    free(a);
}

/* Same, physical arguments (any one length unit for delta, lambda, z). */
void oracle_fresnel(int N, double delta, double lambda, double z, double s,
                    const double *phi, double *I_out)
{
    oracle_propagate(N, oracle_fresnel_radius_px(delta, lambda, z), s, phi, I_out, NULL);
}

/* Direct discretisation of Eq. hxy on the finite N x N screen (O(N^4)):
 *   h[m] = | 1/(2 pi rho^2) sum_{m'} exp(i phi[m']) exp(i |m - m'|^2 / (2 rho^2)) |^2
 * with pixel-centre integer coordinates; no wrap-around. */
void oracle_fresnel_direct(int N, double rho, const double *phi, double *I_out)
{
    double inv2r2 = 1.0 / (2.0 * rho * rho);
    double pref = 1.0 / (2.0 * ORACLE_PI * rho * rho);
#pragma omp parallel for schedule(static)
    for (int y0 = 0; y0 < N; ++y0)
        for (int x0 = 0; x0 < N; ++x0) {
            cplx acc = 0.0;
            for (int y1 = 0; y1 < N; ++y1)
                for (int x1 = 0; x1 < N; ++x1) {
                    double dx = x0 - x1, dy = y0 - y1;
                    double arg = phi[(size_t)y1 * N + x1] + (dx * dx + dy * dy) * inv2r2;
                    acc += cos(arg) + sin(arg) * I;
                }
            acc *= pref;
            I_out[(size_t)y0 * N + x0] = creal(acc) * creal(acc) + cimag(acc) * cimag(acc);
        }
}

/* The paper's own numerics without the smoothing window (Sect. 3.2,
 * Eqs. intens and Gxy): h = |FT[G]|^2 at f = x0 / (2 pi R_F^2), with
 * G = exp(i (phi + r1^2 / 2 R_F^2)) and the observer pixel equal to the
 * screen pixel, which holds when N = 2 pi rho^2 (Sect. 3.4).  The prefactor
 * 1/(2 pi R_F^2) is taken inside the modulus, as in Eq. hxy. */
void oracle_fresnel_onefft(int N, double rho, const double *phi, double *I_out)
{
    size_t NN = (size_t)N * N;
    cplx *g = (cplx *)malloc(sizeof(cplx) * NN);
    double inv2r2 = 1.0 / (2.0 * rho * rho);
    for (int y = 0; y < N; ++y)
        for (int x = 0; x < N; ++x) {
            double arg = phi[(size_t)y * N + x] + ((double)x * x + (double)y * y) * inv2r2;
            g[(size_t)y * N + x] = cos(arg) + sin(arg) * I;
        }
    dft2_inplace(N, g, -1);
    double pref = 1.0 / (2.0 * ORACLE_PI * rho * rho);
    for (size_t i = 0; i < NN; ++i) {
        cplx v = g[i] * pref;
        I_out[i] = creal(v) * creal(v) + cimag(v) * cimag(v);
    }
    free(g);
}

/* ------------------------------------------------------------------------ */
/* Aperture mode: the paper's own numerics with the smoothing window        */
/* (Sect. 3.2, Eqs. intens and Gxy; screen regularisation, Sect. 3.2.1).    */
/*                                                                           */
/* Screen pixel j has the integer coordinate x1 = j - N/2 (pixel units), its */
/* centre lies (j + 1/2) pixels from the screen's left border.  The window   */
/* SF is the paper's raised sine over a margin of L_m = margin_rf * rho      */
/* pixels at each border, applied as SF(x1) SF(y1).  The observer pixel is   */
/* 2 pi rho^2 / N screen pixels and observer pixel m has the coordinate      */
/* x0 = (m - N/2) 2 pi rho^2 / N.  The 2-D Fresnel prefactor 1/(2 pi R_F^2)  */
/* is applied to the field (a uniform, unbounded screen gives I = 1).        */
/* ------------------------------------------------------------------------ */

/* SF at the N pixel centres for a margin of Lm pixels (Lm = 0: no window). */
void oracle_sf_window(int N, double Lm, double *sf)
{
    for (int j = 0; j < N; ++j) {
        double x = j + 0.5, L = (double)N;
        double v;
        if (Lm <= 0.0)
            v = 1.0;
        else if (x <= Lm)
            v = 0.5 * (1.0 + sin(ORACLE_PI * x / Lm - 0.5 * ORACLE_PI));
        else if (x < L - Lm)
            v = 1.0;
        else if (x <= L)
            v = 0.5 * (1.0 + sin(ORACLE_PI * (x - L + Lm) / Lm + 0.5 * ORACLE_PI));
        else
            v = 0.0;
        sf[j] = v;
    }
}

/* h = |FT[SF SF G]|^2 / (2 pi rho^2)^2 on the observer grid: one 2-D DFT of */
/* the windowed G = exp(i (s phi + |x1|^2 / 2 rho^2)), then the frequency    */
/* index k = m - N/2 (mod N) is read out at observer pixel m.               */
void oracle_fresnel_aperture(int N, double rho, double s, double margin_rf, const double *phi,
                             double *I_out)
{
    size_t NN = (size_t)N * N;
    cplx *g = (cplx *)malloc(sizeof(cplx) * NN);
    double *sf = (double *)malloc(sizeof(double) * N);
    oracle_sf_window(N, margin_rf * rho, sf);
    double inv2r2 = 1.0 / (2.0 * rho * rho);
    for (int y = 0; y < N; ++y)
        for (int x = 0; x < N; ++x) {
            double x1 = x - N / 2, y1 = y - N / 2;
            double arg = s * phi[(size_t)y * N + x] + (x1 * x1 + y1 * y1) * inv2r2;
            g[(size_t)y * N + x] = sf[x] * sf[y] * (cos(arg) + sin(arg) * I);
        }
    dft2_inplace(N, g, -1);
    double pref = 1.0 / (2.0 * ORACLE_PI * rho * rho);
    for (int m = 0; m < N; ++m)
        for (int mx = 0; mx < N; ++mx) {
            int ky = (m + N / 2) % N, kx = (mx + N / 2) % N;
            cplx v = g[(size_t)ky * N + kx] * pref;
            I_out[(size_t)m * N + mx] = creal(v) * creal(v) + cimag(v) * cimag(v);
        }
    free(sf);
    free(g);
}

/* The same intensity straight from the Fresnel sum (Eq. hxy) at the        */
/* observer points, O(N^4): h(x0) = |(2 pi rho^2)^-1 sum SF SF e^{i s phi}   */
/* e^{i |x0 - x1|^2 / 2 rho^2}|^2.                                          */
void oracle_fresnel_aperture_direct(int N, double rho, double s, double margin_rf,
                                    const double *phi, double *I_out)
{
    double *sf = (double *)malloc(sizeof(double) * N);
    oracle_sf_window(N, margin_rf * rho, sf);
    double inv2r2 = 1.0 / (2.0 * rho * rho), pix0 = 2.0 * ORACLE_PI * rho * rho / N;
    double pref = 1.0 / (2.0 * ORACLE_PI * rho * rho);
#pragma omp parallel for schedule(static)
    for (int m = 0; m < N; ++m)
        for (int mx = 0; mx < N; ++mx) {
            double x0 = (mx - N / 2) * pix0, y0 = (m - N / 2) * pix0;
            cplx acc = 0.0;
            for (int y = 0; y < N; ++y)
                for (int x = 0; x < N; ++x) {
                    double dx = x0 - (x - N / 2), dy = y0 - (y - N / 2);
                    double arg = s * phi[(size_t)y * N + x] + (dx * dx + dy * dy) * inv2r2;
                    acc += sf[x] * sf[y] * (cos(arg) + sin(arg) * I);
                }
            acc *= pref;
            I_out[(size_t)m * N + mx] = creal(acc) * creal(acc) + cimag(acc) * cimag(acc);
        }
    free(sf);
}

/* ------------------------------------------------------------------------ */
/* Structure-function check of a screen (Sect. 3.1.1, Eq. crec), pixel     */
/* units.  S_rec[b] = <|F_phi|^2>/(L_x L_y) = <|DFT phi|^2>/N^2 over the    */
/* Fourier pixels of signed frequency k' (components in [-N/2, N/2)) whose  */
/* |k'| rounds to b, for b = 0 .. N/2; count[b] = number of such pixels.    */
/* xi(r) = sum_{b=1}^{N/2} 2 pi q_b S_b J0(2 pi q_b r) dq with q_b = b/N and */
/* dq = 1/N (q_min = 1/N, q_max = 1/2, the paper's integration limits);     */
/* D(r) = 2 (xi(0) - xi(r)); R_diff^rec solves D = 1.                       */
/* ------------------------------------------------------------------------ */

void oracle_ring_spectrum(int N, const double *phi, double *S, double *count)
{
    size_t NN = (size_t)N * N;
    cplx *a = (cplx *)malloc(sizeof(cplx) * NN);
    for (size_t i = 0; i < NN; ++i) a[i] = phi[i];
    dft2_inplace(N, a, -1);
    int nb = N / 2 + 1;
    for (int b = 0; b < nb; ++b) { S[b] = 0.0; count[b] = 0.0; }
    for (int ky = 0; ky < N; ++ky)
        for (int kx = 0; kx < N; ++kx) {
            double fy = signed_freq(ky, N), fx = signed_freq(kx, N);
            int b = (int)floor(sqrt(fx * fx + fy * fy) + 0.5);
            if (b >= nb) continue;
            cplx v = a[(size_t)ky * N + kx];
            S[b] += (creal(v) * creal(v) + cimag(v) * cimag(v)) / ((double)N * (double)N);
            count[b] += 1.0;
        }
    for (int b = 0; b < nb; ++b)
        if (count[b] > 0) S[b] /= count[b];
    free(a);
}

double oracle_structure_from_spectrum(int N, const double *S, double r)
{
    double d = 0.0;
    for (int b = 1; b <= N / 2; ++b) {
        double q = (double)b / N;
        d += 2.0 * ORACLE_PI * q * S[b] * (1.0 - j0(2.0 * ORACLE_PI * q * r)) / N;
    }
    return 2.0 * d;
}

double oracle_rdiff_rec(int N, const double *S)
{
    double lo = 1e-3, hi = N / 2.0;
    if (oracle_structure_from_spectrum(N, S, lo) >= 1.0 || oracle_structure_from_spectrum(N, S, hi) < 1.0)
        return NAN;
    for (int it = 0; it < 200 && hi - lo > 1e-12 * hi; ++it) {
        double mid = 0.5 * (lo + hi);
        if (oracle_structure_from_spectrum(N, S, mid) < 1.0) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

/* ------------------------------------------------------------------------ */
/* Polychromatic co-addition (Sect. 3.2.4): the same screen seen at several */
/* wavelengths; the phase scales as 1/lambda (Sect. 2, Eq. phiNl), so the   */
/* screen at lambda_j is (lambda_ref / lambda_j) phi_ref; R_F scales as      */
/* sqrt(lambda).  Weights are normalised to sum 1 (NULL = equal weights).   */
/* ------------------------------------------------------------------------ */

void oracle_polychromatic(int N, double delta, double z, const double *phi_ref,
                          double lambda_ref, const double *lambdas, const double *weights,
                          int n_lambda, double *I_out)
{
    size_t NN = (size_t)N * N;
    double wsum = 0.0;
    for (int j = 0; j < n_lambda; ++j) wsum += weights ? weights[j] : 1.0;
    double *tmp = (double *)malloc(sizeof(double) * NN);
    for (size_t i = 0; i < NN; ++i) I_out[i] = 0.0;
    for (int j = 0; j < n_lambda; ++j) {
        double w = (weights ? weights[j] : 1.0) / wsum;
        double rho = oracle_fresnel_radius_px(delta, lambdas[j], z);
        oracle_propagate(N, rho, lambda_ref / lambdas[j], phi_ref, tmp, NULL);
        for (size_t i = 0; i < NN; ++i) I_out[i] += w * tmp[i];
    }
    free(tmp);
}

/* ------------------------------------------------------------------------ */
/* Extended source (Sect. 3.2.3, Eq. iprh): I_ext = P_r * h, P_r a uniform  */
/* disk of radius R_s normalised to unit sum on the pixel grid: pixels whose */
/* centre lies within R_s (minimum-image distance on the periodic grid).     */
/* ------------------------------------------------------------------------ */

static double disk_weight_count(int N, double Rs, unsigned char *mask)
{
    double count = 0.0;
    for (int y = 0; y < N; ++y)
        for (int x = 0; x < N; ++x) {
            double dx = signed_freq(x, N), dy = signed_freq(y, N);
            int in = dx * dx + dy * dy <= Rs * Rs;
            if (mask) mask[(size_t)y * N + x] = (unsigned char)in;
            count += in;
        }
    return count;
}

/* Via DFT: I_ext = IDFT[ DFT[P] DFT[I] ] / N^2. */
void oracle_smear(int N, const double *I_in, double Rs_px, double *I_out)
{
    size_t NN = (size_t)N * N;
    unsigned char *mask = (unsigned char *)malloc(NN);
    double count = disk_weight_count(N, Rs_px, mask);
    cplx *p = (cplx *)malloc(sizeof(cplx) * NN);
    cplx *f = (cplx *)malloc(sizeof(cplx) * NN);
    for (size_t i = 0; i < NN; ++i) {
        p[i] = mask[i] ? 1.0 / count : 0.0;
        f[i] = I_in[i];
    }
    dft2_inplace(N, p, -1);
    dft2_inplace(N, f, -1);
    double norm = 1.0 / (double)NN;
    for (size_t i = 0; i < NN; ++i) f[i] *= p[i] * norm;
    dft2_inplace(N, f, +1);
    for (size_t i = 0; i < NN; ++i) I_out[i] = creal(f[i]);
    free(mask); free(p); free(f);
}

/* Direct circular convolution, O(N^2 n_disk): I_ext[m] = sum_d P[d] I[m-d]. */
void oracle_smear_direct(int N, const double *I_in, double Rs_px, double *I_out)
{
    int Rc = (int)ceil(Rs_px);
    double count = disk_weight_count(N, Rs_px, NULL);
#pragma omp parallel for schedule(static)
    for (int y = 0; y < N; ++y)
        for (int x = 0; x < N; ++x) {
            double acc = 0.0;
            for (int dy = -Rc; dy <= Rc; ++dy)
                for (int dx = -Rc; dx <= Rc; ++dx) {
                    /* each displacement taken once on the torus */
                    int sx = ((dx % N) + N) % N, sy = ((dy % N) + N) % N;
                    double mx = signed_freq(sx, N), my = signed_freq(sy, N);
                    if (mx != dx || my != dy) continue;
                    if ((double)dx * dx + (double)dy * dy > Rs_px * Rs_px) continue;
                    int yy = ((y - dy) % N + N) % N, xx = ((x - dx) % N + N) % N;
                    acc += I_in[(size_t)yy * N + xx];
                }
            I_out[(size_t)y * N + x] = acc / count;
        }
}

double oracle_disk_count(int N, double Rs_px) { return disk_weight_count(N, Rs_px, NULL); }

/* ------------------------------------------------------------------------ */
/* Modulation index m = sigma_I / mean(I) (Sect. 4), population sigma,       */
/* two-pass with Kahan-compensated sums.                                     */
/* ------------------------------------------------------------------------ */

double oracle_modulation_index(int N, const double *inten)
{
    size_t NN = (size_t)N * N;
    double s = 0.0, c = 0.0;
    for (size_t i = 0; i < NN; ++i) {
        double yv = inten[i] - c, t = s + yv;
        c = (t - s) - yv; s = t;
    }
    double mean = s / (double)NN;
    double v = 0.0; c = 0.0;
    for (size_t i = 0; i < NN; ++i) {
        double d = inten[i] - mean;
        double yv = d * d - c, t = v + yv;
        c = (t - v) - yv; v = t;
    }
    return sqrt(v / (double)NN) / mean;
}

/* m and the mean over the rectangle of w x h pixels whose first pixel is    */
/* (x0, y0): the statistics inside a fiducial zone (Sect. 3.2.1, 4).         */
double oracle_modulation_index_region(int N, const double *inten, int x0, int y0, int w, int h,
                                      double *mean_out)
{
    double s = 0.0, c = 0.0;
    for (int y = y0; y < y0 + h; ++y)
        for (int x = x0; x < x0 + w; ++x) {
            double yv = inten[(size_t)y * N + x] - c, t = s + yv;
            c = (t - s) - yv; s = t;
        }
    double cnt = (double)w * (double)h, mean = s / cnt;
    double v = 0.0; c = 0.0;
    for (int y = y0; y < y0 + h; ++y)
        for (int x = x0; x < x0 + w; ++x) {
            double d = inten[(size_t)y * N + x] - mean;
            double yv = d * d - c, t = v + yv;
            c = (t - v) - yv; v = t;
        }
    if (mean_out) *mean_out = mean;
    return sqrt(v / cnt) / mean;
}

/* ------------------------------------------------------------------------ */
/* Light curves (Sect. 3.3): the pattern sampled along straight lines at a  */
/* constant relative speed.  Pixel (ix, iy) sits at the integer point       */
/* (ix, iy); sample k of a line lies at (x0 + k dx, y0 + k dy) in pixels,   */
/* wrapped onto the periodic pattern.  mode 0 takes the pixel nearest to    */
/* the point, mode 1 interpolates bilinearly between the four around it.    */
/* m of each curve as in Sect. 4 (population sigma over the samples).       */
/* ------------------------------------------------------------------------ */

static long wrap_index(double v, int N)
{
    long i = (long)floor(v);
    long r = i % N;
    return r < 0 ? r + N : r;
}

void oracle_light_curves(int N, const double *inten, int n_lines, const double *lines, int n_samples,
                         int mode, double *curves, double *m_out)
{
    for (int l = 0; l < n_lines; ++l) {
        const double x0 = lines[4 * l], y0 = lines[4 * l + 1], dx = lines[4 * l + 2], dy = lines[4 * l + 3];
        double *c = curves + (size_t)l * n_samples;
        for (int k = 0; k < n_samples; ++k) {
            double x = x0 + k * dx, y = y0 + k * dy;
            if (mode == 0) {
                long ix = wrap_index(x + 0.5, N), iy = wrap_index(y + 0.5, N);
                c[k] = inten[(size_t)iy * N + ix];
            } else {
                double fx = x - floor(x), fy = y - floor(y);
                long ix = wrap_index(x, N), iy = wrap_index(y, N);
                long jx = (ix + 1) % N, jy = (iy + 1) % N;
                c[k] = (1 - fx) * (1 - fy) * inten[(size_t)iy * N + ix] + fx * (1 - fy) * inten[(size_t)iy * N + jx] +
                       (1 - fx) * fy * inten[(size_t)jy * N + ix] + fx * fy * inten[(size_t)jy * N + jx];
            }
        }
        if (m_out) {
            double s = 0.0, cc = 0.0;
            for (int k = 0; k < n_samples; ++k) {
                double yv = c[k] - cc, t = s + yv;
                cc = (t - s) - yv; s = t;
            }
            double mean = s / n_samples, v = 0.0;
            cc = 0.0;
            for (int k = 0; k < n_samples; ++k) {
                double d = c[k] - mean, yv = d * d - cc, t = v + yv;
                cc = (t - v) - yv; v = t;
            }
            m_out[l] = sqrt(v / n_samples) / mean;
        }
    }
}

/* Expected modulation index of an extended source in the strong, quenched */
/* regime for Kolmogorov turbulence (Sect. 4.1, Eq. xparam, after Narayan  */
/* 1992): m = (R_diff/R_F)^(1/3) (R_ref / (2 pi R_s))^(7/6) with           */
/* R_ref = 2 pi R_F^2 / R_diff; any one length unit.                        */
double oracle_m_theory(double r_diff, double r_f, double r_s)
{
    double r_ref = 2.0 * ORACLE_PI * r_f * r_f / r_diff;
    return pow(r_diff / r_f, 1.0 / 3.0) * pow(r_ref / (2.0 * ORACLE_PI * r_s), 7.0 / 6.0);
}

/* ------------------------------------------------------------------------ */
/* Adjoint of the propagation (vector-Jacobian product).                    */
/* Given grad_I = dL/dI: g_A = 2 grad_I A; g_U = N^-2 IDFT[conj(H) DFT[g_A]] */
/* (the adjoint of the linear propagation); dL/dphi = s Im(g_U conj(U)).     */
/* ------------------------------------------------------------------------ */

void oracle_propagate_vjp(int N, double rho, double s, const double *phi,
                          const double *grad_I, double *grad_phi)
{
    size_t NN = (size_t)N * N;
    cplx *a = (cplx *)malloc(sizeof(cplx) * NN);
    double *Iv = (double *)malloc(sizeof(double) * NN);
    oracle_propagate(N, rho, s, phi, Iv, (double *)a);
#pragma omp parallel for schedule(static)
    for (size_t i = 0; i < NN; ++i) a[i] *= 2.0 * grad_I[i];
    propagate_field(N, rho, a, 1);
#pragma omp parallel for schedule(static)
    for (size_t i = 0; i < NN; ++i) {
        cplx u = expi_turns(s * phi[i] / (2.0 * ORACLE_PI));
        grad_phi[i] = s * cimag(a[i] * conj(u));
    }
    free(a); free(Iv);
}

/* Apply the adjoint propagation alone: out = N^-2 IDFT[conj(H) DFT[in]]. */
void oracle_propagate_adjoint_field(int N, double rho, const double *in_ri, double *out_ri)
{
    size_t NN = (size_t)N * N;
    memcpy(out_ri, in_ri, sizeof(cplx) * NN);
    propagate_field(N, rho, (cplx *)out_ri, 1);
}

/* Apply the forward propagation alone to a complex field. */
void oracle_propagate_field(int N, double rho, const double *in_ri, double *out_ri)
{
    size_t NN = (size_t)N * N;
    memcpy(out_ri, in_ri, sizeof(cplx) * NN);
    propagate_field(N, rho, (cplx *)out_ri, 0);
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

// aux_kernels.hip -- batched transposes, chirp tables, disk images and
// deterministic reductions for gfx950.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "aux_kernels.h"
#include "device_common.hpp"
#include "transpose_tile.hpp"

namespace scint {

// ---------------------------------------------------------------- transpose
// One 64 x 128 unit per workgroup of 256 threads (transpose_tile.hpp): grid
// x over units along the columns, y along the rows, z over the batch.
template <typename T>
__global__ __launch_bounds__(256) void transpose_pair_kernel(const T *__restrict__ in, T *__restrict__ out, int N) {
    __shared__ TransposeTile<T> tile;
    const int64_t base = (int64_t)blockIdx.z * N * N;
    transpose_unit<T, 256>(in + base, out + base, N, blockIdx.x, blockIdx.y, tile, threadIdx.x);
}

// complex128: one 16-byte element per lane, TILE x TILE tile.
template <typename T, int TILE>
__global__ __launch_bounds__(256) void transpose_kernel(const T *__restrict__ in, T *__restrict__ out, int N) {
    __shared__ T tile[TILE][TILE + 1];
    constexpr int ROWS = 256 / TILE;
    const int tx = threadIdx.x % TILE, ty = threadIdx.x / TILE;
    const int x0 = blockIdx.x * TILE, y0 = blockIdx.y * TILE;
    const int64_t base = (int64_t)blockIdx.z * N * N;
    const T *src = in + base;
    T *dst = out + base;
    // unguarded loads at clamped addresses (all in flight at once); the slots
    // filled for positions outside the matrix are never read
    T v[TILE / ROWS];
    const int xc = min(x0 + tx, N - 1);
#pragma unroll
    for (int k = 0; k < TILE / ROWS; ++k) v[k] = src[(int64_t)min(y0 + ty + k * ROWS, N - 1) * N + xc];
#pragma unroll
    for (int k = 0; k < TILE / ROWS; ++k) tile[ty + k * ROWS][tx] = v[k];
    __syncthreads();
#pragma unroll
    for (int r = ty; r < TILE; r += ROWS) {
        const int x = x0 + r, y = y0 + tx;
        if (x < N && y < N) dst[(int64_t)x * N + y] = tile[tx][r];
    }
}

struct alignas(8) Elem8 {
    float a, b;
};
struct alignas(16) Elem16 {
    double a, b;
};

hipError_t launch_transpose(const void *in, void *out, int N, int64_t nbatch, int elem_bytes,
                            hipStream_t stream) {
    if (N % 2 != 0) return hipErrorInvalidValue;
    for (int64_t b0 = 0; b0 < nbatch; b0 += 65535) {
        const int nb = (int)((nbatch - b0) < 65535 ? (nbatch - b0) : 65535);
        const int64_t off = b0 * (int64_t)N * N;
        const dim3 grid64(transpose_units_x(N), transpose_units_y(N), nb);
        if (elem_bytes == 4) {
            hipLaunchKernelGGL((transpose_pair_kernel<float>), grid64, dim3(256), 0, stream,
                               static_cast<const float *>(in) + off, static_cast<float *>(out) + off, N);
        } else if (elem_bytes == 8) {
            hipLaunchKernelGGL((transpose_pair_kernel<Elem8>), grid64, dim3(256), 0, stream,
                               static_cast<const Elem8 *>(in) + off, static_cast<Elem8 *>(out) + off, N);
        } else if (elem_bytes == 16) {
            constexpr int TILE = 32;
            dim3 grid((N + TILE - 1) / TILE, (N + TILE - 1) / TILE, nb);
            hipLaunchKernelGGL((transpose_kernel<Elem16, TILE>), grid, dim3(256), 0, stream,
                               static_cast<const Elem16 *>(in) + off, static_cast<Elem16 *>(out) + off, N);
        } else {
            return hipErrorInvalidValue;
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// ---------------------------------------------------------------- low modes
struct LowModeArgs {
    int N, K;
    uint32_t r0, seed_lo, seed_hi;
    double amp0, neg_beta_4;
    int swap;  // C[b][i][j] = c(kx' = j - K, ky' = i - K) instead
};

// C[b][i][j]: one workgroup per (i, b), thread j
__global__ __launch_bounds__(64) void low_mode_coeff_kernel(double2 *C, LowModeArgs a) {
    const int W = 2 * a.K + 1;
    const int i = blockIdx.x, b = blockIdx.y, j = threadIdx.x;
    if (j >= W) return;
    const int fx = (a.swap ? j : i) - a.K, fy = (a.swap ? i : j) - a.K;
    const int kx = fx < 0 ? fx + a.N : fx, ky = fy < 0 ? fy + a.N : fy;
    C[((int64_t)b * W + i) * W + j] =
        spectrum_coeff_f64(kx, ky, a.N, a.r0 + (uint32_t)b, a.seed_lo, a.seed_hi, a.amp0, a.neg_beta_4);
}

// G[b][y][k]: one workgroup per (y, b); the W factors exp(2 pi i ky' y / N)
// (argument reduced exactly in integers) go through LDS, thread k <= K sums
// B(k) and B(-k) in a fixed order
__global__ __launch_bounds__(64) void low_mode_rows_kernel(const double2 *__restrict__ C, double2 *__restrict__ G,
                                                           LowModeArgs a) {
    __shared__ double2 e[64];
    const int W = 2 * a.K + 1;
    const int y = blockIdx.x, b = blockIdx.y, t = threadIdx.x;
    if (t < W) {
        int64_t m = ((int64_t)(t - a.K) * y) % a.N;
        if (m < 0) m += a.N;
        double sn, cs;
        sincospi(2.0 * (double)m / (double)a.N, &sn, &cs);
        e[t] = make_double2(cs, sn);
    }
    __syncthreads();
    if (t > a.K) return;
    const double2 *Cb = C + (int64_t)b * W * W;
    auto B = [&](int fx) {
        const double2 *row = Cb + (int64_t)(fx + a.K) * W;
        double re = 0.0, im = 0.0;
        for (int j = 0; j < W; ++j) {
            const double2 c = row[j], w = e[j];
            re = fma(c.x, w.x, fma(-c.y, w.y, re));
            im = fma(c.x, w.y, fma(c.y, w.x, im));
        }
        return make_double2(re, im);
    };
    constexpr double kSqrt2 = 1.41421356237309504880;
    const double2 bp = B(t);
    double2 g = bp;
    if (t > 0) {
        const double2 bm = B(-t);
        g = make_double2(bp.x + bm.x, bp.y - bm.y);
    }
    G[((int64_t)b * a.N + y) * (a.K + 1) + t] = make_double2(kSqrt2 * g.x, kSqrt2 * g.y);
}

hipError_t launch_low_modes(void *C, void *G, int N, int K, int nbatch, uint32_t r0, uint32_t seed_lo,
                            uint32_t seed_hi, double amp0, double neg_beta_4, hipStream_t stream, bool swap) {
    if (K < 0 || 2 * K + 1 > 64 || K >= N / 2 || nbatch < 1) return hipErrorInvalidValue;
    const int W = 2 * K + 1;
    for (int b0 = 0; b0 < nbatch; b0 += 65535) {
        const int nb = nbatch - b0 < 65535 ? nbatch - b0 : 65535;
        LowModeArgs a{N, K, r0 + (uint32_t)b0, seed_lo, seed_hi, amp0, neg_beta_4, swap ? 1 : 0};
        double2 *Cb = static_cast<double2 *>(C) + (int64_t)b0 * W * W;
        double2 *Gb = static_cast<double2 *>(G) + (int64_t)b0 * N * (K + 1);
        hipLaunchKernelGGL(low_mode_coeff_kernel, dim3(W, nb), dim3(64), 0, stream, Cb, a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(low_mode_rows_kernel, dim3(N, nb), dim3(64), 0, stream, Cb, Gb, a);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// ---------------------------------------------------------------- twiddles
struct TwiddleArgs {
    int n, total;
    int ns[8], R[8], off[8];
};

template <typename Real>
__global__ __launch_bounds__(256) void twiddle_table_kernel(cpx<Real> *tab, TwiddleArgs a) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= a.total) return;
    int s = 0;
    while (s + 1 < a.n && i >= a.off[s + 1]) ++s;
    const int j = i - a.off[s];
    const int64_t k = j / a.R[s], r = j - k * a.R[s];
    const int64_t M = (int64_t)a.ns[s] * a.R[s];
    const int64_t m = (r * k) % M;
    double sn, cs;
    sincospi(2.0 * (double)m / (double)M, &sn, &cs);
    tab[i] = {(Real)cs, (Real)(-sn)};
}

hipError_t launch_twiddle_table(void *tab, int n_stages, const int *ns, const int *R, const int *off, int total,
                                bool f64, hipStream_t stream) {
    if (n_stages < 0 || n_stages > 8 || total < 0) return hipErrorInvalidValue;
    if (total == 0) return hipSuccess;
    TwiddleArgs a{};
    a.n = n_stages;
    a.total = total;
    for (int s = 0; s < n_stages; ++s) {
        a.ns[s] = ns[s];
        a.R[s] = R[s];
        a.off[s] = off[s];
    }
    const dim3 grid((total + 255) / 256);
    if (f64)
        hipLaunchKernelGGL((twiddle_table_kernel<double>), grid, dim3(256), 0, stream, static_cast<cpx<double> *>(tab), a);
    else
        hipLaunchKernelGGL((twiddle_table_kernel<float>), grid, dim3(256), 0, stream, static_cast<cpx<float> *>(tab), a);
    return hipGetLastError();
}

// ---------------------------------------------------------------- chirp
struct ChirpArgs {
    double a[64];
    double amp[64];
};

template <typename Real>
__global__ __launch_bounds__(256) void chirp_kernel(cpx<Real> *tab, int N, ChirpArgs args, int n, double scale) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    const int j = blockIdx.y;
    if (k >= N || j >= n) return;
    const double kk = (double)(k < N / 2 ? k : k - N);
    const double turns = args.a[j] * (kk * kk);
    const double f = turns - rint(turns);
    double s, c;
    sincospi(2.0 * f, &s, &c);
    const double g = scale * args.amp[j];
    tab[(int64_t)j * N + k] = {(Real)(g * c), (Real)(-g * s)};
}

hipError_t launch_chirp_tables(void *tab, int N, const double *a, int n, double scale, bool f64,
                               hipStream_t stream, const double *amp) {
    if (n < 1 || n > 64) return hipErrorInvalidValue;
    ChirpArgs args{};
    for (int j = 0; j < n; ++j) {
        args.a[j] = a[j];
        args.amp[j] = amp ? amp[j] : 1.0;
    }
    dim3 grid((N + 255) / 256, n);
    if (f64)
        hipLaunchKernelGGL((chirp_kernel<double>), grid, dim3(256), 0, stream, static_cast<cpx<double> *>(tab), N,
                           args, n, scale);
    else
        hipLaunchKernelGGL((chirp_kernel<float>), grid, dim3(256), 0, stream, static_cast<cpx<float> *>(tab), N,
                           args, n, scale);
    return hipGetLastError();
}

// ---------------------------------------------------------------- aperture
// A[j] = SF(j + 1/2) exp(i ((j - N/2)^2 / (2 rho^2) + pi j)) in FP64, rounded
// once.  The phase is formed in turns, (j - N/2)^2 exactly times
// 1/(4 pi rho^2), plus j/2, and reduced to [-1/2, 1/2] before sincospi.  The
// window is the raised sine over Lm pixels at each border (Lm = 0: none).
template <typename Real>
__global__ __launch_bounds__(256) void aperture_table_kernel(cpx<Real> *tab, int N, double a, double Lm) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= N) return;
    const double d = (double)(j - N / 2);
    const double turns = a * (d * d) + 0.5 * (double)(j & 1);
    const double f = turns - rint(turns);
    double s, c;
    sincospi(2.0 * f, &s, &c);
    const double x = (double)j + 0.5;
    double w = 1.0;
    if (Lm > 0.0) {
        if (x <= Lm)
            w = 0.5 * (1.0 - cospi(x / Lm));
        else if (x >= (double)N - Lm)
            w = 0.5 * (1.0 + cospi((x - (double)N + Lm) / Lm));
    }
    tab[j] = {(Real)(w * c), (Real)(w * s)};
}

hipError_t launch_aperture_table(void *tab, int N, double a, double Lm, bool f64, hipStream_t stream) {
    dim3 grid((N + 255) / 256);
    if (f64)
        hipLaunchKernelGGL((aperture_table_kernel<double>), grid, dim3(256), 0, stream,
                           static_cast<cpx<double> *>(tab), N, a, Lm);
    else
        hipLaunchKernelGGL((aperture_table_kernel<float>), grid, dim3(256), 0, stream,
                           static_cast<cpx<float> *>(tab), N, a, Lm);
    return hipGetLastError();
}

// ---------------------------------------------------------------- disk
template <typename Real>
__global__ __launch_bounds__(256) void disk_kernel(Real *img, int N, double r2, double value) {
    const int x = blockIdx.x * 256 + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= N) return;
    const double dx = (double)(x < N / 2 ? x : x - N);
    const double dy = (double)(y < N / 2 ? y : y - N);
    img[(int64_t)y * N + x] = (dx * dx + dy * dy <= r2) ? (Real)value : (Real)0;
}

hipError_t launch_disk_image(void *img, int N, double r2, double value, bool f64, hipStream_t stream) {
    dim3 grid((N + 255) / 256, N);
    if (f64)
        hipLaunchKernelGGL((disk_kernel<double>), grid, dim3(256), 0, stream, static_cast<double *>(img), N, r2,
                           value);
    else
        hipLaunchKernelGGL((disk_kernel<float>), grid, dim3(256), 0, stream, static_cast<float *>(img), N, r2,
                           value);
    return hipGetLastError();
}

// ---------------------------------------------------------------- reductions
// Block tree over 256 FP64 partials in LDS (fixed order).
__device__ __forceinline__ double block_tree_sum(double v, double *red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    return red[0];
}

// Partial sums of (x - center)^power over a w-wide region of each batch
// member: element i of the region is x[b * batch_stride + (i / w) *
// row_stride + i % w]; a contiguous run when w == row_stride.
template <typename Real>
__global__ __launch_bounds__(256) void block_sums_kernel(const Real *__restrict__ x, int64_t n, int64_t batch_stride,
                                                         int64_t w, int64_t row_stride, const double *center,
                                                         int power, double *partials) {
    __shared__ double red[256];
    const int b = blockIdx.y, nblk = gridDim.x;
    const Real *xb = x + (int64_t)b * batch_stride;
    const double c = center ? center[b] : 0.0;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)nblk * 256) {
        const int64_t e = (w == row_stride) ? i : (i / w) * row_stride + i % w;
        const double d = (double)xb[e] - c;
        acc += (power == 2) ? d * d : d;
    }
    const double tot = block_tree_sum(acc, red);
    if (threadIdx.x == 0) partials[(int64_t)b * nblk + blockIdx.x] = tot;
}

hipError_t launch_region_sums(const void *x, int64_t batch_stride, int64_t w, int64_t h, int64_t row_stride,
                              int nbatch, const double *center, int power, int nblk, bool f64, double *partials,
                              hipStream_t stream) {
    dim3 grid(nblk, nbatch);
    const int64_t n = w * h;
    // a full-width region (or a single row) is one contiguous run
    const bool run = row_stride == w || h == 1;
    const int64_t ww = run ? 1 : w, rs = run ? 1 : row_stride;
    if (f64)
        hipLaunchKernelGGL((block_sums_kernel<double>), grid, dim3(256), 0, stream, static_cast<const double *>(x),
                           n, batch_stride, ww, rs, center, power, partials);
    else
        hipLaunchKernelGGL((block_sums_kernel<float>), grid, dim3(256), 0, stream, static_cast<const float *>(x), n,
                           batch_stride, ww, rs, center, power, partials);
    return hipGetLastError();
}

hipError_t launch_block_sums(const void *x, int64_t n_per_batch, int nbatch, const double *center, int power,
                             int nblk, bool f64, double *partials, hipStream_t stream) {
    return launch_region_sums(x, n_per_batch, n_per_batch, 1, n_per_batch, nbatch, center, power, nblk, f64,
                              partials, stream);
}

// ---------------------------------------------------------------- light curves
// One workgroup per (pattern, line): sample k of line l lies at
// (x0 + k dx, y0 + k dy) pixels (pixel (ix, iy) at the integer point), wrapped
// onto the periodic pattern; mode 0 takes the nearest pixel, mode 1
// interpolates bilinearly (weights and sum in FP64).  The curve is written
// and its mean and population variance formed in FP64 in a fixed order.
__device__ __forceinline__ int64_t wrap_floor(double v, int N) {
    const int64_t i = (int64_t)floor(v);
    const int64_t r = i % N;
    return r < 0 ? r + N : r;
}

// x0 + k dx with the product and the sum rounded separately (no fused
// multiply-add), the same position a plain evaluation of the formula gives
__device__ __forceinline__ double sample_coord(double x0, int k, double dx) {
#pragma clang fp contract(off)
    return x0 + (double)k * dx;
}

template <typename Real>
__global__ __launch_bounds__(256) void light_curve_kernel(const Real *__restrict__ I, int N, LineSet ls, int n_samples,
                                                          int mode, Real *__restrict__ out, int n_lines_total,
                                                          int line0, double *stats) {
    __shared__ double red[256];
    const int l = blockIdx.x, b = blockIdx.y;
    const Real *img = I + (int64_t)b * N * N;
    Real *c = out + ((int64_t)b * n_lines_total + line0 + l) * n_samples;
    const double x0 = ls.p[l][0], y0 = ls.p[l][1], dx = ls.p[l][2], dy = ls.p[l][3];
    double acc = 0.0;
    for (int k = threadIdx.x; k < n_samples; k += 256) {
        const double x = sample_coord(x0, k, dx), y = sample_coord(y0, k, dy);
        Real v;
        if (mode == 0) {
            v = img[wrap_floor(y + 0.5, N) * N + wrap_floor(x + 0.5, N)];
        } else {
            const double fx = x - floor(x), fy = y - floor(y);
            const int64_t ix = wrap_floor(x, N), iy = wrap_floor(y, N);
            const int64_t jx = ix + 1 == N ? 0 : ix + 1, jy = iy + 1 == N ? 0 : iy + 1;
            v = (Real)((1.0 - fx) * (1.0 - fy) * (double)img[iy * N + ix] + fx * (1.0 - fy) * (double)img[iy * N + jx] +
                       (1.0 - fx) * fy * (double)img[jy * N + ix] + fx * fy * (double)img[jy * N + jx]);
        }
        c[k] = v;
        acc += (double)v;
    }
    const double mean = block_tree_sum(acc, red) / (double)n_samples;
    __syncthreads();
    double acc2 = 0.0;
    for (int k = threadIdx.x; k < n_samples; k += 256) {  // each thread re-reads its own samples
        const double d = (double)c[k] - mean;
        acc2 += d * d;
    }
    const double var = block_tree_sum(acc2, red) / (double)n_samples;
    if (threadIdx.x == 0 && stats) {
        stats[2 * ((int64_t)b * n_lines_total + line0 + l)] = mean;
        stats[2 * ((int64_t)b * n_lines_total + line0 + l) + 1] = var;
    }
}

hipError_t launch_light_curves(const void *I, int N, int nbatch, const double *lines, int n_lines, int n_samples,
                               int mode, bool f64, void *out, double *stats, hipStream_t stream) {
    for (int l0 = 0; l0 < n_lines; l0 += kLinesPerLaunch) {
        const int nl = n_lines - l0 < kLinesPerLaunch ? n_lines - l0 : kLinesPerLaunch;
        LineSet ls{};
        for (int l = 0; l < nl; ++l)
            for (int q = 0; q < 4; ++q) ls.p[l][q] = lines[4 * (l0 + l) + q];
        dim3 grid(nl, nbatch);
        if (f64)
            hipLaunchKernelGGL((light_curve_kernel<double>), grid, dim3(256), 0, stream,
                               static_cast<const double *>(I), N, ls, n_samples, mode, static_cast<double *>(out),
                               n_lines, l0, stats);
        else
            hipLaunchKernelGGL((light_curve_kernel<float>), grid, dim3(256), 0, stream,
                               static_cast<const float *>(I), N, ls, n_samples, mode, static_cast<float *>(out),
                               n_lines, l0, stats);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// ---------------------------------------------------------------- structure function
// Ring sums of a power map P [batch][N][N] (either orientation): ring b holds
// the pixels of signed frequency k' (components in [-N/2, N/2)) with
// (2b - 1)^2 <= 4 |k'|^2 < (2b + 1)^2 (|k'| rounds to b).  One workgroup per
// (ring, batch member); each thread walks whole rows of the ring and the
// partial sums meet in a fixed-order tree, so the result is reproducible.
__device__ __forceinline__ int64_t isqrt_floor(int64_t v) {  // floor(sqrt(v)), v >= 0
    int64_t r = (int64_t)sqrt((double)v);
    while (r * r > v) --r;
    while ((r + 1) * (r + 1) <= v) ++r;
    return r;
}

template <typename Real>
__global__ __launch_bounds__(256) void ring_sum_kernel(const Real *__restrict__ P, int N, double *S, double *count) {
    __shared__ double red[256];
    const int b = blockIdx.x, bat = blockIdx.y;
    const Real *img = P + (int64_t)bat * N * N;
    const int64_t lo2 = b == 0 ? 0 : (int64_t)(2 * b - 1) * (2 * b - 1), hi2 = (int64_t)(2 * b + 1) * (2 * b + 1);
    const int h = N / 2;
    double acc = 0.0, cnt = 0.0;
    for (int ky = -(b + 1) + (int)threadIdx.x; ky <= b + 1; ky += 256) {
        if (ky < -h || ky >= h) continue;
        const int64_t t = 4 * (int64_t)ky * ky;
        if (t >= hi2) continue;
        // kx >= 0 with lo2 <= 4 kx^2 + t < hi2
        const int64_t kmin = (lo2 - t <= 0) ? 0 : isqrt_floor((lo2 - t + 3) / 4 - 1) + 1;
        const int64_t kmax = isqrt_floor((hi2 - t - 1) / 4);
        const Real *row = img + (int64_t)(ky < 0 ? ky + N : ky) * N;
        for (int64_t kx = kmin; kx <= kmax; ++kx) {
            if (kx < h) {  // +kx
                acc += (double)row[kx];
                cnt += 1.0;
            }
            if (kx > 0 && kx <= h) {  // -kx
                acc += (double)row[N - kx];
                cnt += 1.0;
            }
        }
    }
    const double tot = block_tree_sum(acc, red);
    __syncthreads();
    const double c = block_tree_sum(cnt, red);
    if (threadIdx.x == 0) {
        S[(int64_t)bat * gridDim.x + b] = c > 0 ? tot / c : 0.0;
        if (count && bat == 0) count[b] = c;
    }
}

hipError_t launch_ring_sums(const void *P, int N, int nbatch, bool f64, double *S, double *count, hipStream_t stream) {
    dim3 grid(N / 2 + 1, nbatch);
    if (f64)
        hipLaunchKernelGGL((ring_sum_kernel<double>), grid, dim3(256), 0, stream, static_cast<const double *>(P), N, S,
                           count);
    else
        hipLaunchKernelGGL((ring_sum_kernel<float>), grid, dim3(256), 0, stream, static_cast<const float *>(P), N, S,
                           count);
    return hipGetLastError();
}

// J0, the Bessel function of the first kind of order 0, in FP64: its power
// series sum_k (-x^2/4)^k / (k!)^2 below x = 14 (largest term about 1e4, so
// an absolute error near 1e-12), and above it Hankel's asymptotic expansion
// J0 = sqrt(2 / (pi x)) (P cos(x - pi/4) - Q sin(x - pi/4)),
// P = sum_k (-1)^k a_2k / x^2k, Q = sum_k (-1)^k a_(2k+1) / x^(2k+1),
// a_k = prod_{j <= k} (2j - 1)^2 / (k! 8^k), summed while the terms shrink.
__device__ double bessel_j0(double x) {
    x = fabs(x);
    if (x < 14.0) {
        const double y = 0.25 * x * x;
        double t = 1.0, sum = 1.0;
        for (int k = 1; k < 80; ++k) {
            t *= -y / ((double)k * (double)k);
            sum += t;
            if (fabs(t) < 1e-17 * fabs(sum) && (double)k * k > y) break;
        }
        return sum;
    }
    double P = 1.0, Q = 0.0, a = 1.0, xp = 1.0, last = 1.0;
    for (int k = 1; k < 60; ++k) {
        a *= (double)((2 * k - 1) * (2 * k - 1)) / (8.0 * k);
        xp *= x;
        const double term = a / xp;
        if (term > last) break;  // the asymptotic series starts to diverge
        last = term;
        if (k & 1)
            Q += ((k / 2) & 1) ? term : -term;  // k = 1: -a1/x, k = 3: +a3/x^3, ...
        else
            P += ((k / 2) & 1) ? -term : term;  // k = 2: -a2/x^2, k = 4: +a4/x^4, ...
        if (term < 1e-17) break;
    }
    const double ph = x - 0.25 * 3.14159265358979323846;
    return sqrt(2.0 / (3.14159265358979323846 * x)) * (P * cos(ph) - Q * sin(ph));
}

// D(r) = 2 sum_{b=1}^{N/2} 2 pi (b/N) S_b (1 - J0(2 pi b r / N)) / N for the
// workgroup's ring spectrum S (pixel units), summed over the block.
__device__ double structure_at(const double *S, int N, double r, double *red) {
    double acc = 0.0;
    for (int b = 1 + (int)threadIdx.x; b <= N / 2; b += 256) {
        const double q = (double)b / N;
        acc += q * S[b] * (1.0 - bessel_j0(2.0 * 3.14159265358979323846 * q * r));
    }
    __syncthreads();
    const double tot = block_tree_sum(acc, red);
    return 4.0 * 3.14159265358979323846 * tot / N;
}

// One workgroup per screen: D at the given radii (pixels) and, if rdiff !=
// NULL, R_diff^rec solving D = 1 by bisection on [1e-3, N/2] (NaN when the
// root is not bracketed).
__global__ __launch_bounds__(256) void hankel_kernel(const double *S, int N, RadiusSet rs, int n_r, double *D,
                                                     int ld_D, int r0, double *rdiff) {
    __shared__ double red[256];
    const int bat = blockIdx.x;
    const double *Sb = S + (int64_t)bat * (N / 2 + 1);
    for (int j = 0; j < n_r; ++j) {
        const double d = structure_at(Sb, N, rs.r[j], red);
        if (threadIdx.x == 0) D[(int64_t)bat * ld_D + r0 + j] = d;
    }
    if (!rdiff) return;
    double lo = 1e-3, hi = 0.5 * N;
    const double dlo = structure_at(Sb, N, lo, red), dhi = structure_at(Sb, N, hi, red);
    if (!(dlo < 1.0 && dhi >= 1.0)) {
        if (threadIdx.x == 0) rdiff[bat] = __longlong_as_double(0x7ff8000000000000LL);
        return;
    }
    for (int it = 0; it < 200 && hi - lo > 1e-12 * hi; ++it) {  // every thread sees the same lo, hi
        const double mid = 0.5 * (lo + hi);
        if (structure_at(Sb, N, mid, red) < 1.0)
            lo = mid;
        else
            hi = mid;
    }
    if (threadIdx.x == 0) rdiff[bat] = 0.5 * (lo + hi);
}

hipError_t launch_hankel(const double *S, int N, int nbatch, const double *radii, int n_r, double *D, double *rdiff,
                         hipStream_t stream) {
    if (n_r == 0) {
        RadiusSet rs{};
        hipLaunchKernelGGL(hankel_kernel, dim3(nbatch), dim3(256), 0, stream, S, N, rs, 0, D, 0, 0, rdiff);
        return hipGetLastError();
    }
    for (int j0 = 0; j0 < n_r; j0 += kRadiiPerLaunch) {
        const int nr = n_r - j0 < kRadiiPerLaunch ? n_r - j0 : kRadiiPerLaunch;
        RadiusSet rs{};
        for (int j = 0; j < nr; ++j) rs.r[j] = radii[j0 + j];
        // the root is found once, with the first chunk of radii
        hipLaunchKernelGGL(hankel_kernel, dim3(nbatch), dim3(256), 0, stream, S, N, rs, nr, D, n_r, j0,
                           j0 == 0 ? rdiff : nullptr);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

__global__ __launch_bounds__(256) void finalize_kernel(const double *partials, int nblk, double scale, double *out) {
    __shared__ double red[256];
    const int b = blockIdx.x;
    double acc = 0.0;
    for (int i = threadIdx.x; i < nblk; i += 256) acc += partials[(int64_t)b * nblk + i];
    const double tot = block_tree_sum(acc, red);
    if (threadIdx.x == 0) out[b] = scale * tot;
}

hipError_t launch_finalize_sums(const double *partials, int nblk, int nbatch, double scale, double *out,
                                hipStream_t stream) {
    hipLaunchKernelGGL(finalize_kernel, dim3(nbatch), dim3(256), 0, stream, partials, nblk, scale, out);
    return hipGetLastError();
}

template <typename Real>
__global__ __launch_bounds__(256) void l2_loss_kernel(const Real *__restrict__ I, const Real *__restrict__ It,
                                                      Real *__restrict__ grad, int64_t n, double *partials) {
    __shared__ double red[256];
    const int b = blockIdx.y, nblk = gridDim.x;
    const int64_t off = (int64_t)b * n;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)nblk * 256) {
        const Real d = I[off + i] - It[off + i];
        if (grad) grad[off + i] = (Real)2 * d;
        acc += (double)d * (double)d;
    }
    const double tot = block_tree_sum(acc, red);
    if (threadIdx.x == 0) partials[(int64_t)b * nblk + blockIdx.x] = tot;
}

hipError_t launch_l2_loss(const void *I, const void *It, void *grad, int64_t n_per_batch, int nbatch, int nblk,
                          bool f64, double *partials, hipStream_t stream) {
    dim3 grid(nblk, nbatch);
    if (f64)
        hipLaunchKernelGGL((l2_loss_kernel<double>), grid, dim3(256), 0, stream, static_cast<const double *>(I),
                           static_cast<const double *>(It), static_cast<double *>(grad), n_per_batch, partials);
    else
        hipLaunchKernelGGL((l2_loss_kernel<float>), grid, dim3(256), 0, stream, static_cast<const float *>(I),
                           static_cast<const float *>(It), static_cast<float *>(grad), n_per_batch, partials);
    return hipGetLastError();
}

}  // namespace scint

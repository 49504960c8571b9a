// scint_api.cpp -- the C ABI declared in include/scint.h: argument
// validation, per-device caches (twiddle tables, disk spectra), per-stream
// workspace, and the sequence of passes behind each entry point.
//
// Every 2-D transform is a row pass, a batched transpose and a second row
// pass; the pointwise steps of the method are fused into the row passes:
//   screen:      [noise -> IDFT along ky] T [IDFT along kx -> sqrt2 Re]
//   propagation: [exp(i s phi) -> DFT_x -> H1 -> IDFT_x] T
//                [DFT_y -> H1 -> IDFT_y -> |.|^2 (sum over wavelengths)] T
// The spectrum is generated with rows indexed by kx so that the first pass
// runs along ky; the transposes leave every output in natural [y][x] order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/scint.h"
#include "aux_kernels.h"
#include "fft_plan.hpp"
#include "row_launch.h"
#include "transpose_tile.hpp"

using namespace scint;

// Device memory of fresnel_propagate_noalloc: one array per GPU, held from the
// library's load until the process ends, shared by every call on that GPU.
// Host code uses it only through the address hipGetSymbolAddress returns for
// the current device (g_scratch below), never through this name.
constexpr size_t kNoAllocScratchBytes = (size_t)65 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

thread_local std::string g_last_error;
thread_local std::string g_last_warning;

int fail(int code, const std::string &msg) {
    g_last_error = msg;
    return code;
}

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail(PS_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));        \
    } while (0)

constexpr double kPiD = 3.141592653589793238462643383279502884;

bool supported_f64(int N) {
    switch (N) {
#define SCINT_CASE(LL) case LL:
        SCINT_SIZES_F64(SCINT_CASE)
#undef SCINT_CASE
        return true;
    default:
        return false;
    }
}
bool supported_f32(int N) {
    switch (N) {
#define SCINT_CASE(LL) case LL:
        SCINT_SIZES_F32(SCINT_CASE)
#undef SCINT_CASE
        return true;
    default:
        return false;
    }
}

std::vector<int> size_list(int dtype) {
    std::vector<int> v;
#define SCINT_CASE(LL) v.push_back(LL);
    if (dtype == PS_F64) {
        SCINT_SIZES_F64(SCINT_CASE)
    } else {
        SCINT_SIZES_F32(SCINT_CASE)
    }
#undef SCINT_CASE
    std::sort(v.begin(), v.end());
    return v;
}

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

int check_common(int N, int dtype, int n) {
    if (dtype != PS_F32 && dtype != PS_F64) return fail(PS_E_DTYPE, "dtype must be PS_F32 or PS_F64");
    if (!(dtype == PS_F64 ? supported_f64(N) : supported_f32(N)))
        return fail(PS_E_SIZE, "unsupported grid size N=" + std::to_string(N) + " for this dtype");
    if (n < 1) return fail(PS_E_SIZE, "batch count must be >= 1");
    // bound the number of rows so that every row index fits an int
    if ((int64_t)n * N > (int64_t)1 << 30) return fail(PS_E_SIZE, "batch too large");
    return PS_OK;
}

size_t real_bytes(int dtype) { return dtype == PS_F64 ? 8 : 4; }

// Device arrays must be 16-byte aligned (the kernels use 8- and 16-byte
// vector accesses).  NULL passes (optional arrays are checked separately).
bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }
int check_aligned(std::initializer_list<const void *> ptrs) {
    for (const void *p : ptrs)
        if (p && !aligned16(p)) return fail(PS_E_PARAM, "device arrays must be 16-byte aligned");
    return PS_OK;
}

// true if [a, a+na) and [b, b+nb) overlap
bool overlaps(const void *a, size_t na, const void *b, size_t nb) {
    const uintptr_t pa = (uintptr_t)a, pb = (uintptr_t)b;
    return pa < pb + nb && pb < pa + na;
}

// True if `stream` is being captured into a graph.  A failing query (the
// null stream while another stream captures in global mode) counts as
// capturing; its error is cleared so that later launch checks do not see it.
bool capturing(hipStream_t stream) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(stream, &st) != hipSuccess) {
        (void)hipGetLastError();
        return true;
    }
    return st != hipStreamCaptureStatusNone;
}

// PS_E_CAPTURE if `stream` is being captured: called where a call would
// allocate device memory, copy from the host or synchronise, none of which a
// captured graph may contain.
int refuse_in_capture(hipStream_t stream, const char *what) {
    if (!capturing(stream)) return PS_OK;
    return fail(PS_E_CAPTURE, std::string(what) +
                                  " would allocate or synchronise while the stream is being captured: run the "
                                  "same call once before the capture (or ps_tune_plans for the FFT plans)");
}

// ------------------------------------------------------------ device caches
struct DeviceCache {
    std::map<std::tuple<int, int, int>, void *> twiddles;  // (L, variant, dtype) -> table
    std::map<std::pair<int, int>, int> variant;             // (L, dtype) -> plan variant in use
    std::map<std::pair<int, int>, std::vector<float>> variant_ms;  // tuner timings
    // (N, dtype, radius bits...) -> n_r contiguous disk spectra
    std::map<std::pair<std::pair<int, int>, std::vector<uint64_t>>, void *> disks;
    std::map<hipStream_t, std::pair<void *, size_t>> workspace;
    size_t budget = 0;  // workspace bytes a call plans for, fixed at first use
};

std::mutex g_mutex;
std::map<int, DeviceCache> g_cache;

int current_device(int *dev) {
    hipError_t e = hipGetDevice(dev);
    if (e != hipSuccess) return fail(PS_E_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    return PS_OK;
}

// Twiddle table of plan (L, V) in the working precision.
int get_twiddles(int L, int V, int dtype, const void **out, hipStream_t stream) {
    int dev;
    if (int rc = current_device(&dev)) return rc;
    std::lock_guard<std::mutex> lock(g_mutex);
    auto &dc = g_cache[dev];
    auto key = std::make_tuple(L, V, dtype);
    auto it = dc.twiddles.find(key);
    if (it != dc.twiddles.end()) {
        *out = it->second;
        return PS_OK;
    }
    if (int rc = refuse_in_capture(stream, "building an FFT twiddle table")) return rc;
    const int n = twiddle_entries(L, V);
    std::vector<double> ri(2 * (size_t)std::max(n, 1));
    if (n > 0 && !build_twiddles(L, V, ri.data())) return fail(PS_E_SIZE, "no FFT plan for this size");
    const size_t bytes = 2 * real_bytes(dtype) * (size_t)std::max(n, 1);
    void *d = nullptr;
    if (hipMalloc(&d, bytes) != hipSuccess) return fail(PS_E_ALLOC, "hipMalloc of twiddle table failed");
    hipError_t e;
    if (dtype == PS_F64) {
        e = hipMemcpy(d, ri.data(), bytes, hipMemcpyHostToDevice);
    } else {
        std::vector<float> f(ri.size());
        for (size_t i = 0; i < ri.size(); ++i) f[i] = (float)ri[i];
        e = hipMemcpy(d, f.data(), bytes, hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        (void)hipFree(d);
        return fail(PS_E_DEVICE, std::string("hipMemcpy twiddles: ") + hipGetErrorString(e));
    }
    dc.twiddles[key] = d;
    *out = d;
    return PS_OK;
}

// Workspace of at least `bytes` for this device and stream.
int get_workspace(hipStream_t stream, size_t bytes, void **out) {
    int dev;
    if (int rc = current_device(&dev)) return rc;
    std::lock_guard<std::mutex> lock(g_mutex);
    auto &ws = g_cache[dev].workspace[stream];
    if (ws.second < bytes) {
        if (int rc = refuse_in_capture(stream, "growing the workspace")) return rc;
        if (ws.first) {
            // work queued on this stream may still use the old buffer
            HIP_TRY(hipStreamSynchronize(stream));
            (void)hipFree(ws.first);
            ws.first = nullptr;
            ws.second = 0;
        }
        const size_t want = (bytes + 255) & ~(size_t)255;
        if (hipMalloc(&ws.first, want) != hipSuccess) {
            ws.first = nullptr;
            return fail(PS_E_ALLOC, "hipMalloc of " + std::to_string(want) + " workspace bytes failed");
        }
        ws.second = want;
    }
    *out = ws.first;
    return PS_OK;
}

// Carves aligned sub-buffers out of one workspace allocation.
struct Carver {
    size_t used = 0;
    size_t take(size_t bytes) {
        size_t off = used;
        used += (bytes + 255) & ~(size_t)255;
        return off;
    }
};

// ------------------------------------------------------------ timing
// Optional per-kernel timing with events on the launch stream.
struct PendingTiming {
    std::string name;
    hipEvent_t start, stop;
    double bytes, sched_bytes, flops;
};
struct TimingTotal {
    double ms = 0.0;
    long long launches = 0;
    double bytes = 0.0;        // algorithmic bytes (each operand of the method moved once)
    double sched_bytes = 0.0;  // operand bytes of the schedule as launched
    double flops = 0.0;
};
std::mutex g_timing_mutex;
bool g_timing_on = false;
std::vector<PendingTiming> g_pending;
std::vector<hipEvent_t> g_event_pool;
std::map<std::string, TimingTotal> g_totals;

hipEvent_t pool_event() {
    if (!g_event_pool.empty()) {
        hipEvent_t e = g_event_pool.back();
        g_event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Records the start event; returns false when timing is off.
bool timing_begin(hipStream_t stream, hipEvent_t *start) {
    std::lock_guard<std::mutex> lock(g_timing_mutex);
    if (!g_timing_on) return false;
    *start = pool_event();
    if (!*start) return false;
    if (hipEventRecord(*start, stream) != hipSuccess) {
        g_event_pool.push_back(*start);
        return false;
    }
    return true;
}

void timing_end(hipStream_t stream, hipEvent_t start, const std::string &name, double bytes, double sched_bytes,
                double flops) {
    std::lock_guard<std::mutex> lock(g_timing_mutex);
    hipEvent_t stop = pool_event();
    if (!stop) return;
    if (hipEventRecord(stop, stream) != hipSuccess) {
        g_event_pool.push_back(stop);
        return;
    }
    g_pending.push_back({name, start, stop, bytes, sched_bytes, flops});
}

void timing_drain() {
    std::lock_guard<std::mutex> lock(g_timing_mutex);
    for (auto &p : g_pending) {
        float ms = 0.0f;
        if (hipEventSynchronize(p.stop) == hipSuccess && hipEventElapsedTime(&ms, p.start, p.stop) == hipSuccess) {
            auto &t = g_totals[p.name];
            t.ms += ms;
            t.launches += 1;
            t.bytes += p.bytes;
            t.sched_bytes += p.sched_bytes;
            t.flops += p.flops;
        }
        g_event_pool.push_back(p.start);
        g_event_pool.push_back(p.stop);
    }
    g_pending.clear();
}

const char *real_name(int dtype) { return dtype == PS_F64 ? "f64" : "f32"; }

// ------------------------------------------------------------ row programs
struct ProgBuilder {
    RowProgram p;
    int n = 0;
    ProgBuilder(int N, int64_t total_rows) {
        std::memset(&p, 0, sizeof(p));
        p.N = N;
        p.total_rows = (int32_t)total_rows;
        p.n_iter = 1;
        for (int i = 0; i < kRowMaxIter; ++i) {
            p.scale[i] = 1.0;
            p.weight[i] = 1.0;
        }
    }
    ProgBuilder &op(int code, const void *ptr = nullptr, int64_t batch_stride = 0, int64_t row_stride = 0,
                    int64_t iter_stride = 0, int flags = 0, double param = 0.0, void *ptr2 = nullptr) {
        RowOp &o = p.op[n++];
        o.code = code;
        o.ptr = ptr;
        o.ptr2 = ptr2;
        o.batch_stride = batch_stride;
        o.row_stride = row_stride;
        o.iter_stride = iter_stride;
        o.flags = flags;
        o.param = param;
        return *this;
    }
};

// Bytes of one row-pass launch, per element of a row summed over its rows.
// Schedule bytes (algorithmic = false): every operand access as the
// program makes it, those inside the loop once per iteration.  Algorithmic
// bytes (algorithmic = true): each array the method must read or write,
// once -- an operand inside the loop counts once per iteration only if its
// address moves with the iteration (a phase screen re-read for every
// wavelength counts once).  The 1-D chirp tables and row factors are not
// counted by either.
double row_bytes(const RowProgram &p, int n_ops, int dtype, bool algorithmic) {
    const double rb = (double)real_bytes(dtype);
    double per = 0.0;
    bool in_loop = false;
    for (int i = 0; i < n_ops; ++i) {
        const RowOp &o = p.op[i];
        double b = 0.0;
        switch (o.code) {
        case ROP_LOOP: in_loop = true; break;
        case ROP_ENDLOOP: in_loop = false; break;
        case ROP_LOAD_C: case ROP_STORE_C: b = 2 * rb; break;
        case ROP_LOAD_R: case ROP_LOAD_PHASE: case ROP_KEEP_R: case ROP_MUL_RLOAD: case ROP_MUL_RTAB2D:
        case ROP_GRAD_PHI: case ROP_DOT_R: b = rb; break;
        case ROP_STORE_R: b = o.ptr ? rb : 0.0; break;
        case ROP_STORE_ACC: b = (o.flags & RF_ADD) ? 2 * rb : rb; break;
        default: break;
        }
        const bool per_iter = in_loop && (!algorithmic || o.iter_stride != 0);
        per += per_iter ? b * p.n_iter : b;
    }
    return per * (double)p.N * (double)p.total_rows;
}

// Algorithmic floating-point operations of one row-pass launch: 5 N log2 N
// per length-N complex DFT (the usual count), 6 per complex multiply, 2 per
// real-by-complex multiply, 5 for w |v|^2 accumulated; sine/cosine and the
// noise generator are not counted.
double row_flops(const RowProgram &p, int n_ops) {
    const double log2n = std::log2((double)p.N);
    double per = 0.0;
    bool in_loop = false;
    for (int i = 0; i < n_ops; ++i) {
        double f = 0.0;
        switch (p.op[i].code) {
        case ROP_LOOP: in_loop = true; break;
        case ROP_ENDLOOP: in_loop = false; break;
        case ROP_FFT_FWD: case ROP_FFT_INV: f = 5.0 * log2n; break;
        case ROP_MUL_TAB: case ROP_MUL_ROWTAB: f = 6.0; break;
        case ROP_MUL_RTAB2D: case ROP_MUL_RLOAD: case ROP_DOT_R: f = 2.0; break;
        case ROP_ACC_ABS2: f = 5.0; break;
        case ROP_ACC_ABS2U: f = 4.0; break;
        case ROP_GRAD_PHI: f = 4.0; break;
        case ROP_SQRT2RE: f = 1.0; break;
        default: break;
        }
        per += in_loop ? f * p.n_iter : f;
    }
    return per * (double)p.N * (double)p.total_rows;
}

template <class Tag> const char *prog_name();
#define SCINT_PROG_NAME(P) \
    template <> const char *prog_name<P##Tag>() { return #P; }
SCINT_PROG_NAME(ProgNoise)
SCINT_PROG_NAME(ProgNoiseSwap)
SCINT_PROG_NAME(ProgScreen)
SCINT_PROG_NAME(ProgScreenProp)
SCINT_PROG_NAME(ProgPhaseProp)
SCINT_PROG_NAME(ProgPropIntensity)
SCINT_PROG_NAME(ProgRealFwd)
SCINT_PROG_NAME(ProgFwdRe)
SCINT_PROG_NAME(ProgSmearMid)
SCINT_PROG_NAME(ProgInvRe)
SCINT_PROG_NAME(ProgVjpY)
SCINT_PROG_NAME(ProgPropField)
SCINT_PROG_NAME(ProgVjpYField)
SCINT_PROG_NAME(ProgVjpX)
SCINT_PROG_NAME(ProgApertureX)
SCINT_PROG_NAME(ProgAbs2)
SCINT_PROG_NAME(ProgNoiseT)
SCINT_PROG_NAME(ProgNoiseSwapT)
SCINT_PROG_NAME(ProgPhasePropT)
SCINT_PROG_NAME(ProgPropIntensityT)
SCINT_PROG_NAME(ProgRealFwdT)
SCINT_PROG_NAME(ProgSmearMidT)
SCINT_PROG_NAME(ProgInvReT)
#undef SCINT_PROG_NAME

int plan_variant(int N, int dtype, int *V, hipStream_t stream);

template <class Tag> int run_row(int dtype, int N, const RowProgram &p, int n_ops, hipStream_t stream) {
    int V = 0;
    if (int rc = plan_variant(N, dtype, &V, stream)) return rc;
    const void *tw = nullptr;
    if (int rc = get_twiddles(N, V, dtype, &tw, stream)) return rc;
    hipEvent_t t0 = nullptr;
    const bool timed = timing_begin(stream, &t0);
    hipError_t e = dtype == PS_F64 ? launch_row<double, Tag>(N, V, p, tw, stream)
                                   : launch_row<float, Tag>(N, V, p, tw, stream);
    if (e != hipSuccess) return fail(PS_E_DEVICE, std::string("row pass launch: ") + hipGetErrorString(e));
    if (timed)
        timing_end(stream, t0,
                   std::string("row_") + prog_name<Tag>() + "_" + real_name(dtype) + "_N" + std::to_string(N),
                   row_bytes(p, n_ops, dtype, true), row_bytes(p, n_ops, dtype, false), row_flops(p, n_ops));
    return PS_OK;
}

// Elements of the N x N matrices that side-transpose units [u0, u1) cover
// (units of 64 rows by 128 columns, ragged at the right and bottom edges).
double side_elements(const RowSide &sd, int N) {
    const int nx = transpose_units_x(N), ny = transpose_units_y(N);
    const int64_t per = (int64_t)nx * ny;
    auto unit_elems = [&](int64_t u) {
        const int rem = (int)(u % per), uy = rem / nx, ux = rem - uy * nx;
        return (double)std::min(kTransposeUnitRows, N - uy * kTransposeUnitRows) *
               (double)std::min(kTransposeUnitCols, N - ux * kTransposeUnitCols);
    };
    double e = 0.0;
    int64_t u = sd.u0;
    for (; u < sd.u1 && u % per; ++u) e += unit_elems(u);          // head of a partial matrix
    const int64_t whole = (sd.u1 - u) / per;                        // whole matrices
    e += (double)whole * N * N;
    for (u += whole * per; u < sd.u1; ++u) e += unit_elems(u);      // tail
    return e;
}

// Row pass whose launch also runs the transposes of p.side (FP32 programs
// only).  Its timing entry counts their bytes among the schedule's (each
// element read once and written once), not among the algorithmic ones.
template <class Tag> int run_row_side(int N, const RowProgram &p, int n_ops, hipStream_t stream) {
    int V = 0;
    if (int rc = plan_variant(N, PS_F32, &V, stream)) return rc;
    const void *tw = nullptr;
    if (int rc = get_twiddles(N, V, PS_F32, &tw, stream)) return rc;
    hipEvent_t t0 = nullptr;
    const bool timed = timing_begin(stream, &t0);
    hipError_t e = launch_row<float, Tag>(N, V, p, tw, stream);
    if (e != hipSuccess) return fail(PS_E_DEVICE, std::string("row pass launch: ") + hipGetErrorString(e));
    if (timed)
        timing_end(stream, t0, std::string("row_") + prog_name<Tag>() + "_f32_N" + std::to_string(N),
                   row_bytes(p, n_ops, PS_F32, true),
                   row_bytes(p, n_ops, PS_F32, false) + 16.0 * side_elements(p.side, N), row_flops(p, n_ops));
    return PS_OK;
}

// ------------------------------------------------------------ plan tuner
// The large FP32 sizes have several compiled Stockham plans (fft_plan.hpp).
// On the first FP32 call of such a size on a device, each plan is timed on a
// propagation row pass (FFT, chirp multiply, inverse FFT, |.|^2, 32 iterations)
// over 2^24 points of scratch data, on a private stream; the fastest is kept,
// unless it beats plan 0 by less than 3% (stable choices across runs).
// SCINT_PLAN_VARIANT=<v> in the environment, or ps_set_plan_variant, pins it.
int tune_plan(int N, std::vector<float> *ms_out, int *best) {
    const int nv = plan_variants(N);
    // about 2^24 points per launch (several waves of workgroups at every
    // size) and 32 wavelength iterations, as in a polychromatic pass: with
    // only 4, the once-per-workgroup setup (the LDS twiddle cache) weighed
    // enough to rank near-equal plans against what the full passes measure
    const int rows = std::max(1024, (1 << 24) / N), iters = 32;
    const size_t cb = (size_t)rows * N * 8;
    void *buf = nullptr;
    if (hipMalloc(&buf, cb + (size_t)rows * N * 4 + (size_t)iters * N * 8 + 1024) != hipSuccess)
        return fail(PS_E_ALLOC, "hipMalloc of tuner scratch failed");
    char *S = static_cast<char *>(buf);
    char *Sr = S + cb;
    char *H = Sr + (size_t)rows * N * 4;
    hipStream_t s = nullptr;
    int rc = PS_OK;
    if (hipStreamCreate(&s) != hipSuccess) rc = fail(PS_E_DEVICE, "hipStreamCreate for the tuner failed");
    hipEvent_t a = nullptr, b = nullptr;
    if (!rc && (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess))
        rc = fail(PS_E_DEVICE, "hipEventCreate for the tuner failed");
    if (!rc && hipMemsetAsync(buf, 0, cb + (size_t)rows * N * 4 + (size_t)iters * N * 8, s) != hipSuccess)
        rc = fail(PS_E_DEVICE, "tuner scratch clear failed");
    ProgBuilder p(N, rows);
    p.p.n_iter = iters;
    p.op(ROP_LOOP)
        .op(ROP_LOAD_C, S, (int64_t)N * N, N)
        .op(ROP_FFT_FWD)
        .op(ROP_MUL_TAB, H, 0, 0, N)
        .op(ROP_FFT_INV)
        .op(ROP_ACC_ABS2U)
        .op(ROP_ENDLOOP)
        .op(ROP_STORE_ACC, Sr, (int64_t)N * N, N);  // row g at g N: inside the scratch
    // rounds over all variants in turn (so drift affects them alike); the
    // first round warms up, then the minimum over the timed rounds counts
    ms_out->assign(nv, 1e30f);
    std::vector<const void *> tws(nv, nullptr);
    for (int v = 0; v < nv && !rc; ++v) rc = get_twiddles(N, v, PS_F32, &tws[v], s);
    for (int r = 0; r < 6 && !rc; ++r) {
        for (int v = 0; v < nv && !rc; ++v) {
            (void)hipEventRecord(a, s);
            hipError_t e = launch_row<float, ProgPropIntensityTag>(N, v, p.p, tws[v], s);
            (void)hipEventRecord(b, s);
            if (e != hipSuccess || hipEventSynchronize(b) != hipSuccess) {
                rc = fail(PS_E_DEVICE, "tuner launch failed");
                break;
            }
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, a, b);
            if (r > 0) (*ms_out)[v] = std::min((*ms_out)[v], ms);
        }
    }
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (s) (void)hipStreamDestroy(s);
    (void)hipFree(buf);
    if (rc) return rc;
    int bv = 0;
    for (int v = 1; v < nv; ++v)
        if ((*ms_out)[v] < (*ms_out)[bv]) bv = v;
    if (bv != 0 && (*ms_out)[bv] > 0.97f * (*ms_out)[0]) bv = 0;
    *best = bv;
    return PS_OK;
}

int plan_variant(int N, int dtype, int *V, hipStream_t stream) {
    *V = 0;
    if (dtype == PS_F64 || plan_variants(N) == 1) return PS_OK;
    int dev;
    if (int rc = current_device(&dev)) return rc;
    const auto key = std::make_pair(N, dtype);
    {
        std::lock_guard<std::mutex> lock(g_mutex);
        auto &dc = g_cache[dev];
        auto it = dc.variant.find(key);
        if (it != dc.variant.end()) {
            *V = it->second;
            return PS_OK;
        }
    }
    int chosen = -1;
    if (const char *env = std::getenv("SCINT_PLAN_VARIANT")) {
        const int v = std::atoi(env);
        if (v >= 0 && v < plan_variants(N)) chosen = v;
    }
    std::vector<float> ms;
    if (chosen < 0) {
        if (int rc = refuse_in_capture(stream, "tuning the FFT plan of this size")) return rc;
        if (int rc = tune_plan(N, &ms, &chosen)) return rc;
    }
    std::lock_guard<std::mutex> lock(g_mutex);
    auto &dc = g_cache[dev];
    dc.variant[key] = chosen;
    if (!ms.empty()) dc.variant_ms[key] = ms;
    *V = chosen;
    return PS_OK;
}

int transpose(const void *in, void *out, int N, int64_t nbatch, int elem_bytes, hipStream_t stream) {
    hipEvent_t t0 = nullptr;
    const bool timed = timing_begin(stream, &t0);
    HIP_TRY(launch_transpose(in, out, N, nbatch, elem_bytes, stream));
    if (timed)
        timing_end(stream, t0, "transpose_" + std::to_string(elem_bytes) + "B_N" + std::to_string(N), 0.0,
                   2.0 * elem_bytes * (double)N * N * (double)nbatch, 0.0);
    return PS_OK;
}

// Chirp tables H1(k)/N for n wavelengths with Fresnel radii rho[j] pixels.
// amp (optional, one per wavelength) multiplies each table.
int chirp_tables(void *tab, int N, const std::vector<double> &rho, int dtype, bool normalise, hipStream_t stream,
                 const std::vector<double> *amp = nullptr) {
    const int n = (int)rho.size();
    for (int j0 = 0; j0 < n; j0 += 64) {
        const int m = std::min(64, n - j0);
        double a[64];
        for (int j = 0; j < m; ++j) a[j] = kPiD * rho[j0 + j] * rho[j0 + j] / ((double)N * (double)N);
        char *base = static_cast<char *>(tab) + (size_t)j0 * N * 2 * real_bytes(dtype);
        HIP_TRY(launch_chirp_tables(base, N, a, m, normalise ? 1.0 / N : 1.0, dtype == PS_F64, stream,
                                    amp ? amp->data() + j0 : nullptr));
    }
    return PS_OK;
}

// Weights of the co-added intensities carried by the chirp tables: both 1-D
// passes multiply by the table of wavelength j, so a factor w_j^(1/4) in it
// scales the field by sqrt(w_j) and its |.|^2 by w_j, and the accumulation
// needs no product by the weight.
static std::vector<double> weight_amps(const std::vector<double> &w, size_t j0, size_t m) {
    std::vector<double> a(m);
    for (size_t j = 0; j < m; ++j) a[j] = std::sqrt(std::sqrt(w[j0 + j]));
    return a;
}

double f_beta(double beta) { return std::pow(2.0, -beta) * beta * std::tgamma(-beta / 2.0) / std::tgamma(beta / 2.0); }

// Fills the noise operands: amp0 = sqrt(C_beta R^(2-beta)) N^(beta/2) / N.
// FP32 screens leave the lowest modes to the FP64 synthesis (low_k).
void set_noise(RowProgram &p, int N, double R, double beta, uint64_t seed, uint32_t r0, int dtype) {
    const double c_beta = 1.0 / (2.0 * std::pow(2.0 * kPiD, beta - 1.0) * f_beta(beta));
    p.amp0 = std::sqrt(c_beta * std::pow(R, 2.0 - beta)) * std::pow((double)N, beta / 2.0) / (double)N;
    p.neg_beta_4 = -beta / 4.0;
    p.seed_lo = (uint32_t)(seed & 0xFFFFFFFFull);
    p.seed_hi = (uint32_t)(seed >> 32);
    p.r0 = (int32_t)r0;
    p.low_k = dtype == PS_F32 ? low_modes_k_of(N) : 0;
}

int64_t nn(int N) { return (int64_t)N * N; }

// Workspace of the FP64 low-mode tables of nb FP32 screens (0 for FP64).
size_t low_mode_bytes(int N, int nb, int dtype) {
    if (dtype != PS_F32) return 0;
    const size_t K = (size_t)low_modes_k_of(N), W = 2 * K + 1;
    return (size_t)nb * ((size_t)N * (K + 1) + W * W) * 16 + 512;
}

// The FP64 low modes of FP32 screens r0 .. r0 + nb - 1 (Sect. 3.1): the FP32
// transforms carry the Fourier modes outside the square |kx'|, |ky'| <= K,
// and the second screen pass adds the square's part, summed in FP64 from the
// row table built here at `tab` (low_mode_bytes of workspace), to the
// screen.  Sets p.low_k and p.low_tab of that pass (nothing for FP64).  With
// swap the table serves screens made transposed ([b][x][y]; screen_passes
// with swap).
int low_mode_pass(RowProgram &p, int N, double R, double beta, uint64_t seed, uint32_t r0, int nb, int dtype,
                  void *tab, hipStream_t stream, bool swap) {
    if (dtype != PS_F32) return PS_OK;
    RowProgram q;
    std::memset(&q, 0, sizeof(q));
    set_noise(q, N, R, beta, seed, r0, dtype);
    const int K = q.low_k;
    char *G = static_cast<char *>(tab);
    char *C = G + (size_t)nb * N * (K + 1) * 16;
    HIP_TRY(launch_low_modes(C, G, N, K, nb, r0, q.seed_lo, q.seed_hi, q.amp0, q.neg_beta_4, stream, swap));
    p.low_k = K;
    p.low_tab = G;
    return PS_OK;
}

// Upper bound on workspace bytes a call plans for (whole-batch processing is
// split into chunks above it): a quarter of the free device memory at the
// first call on the device, at most 32 GiB, unless ps_set_workspace_budget
// set it (a caller that owns the GPU can give more: the pipelined jobs of 32
// wavelengths of an 8192^2 screen take 64 GiB, 3 % faster per batch than the
// 8-wavelength jobs of the default).
// Fixed afterwards, so that a given call always takes the same chunking (and
// no call queries the device again).
size_t workspace_budget() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return (size_t)8 << 30;
    std::lock_guard<std::mutex> lock(g_mutex);
    auto &dc = g_cache[dev];
    if (dc.budget == 0) {
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) free_b = (size_t)16 << 30;
        dc.budget = std::max<size_t>((size_t)1 << 30, std::min<size_t>((size_t)32 << 30, free_b / 4));
    }
    return dc.budget;
}

// ------------------------------------------------------------ pipelines
// Interleaving of the pipelined propagation below: the share of each job's
// transpose units carried by the next job's x pass (the rest rides on the y
// pass two jobs back), and per pass the row workgroups and transpose
// workgroups of one group of the grid.  Measured at 8192^2 x 32 wavelengths
// on the MI355X (step times within 1 %: shares of 0.5 to 1 on the x pass;
// groups of 16 + 4, 32 + 8 or 64 + 16 row + transpose workgroups, i.e. 128
// units per transpose workgroup; 12-16 % slower: 1 : 1 and 3 : 1 groups):
// the x pass takes all of a job's transposes (the y pass only the last
// job's), in groups of 32 + 8.  SCINT_PIPELINE=0 in the environment turns
// the pipeline off; SCINT_SIDE_SPLIT=<f> and SCINT_SIDE_GROUPS=
// <rows_x>:<side_x>:<rows_y>:<side_y> override the defaults.  The screen
// passes split a batch into up to screen_jobs jobs (SCINT_SCREEN_JOBS=<n>;
// 1 turns that pipeline off).  The x passes of the pipelined propagation
// give each row two workgroups, each taking half of the wavelengths, so that
// the phase row both re-read for every wavelength is fetched from one L2
// (measured at 8192^2 x 32 wavelengths, per x pass with transposes: 10.29
// against 10.45 ms on one MI355X, equal on another); SCINT_ITER_SPLIT=1
// keeps one workgroup per row.
struct SideCfg {
    bool on = true;
    double split = 1.0;
    int fft_x = 32, side_x = 8, fft_y = 32, side_y = 8;
    int screen_jobs = 4;
    int iter_split = 2;
};
static SideCfg side_cfg() {
    SideCfg c;
    if (const char *e = std::getenv("SCINT_PIPELINE")) c.on = std::atoi(e) != 0;
    if (const char *e = std::getenv("SCINT_SIDE_SPLIT")) {
        const double v = std::atof(e);
        if (v >= 0.0 && v <= 1.0) c.split = v;
    }
    if (const char *e = std::getenv("SCINT_ITER_SPLIT")) {
        const int v = std::atoi(e);
        if (v == 1 || v == 2) c.iter_split = v;
    }
    if (const char *e = std::getenv("SCINT_SCREEN_JOBS")) {
        const int v = std::atoi(e);
        if (v >= 1 && v <= 64) c.screen_jobs = v;
    }
    if (const char *e = std::getenv("SCINT_SIDE_GROUPS")) {
        int a = 0, b = 0, d = 0, f = 0;
        if (std::sscanf(e, "%d:%d:%d:%d", &a, &b, &d, &f) == 4 && a >= 1 && b >= 1 && d >= 1 && f >= 1 &&
            a <= 1024 && b <= 1024 && d <= 1024 && f <= 1024) {
            c.fft_x = a;
            c.side_x = b;
            c.fft_y = d;
            c.side_y = f;
        }
    }
    return c;
}

// The first pass of the screens of nb realisations (noise, spectral filter,
// inverse DFT along rows) into W1 and its transpose into W2, both complex
// [nb][N][N].  In FP32 from N = 2048 the batch is split into up to
// screen_jobs jobs of consecutive realisations: the noise pass of job k
// carries the transpose of job k-1 as extra workgroups (its arithmetic-bound
// FFTs leave memory bandwidth free), and only the last job's transpose runs
// on its own.  Each element is computed by the same kernel code either way,
// so the results do not depend on the split.  With swap the first pass runs
// along kx instead (rows ky), so that the second pass makes the screens
// transposed, [b][x][y].
int screen_passes(int N, double R, double beta, uint64_t seed, uint32_t r0, int nb, int dtype, void *W1, void *W2,
                  hipStream_t stream, bool swap) {
    const SideCfg sc = side_cfg();
    const int J = (dtype == PS_F32 && N >= 2048 && sc.on) ? std::min(nb, sc.screen_jobs) : 1;
    const size_t cbytes = (size_t)nn(N) * 2 * real_bytes(dtype);
    const int64_t upm = (int64_t)transpose_units_x(N) * transpose_units_y(N);
    int prev0 = 0, prev_n = 0;  // realisations of the previous job
    for (int k = 0; k < J; ++k) {
        const int j0 = (int)((int64_t)nb * k / J), jn = (int)((int64_t)nb * (k + 1) / J) - j0;
        ProgBuilder a(N, (int64_t)jn * N);
        set_noise(a.p, N, R, beta, seed, r0 + (uint32_t)j0, dtype);
        if (k > 0) a.op(ROP_SIDE_T);
        a.op(swap ? ROP_NOISE_SWAP : ROP_NOISE)
            .op(ROP_FFT_INV)
            .op(ROP_STORE_C, static_cast<char *>(W1) + j0 * cbytes, nn(N), N);
        if (k == 0) {
            const int rc = swap ? run_row<ProgNoiseSwapTag>(dtype, N, a.p, a.n, stream)
                                : run_row<ProgNoiseTag>(dtype, N, a.p, a.n, stream);
            if (rc) return rc;
        } else {
            RowSide &sd = a.p.side;
            sd.in = static_cast<char *>(W1) + prev0 * cbytes;
            sd.out = static_cast<char *>(W2) + prev0 * cbytes;
            sd.u0 = 0;
            sd.u1 = upm * prev_n;
            sd.fft_blocks = sc.fft_x;
            sd.side_blocks = sc.side_x;
            const int rc = swap ? run_row_side<ProgNoiseSwapTTag>(N, a.p, a.n, stream)
                                : run_row_side<ProgNoiseTTag>(N, a.p, a.n, stream);
            if (rc) return rc;
        }
        prev0 = j0;
        prev_n = jn;
    }
    return transpose(static_cast<char *>(W1) + prev0 * cbytes, static_cast<char *>(W2) + prev0 * cbytes, N, prev_n,
                     2 * (int)real_bytes(dtype), stream);
}

// Second propagation pass of nb screens (rows x of the transposed field W2:
// DFT along y, chirp, inverse DFT, |.|^2 into Iacc, transposed layout; for
// screens made transposed, the same along x on rows y, natural layout).  With
// F non-NULL the field A itself is kept there too, [b][x][y] complex, as the
// adjoint's checkpoint.
int prop_y_pass(int N, int dtype, int nb, const void *W2, const void *H, void *Iacc, void *F, hipStream_t stream) {
    ProgBuilder d(N, (int64_t)nb * N);
    if (F) {
        d.op(ROP_LOAD_C, W2, nn(N), N)
            .op(ROP_FFT_FWD)
            .op(ROP_MUL_TAB, H)
            .op(ROP_FFT_INV)
            .op(ROP_STORE_C, F, nn(N), N)
            .op(ROP_ACC_ABS2U)
            .op(ROP_STORE_ACC, Iacc, nn(N), N);
        return run_row<ProgPropFieldTag>(dtype, N, d.p, d.n, stream);
    }
    d.op(ROP_LOOP)
        .op(ROP_LOAD_C, W2, nn(N), N)
        .op(ROP_FFT_FWD)
        .op(ROP_MUL_TAB, H)
        .op(ROP_FFT_INV)
        .op(ROP_ACC_ABS2U)
        .op(ROP_ENDLOOP)
        .op(ROP_STORE_ACC, Iacc, nn(N), N);
    return run_row<ProgPropIntensityTag>(dtype, N, d.p, d.n, stream);
}

// ------------------------------------------------------------ no-allocation path
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void *g_scratch[kMaxDevices];  // device address of `scratch` per GPU, set on first use

// The scratch array's device address on the current GPU: looked up once per
// device (the first call there), then read from g_scratch.
int noalloc_scratch(void **out) {
    int dev;
    if (int rc = current_device(&dev)) return rc;
    if (dev < 0 || dev >= kMaxDevices) return fail(PS_E_DEVICE, "device ordinal beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(PS_E_DEVICE, std::string("hipGetSymbolAddress of the scratch array: ") + hipGetErrorString(e));
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return PS_OK;
}

// Row pass with plan 0 and a given twiddle table: kernels only (no tuning,
// no table cache, no timing events).
template <class Tag> int launch_row_plan0(int dtype, int N, const RowProgram &p, const void *tw, hipStream_t stream) {
    const hipError_t e = dtype == PS_F64 ? launch_row<double, Tag>(N, 0, p, tw, stream)
                                         : launch_row<float, Tag>(N, 0, p, tw, stream);
    if (e != hipSuccess) return fail(PS_E_DEVICE, std::string("row pass launch: ") + hipGetErrorString(e));
    return PS_OK;
}

}  // namespace

// ============================================================ C ABI
extern "C" {

int ps_version(void) { return 10100; }

int ps_num_plan_variants(int N, int dtype) {
    if (dtype == PS_F64) return supported_f64(N) ? 1 : 0;
    if (dtype == PS_F32) return supported_f32(N) ? plan_variants(N) : 0;
    return 0;
}

int ps_plan_variant(int N, int dtype, int *variant_out, float *ms_out) {
    g_last_error.clear();
    if (int rc = check_common(N, dtype, 1)) return rc;
    if (!variant_out) return fail(PS_E_NULL, "variant_out is NULL");
    int V = 0;
    if (int rc = plan_variant(N, dtype, &V, nullptr)) return rc;
    *variant_out = V;
    if (ms_out) {
        int dev = 0;
        (void)hipGetDevice(&dev);
        std::lock_guard<std::mutex> lock(g_mutex);
        auto &dc = g_cache[dev];
        auto it = dc.variant_ms.find(std::make_pair(N, dtype));
        const int nv = ps_num_plan_variants(N, dtype);
        for (int v = 0; v < nv; ++v)
            ms_out[v] = (it != dc.variant_ms.end() && v < (int)it->second.size()) ? it->second[v] : -1.0f;
    }
    return PS_OK;
}

int ps_set_plan_variant(int N, int dtype, int variant) {
    g_last_error.clear();
    if (int rc = check_common(N, dtype, 1)) return rc;
    if (variant < -1 || variant >= ps_num_plan_variants(N, dtype))
        return fail(PS_E_PARAM, "plan variant out of range");
    int dev;
    if (int rc = current_device(&dev)) return rc;
    std::lock_guard<std::mutex> lock(g_mutex);
    auto &dc = g_cache[dev];
    if (variant < 0)
        dc.variant.erase(std::make_pair(N, dtype));
    else
        dc.variant[std::make_pair(N, dtype)] = variant;
    return PS_OK;
}

int ps_tune_plans(int N, int dtype) {
    g_last_error.clear();
    if (int rc = check_common(N, dtype, 1)) return rc;
    int V = 0;
    if (int rc = plan_variant(N, dtype, &V, nullptr)) return rc;
    const void *tw = nullptr;
    return get_twiddles(N, V, dtype, &tw, nullptr);
}

int ps_set_workspace_budget(size_t bytes) {
    g_last_error.clear();
    if (bytes != 0 && bytes < ((size_t)64 << 20)) return fail(PS_E_PARAM, "workspace budget below 64 MiB");
    int dev;
    if (int rc = current_device(&dev)) return rc;
    std::lock_guard<std::mutex> lock(g_mutex);
    g_cache[dev].budget = bytes;  // 0: the default, taken again at the next call
    return PS_OK;
}

int ps_timing_enable(int on) {
    timing_drain();
    std::lock_guard<std::mutex> lock(g_timing_mutex);
    if (on) g_totals.clear();
    g_timing_on = on != 0;
    return PS_OK;
}

int ps_timing_count(void) {
    timing_drain();
    std::lock_guard<std::mutex> lock(g_timing_mutex);
    return (int)g_totals.size();
}

int ps_timing_entry(int i, char *name_buf, int buf_len, double *total_ms, long long *launches, double *bytes,
                    double *schedule_bytes, double *flops) {
    std::lock_guard<std::mutex> lock(g_timing_mutex);
    if (i < 0 || i >= (int)g_totals.size()) return fail(PS_E_SIZE, "timing entry index out of range");
    auto it = g_totals.begin();
    std::advance(it, i);
    if (name_buf && buf_len > 0) {
        std::strncpy(name_buf, it->first.c_str(), (size_t)buf_len - 1);
        name_buf[buf_len - 1] = '\0';
    }
    if (total_ms) *total_ms = it->second.ms;
    if (launches) *launches = it->second.launches;
    if (bytes) *bytes = it->second.bytes;
    if (schedule_bytes) *schedule_bytes = it->second.sched_bytes;
    if (flops) *flops = it->second.flops;
    return PS_OK;
}

const char *ps_last_error(void) { return g_last_error.c_str(); }
const char *ps_last_warning(void) { return g_last_warning.c_str(); }

int ps_supported_size(int N, int dtype) {
    if (dtype == PS_F64) return supported_f64(N) ? 1 : 0;
    if (dtype == PS_F32) return supported_f32(N) ? 1 : 0;
    return 0;
}

int ps_num_supported_sizes(int dtype) {
    if (dtype != PS_F32 && dtype != PS_F64) return 0;
    return (int)size_list(dtype).size();
}

int ps_supported_size_at(int dtype, int i) {
    if (dtype != PS_F32 && dtype != PS_F64) return 0;
    auto v = size_list(dtype);
    return (i >= 0 && i < (int)v.size()) ? v[i] : 0;
}

int ps_release_cache(void) {
    std::lock_guard<std::mutex> lock(g_mutex);
    int prev = -1;
    (void)hipGetDevice(&prev);
    for (auto &kv : g_cache) {
        (void)hipSetDevice(kv.first);
        (void)hipDeviceSynchronize();
        for (auto &t : kv.second.twiddles) (void)hipFree(t.second);
        for (auto &d : kv.second.disks) (void)hipFree(d.second);
        for (auto &w : kv.second.workspace)
            if (w.second.first) (void)hipFree(w.second.first);
    }
    g_cache.clear();
    if (prev >= 0) (void)hipSetDevice(prev);
    return PS_OK;
}

int ps_generate(int N, double delta, double r_diff, double beta, uint64_t seed, uint32_t first_realisation,
                int n_real, int dtype, void *phi_out, void *hip_stream) {
    g_last_error.clear();
    g_last_warning.clear();
    if (int rc = check_common(N, dtype, n_real)) return rc;
    if (!phi_out) return fail(PS_E_NULL, "phi_out is NULL");
    if (int rc = check_aligned({phi_out})) return rc;
    if (!finite_pos(delta) || !finite_pos(r_diff)) return fail(PS_E_PARAM, "delta and r_diff must be finite and > 0");
    if (!(std::isfinite(beta) && beta > 2.0 && beta < 4.0)) return fail(PS_E_PARAM, "beta must lie in (2, 4)");
    if (delta >= r_diff / 2.0) g_last_warning = "pixel side >= R_diff/2: the phase variations are undersampled";
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    const size_t cbytes = (size_t)nn(N) * 2 * real_bytes(dtype);
    const int nb_max = (int)std::max<size_t>(1, workspace_budget() / (2 * cbytes));
    for (int b0 = 0; b0 < n_real; b0 += nb_max) {
        const int nb = std::min(nb_max, n_real - b0);
        const uint32_t r0 = first_realisation + (uint32_t)b0;
        void *ws = nullptr;
        if (int rc = get_workspace(stream, 2 * cbytes * nb + low_mode_bytes(N, nb, dtype) + 1024, &ws)) return rc;
        Carver c;
        char *base = static_cast<char *>(ws);
        void *W1 = base + c.take(cbytes * nb);
        void *W2 = base + c.take(cbytes * nb);
        void *LT = base + c.take(low_mode_bytes(N, nb, dtype));
        if (int rc = screen_passes(N, r_diff / delta, beta, seed, r0, nb, dtype, W1, W2, stream, false)) return rc;
        ProgBuilder b(N, (int64_t)nb * N);
        if (int rc = low_mode_pass(b.p, N, r_diff / delta, beta, seed, r0, nb, dtype, LT, stream, false)) return rc;
        char *phi = static_cast<char *>(phi_out) + (size_t)b0 * nn(N) * real_bytes(dtype);
        b.op(ROP_LOAD_C, W2, nn(N), N).op(ROP_FFT_INV).op(ROP_SQRT2RE).op(ROP_STORE_R, phi, nn(N), N, 0, 0, 1.0);
        if (int rc = run_row<ProgScreenTag>(dtype, N, b.p, b.n, stream)) return rc;
    }
    return PS_OK;
}

int ps_screen_fresnel(int N, double delta, double r_diff, double beta, uint64_t seed, uint32_t first_realisation,
                      int n_real, double lambda, double z, int dtype, void *phi_out, void *I_out, void *field_out,
                      void *hip_stream) {
    g_last_error.clear();
    g_last_warning.clear();
    if (int rc = check_common(N, dtype, n_real)) return rc;
    if (!I_out) return fail(PS_E_NULL, "I_out is NULL");
    if (int rc = check_aligned({I_out, phi_out, field_out})) return rc;
    if (!finite_pos(delta) || !finite_pos(r_diff) || !finite_pos(lambda) || !finite_pos(z))
        return fail(PS_E_PARAM, "delta, r_diff, lambda and z must be finite and > 0");
    if (!(std::isfinite(beta) && beta > 2.0 && beta < 4.0)) return fail(PS_E_PARAM, "beta must lie in (2, 4)");
    const size_t rbytes = (size_t)nn(N) * real_bytes(dtype) * n_real;
    if (phi_out && overlaps(phi_out, rbytes, I_out, rbytes)) return fail(PS_E_ALIAS, "phi_out overlaps I_out");
    if (field_out && (overlaps(field_out, 2 * rbytes, I_out, rbytes) ||
                      (phi_out && overlaps(field_out, 2 * rbytes, phi_out, rbytes))))
        return fail(PS_E_ALIAS, "field_out overlaps I_out or phi_out");
    if (delta >= r_diff / 2.0) g_last_warning = "pixel side >= R_diff/2: the phase variations are undersampled";
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    const double rho = std::sqrt(lambda * z / (2.0 * kPiD)) / delta;
    const size_t cbytes = (size_t)nn(N) * 2 * real_bytes(dtype);
    const size_t tbytes = (size_t)N * 2 * real_bytes(dtype);
    const int nb_max = (int)std::max<size_t>(1, workspace_budget() / (2 * cbytes));
    for (int b0 = 0; b0 < n_real; b0 += nb_max) {
        const int nb = std::min(nb_max, n_real - b0);
        const uint32_t r0 = first_realisation + (uint32_t)b0;
        void *ws = nullptr;
        if (int rc = get_workspace(stream, 2 * cbytes * nb + tbytes + low_mode_bytes(N, nb, dtype) + 1536, &ws))
            return rc;
        Carver c;
        char *base = static_cast<char *>(ws);
        void *W1 = base + c.take(cbytes * nb);
        void *W2 = base + c.take(cbytes * nb);
        void *H = base + c.take(tbytes);
        void *LT = base + c.take(low_mode_bytes(N, nb, dtype));
        if (int rc = chirp_tables(H, N, {rho}, dtype, true, stream)) return rc;
        // Without the screen and the field to return, the screens are made
        // transposed ([b][x][y]: the first pass along kx), the first
        // propagation pass runs along y and the second along x, so that the
        // pattern comes out of it in the natural layout and needs no final
        // transpose.  With either returned, the natural order (screen rows y,
        // the field's checkpoint layout [b][x][y]).
        const bool swap = !phi_out && !field_out;
        if (int rc = screen_passes(N, r_diff / delta, beta, seed, r0, nb, dtype, W1, W2, stream, swap)) return rc;
        char *phi = phi_out ? static_cast<char *>(phi_out) + (size_t)b0 * nn(N) * real_bytes(dtype) : nullptr;
        ProgBuilder b(N, (int64_t)nb * N);
        if (int rc = low_mode_pass(b.p, N, r_diff / delta, beta, seed, r0, nb, dtype, LT, stream, swap)) return rc;
        b.op(ROP_LOAD_C, W2, nn(N), N)
            .op(ROP_FFT_INV)
            .op(ROP_SQRT2RE)
            .op(ROP_STORE_R, phi, nn(N), N, 0, 0, 1.0)
            .op(ROP_EXP_RE, nullptr, 0, 0, 0, 0, 1.0)
            .op(ROP_FFT_FWD)
            .op(ROP_MUL_TAB, H)
            .op(ROP_FFT_INV)
            .op(ROP_STORE_C, W1, nn(N), N);
        if (int rc = run_row<ProgScreenPropTag>(dtype, N, b.p, b.n, stream)) return rc;
        if (int rc = transpose(W1, W2, N, nb, 2 * (int)real_bytes(dtype), stream)) return rc;
        char *F = field_out ? static_cast<char *>(field_out) + (size_t)b0 * cbytes : nullptr;
        char *I = static_cast<char *>(I_out) + (size_t)b0 * nn(N) * real_bytes(dtype);
        if (swap) {
            if (int rc = prop_y_pass(N, dtype, nb, W2, H, I, nullptr, stream)) return rc;
            continue;
        }
        if (int rc = prop_y_pass(N, dtype, nb, W2, H, W1, F, stream)) return rc;
        if (int rc = transpose(W1, I, N, nb, (int)real_bytes(dtype), stream)) return rc;
    }
    return PS_OK;
}

// Propagation of nb screens for a chunk of wavelengths: intensities summed
// with the given weights into Iacc (transposed layout [b][x][y]); add != 0
// accumulates onto Iacc.
static int poly_chunk(int N, const void *phi, int nb, const std::vector<double> &rho,
                      const std::vector<double> &scale, const std::vector<double> &weight, int dtype, void *W1,
                      void *W2, void *H, void *Iacc, bool add, hipStream_t stream) {
    const int C = (int)rho.size();
    const std::vector<double> amp = weight_amps(weight, 0, C);
    if (int rc = chirp_tables(H, N, rho, dtype, true, stream, &amp)) return rc;
    ProgBuilder a(N, (int64_t)nb * N);
    a.p.n_iter = C;
    for (int j = 0; j < C; ++j) a.p.scale[j] = scale[j];
    a.op(ROP_LOOP)
        .op(ROP_LOAD_PHASE, phi, nn(N), N, 0, RF_ITER_SCALE)
        .op(ROP_FFT_FWD)
        .op(ROP_MUL_TAB, H, 0, 0, N)
        .op(ROP_FFT_INV)
        .op(ROP_STORE_C, W1, nn(N), N, (int64_t)nb * nn(N))
        .op(ROP_ENDLOOP);
    if (int rc = run_row<ProgPhasePropTag>(dtype, N, a.p, a.n, stream)) return rc;
    if (int rc = transpose(W1, W2, N, (int64_t)nb * C, 2 * (int)real_bytes(dtype), stream)) return rc;
    ProgBuilder b(N, (int64_t)nb * N);
    b.p.n_iter = C;
    b.op(ROP_LOOP)
        .op(ROP_LOAD_C, W2, nn(N), N, (int64_t)nb * nn(N))
        .op(ROP_FFT_FWD)
        .op(ROP_MUL_TAB, H, 0, 0, N)
        .op(ROP_FFT_INV)
        .op(ROP_ACC_ABS2U)
        .op(ROP_ENDLOOP)
        .op(ROP_STORE_ACC, Iacc, nn(N), N, 0, add ? RF_ADD : 0);
    return run_row<ProgPropIntensityTag>(dtype, N, b.p, b.n, stream);
}

// One job of the polychromatic propagation: nb realisations from b0, m
// wavelengths from j0.
struct PolyJob {
    int b0, nb, j0, m;
};

// Pipelined polychromatic propagation (FP32).  Each job runs the x pass
// (exp(i s phi), DFT, chirp, IDFT per wavelength) into a raw field buffer,
// the transpose of that buffer, and the y pass (DFT, chirp, IDFT, weighted
// |.|^2 summed into Iacc).  Step k launches the x pass of job k, then the y
// pass of job k-2; the transpose of job k-1 rides on these two launches as
// extra workgroups (split by SideCfg), so its memory traffic overlaps their
// FFT arithmetic.  Two raw and two transposed buffers alternate between
// jobs and three chirp tables between the jobs in flight; the kernels and
// the order of every sum are those of the plain chunk loop, so the results
// are the same bit for bit for the same chunking.
static int poly_pipelined(int N, const char *phi_ref, const std::vector<PolyJob> &jobs, int C, int nb_max,
                          int n_lambda, const std::vector<double> &rho, const std::vector<double> &scale,
                          const std::vector<double> &weight, void *I_out, const SideCfg &sc, hipStream_t stream) {
    const size_t cbytes = (size_t)nn(N) * 8, rb1 = (size_t)nn(N) * 4;
    const size_t wbytes = cbytes * (size_t)C * nb_max, tbytes = (size_t)C * N * 8;
    void *ws = nullptr;
    if (int rc = get_workspace(stream, 4 * wbytes + rb1 * nb_max + 3 * tbytes + 4096, &ws)) return rc;
    Carver c;
    char *base = static_cast<char *>(ws);
    void *W1[2], *W2[2], *H[3];
    for (auto &w : W1) w = base + c.take(wbytes);
    for (auto &w : W2) w = base + c.take(wbytes);
    void *Iacc = base + c.take(rb1 * nb_max);
    for (auto &h : H) h = base + c.take(tbytes);
    const int K = (int)jobs.size();
    const int64_t upm = (int64_t)transpose_units_x(N) * transpose_units_y(N);
    for (int k = 0; k <= K + 1; ++k) {
        const bool has_x = k < K, has_y = k >= 2 && k - 2 < K;
        const int t = k - 1;
        const bool has_t = t >= 0 && t < K;
        const int64_t U = has_t ? upm * jobs[t].nb * jobs[t].m : 0;
        int64_t ua = 0;  // units [0, ua) ride on the x pass, [ua, U) on the y pass
        if (has_t) ua = (has_x && has_y) ? std::llround((double)U * sc.split) : has_x ? U : 0;
        auto side = [&](RowSide &sd, int64_t u0, int64_t u1, int fb, int sb) {
            sd.in = W1[t % 2];
            sd.out = W2[t % 2];
            sd.u0 = u0;
            sd.u1 = u1;
            sd.fft_blocks = fb;
            sd.side_blocks = sb;
        };
        if (has_x) {
            const PolyJob &jb = jobs[k];
            std::vector<double> r(rho.begin() + jb.j0, rho.begin() + jb.j0 + jb.m);
            const std::vector<double> amp = weight_amps(weight, jb.j0, jb.m);
            if (int rc = chirp_tables(H[k % 3], N, r, PS_F32, true, stream, &amp)) return rc;
            const bool with_side = has_t && ua > 0;
            ProgBuilder a(N, (int64_t)jb.nb * N);
            a.p.n_iter = jb.m;
            a.p.iter_split = sc.iter_split;
            for (int j = 0; j < jb.m; ++j) a.p.scale[j] = scale[jb.j0 + j];
            if (with_side) {
                a.op(ROP_SIDE_T);
                side(a.p.side, 0, ua, sc.fft_x, sc.side_x);
            }
            a.op(ROP_LOOP)
                .op(ROP_LOAD_PHASE, phi_ref + (size_t)jb.b0 * rb1, nn(N), N, 0, RF_ITER_SCALE)
                .op(ROP_FFT_FWD)
                .op(ROP_MUL_TAB, H[k % 3], 0, 0, N)
                .op(ROP_FFT_INV)
                .op(ROP_STORE_C, W1[k % 2], nn(N), N, (int64_t)jb.nb * nn(N))
                .op(ROP_ENDLOOP);
            const int rc = with_side ? run_row_side<ProgPhasePropTTag>(N, a.p, a.n, stream)
                                     : run_row<ProgPhasePropTag>(PS_F32, N, a.p, a.n, stream);
            if (rc) return rc;
        }
        if (has_y) {
            const PolyJob &jb = jobs[k - 2];
            const bool with_side = has_t && ua < U;
            ProgBuilder b(N, (int64_t)jb.nb * N);
            b.p.n_iter = jb.m;
            if (with_side) {
                b.op(ROP_SIDE_T);
                side(b.p.side, ua, U, sc.fft_y, sc.side_y);
            }
            b.op(ROP_LOOP)
                .op(ROP_LOAD_C, W2[(k - 2) % 2], nn(N), N, (int64_t)jb.nb * nn(N))
                .op(ROP_FFT_FWD)
                .op(ROP_MUL_TAB, H[(k - 2) % 3], 0, 0, N)
                .op(ROP_FFT_INV)
                .op(ROP_ACC_ABS2U)
                .op(ROP_ENDLOOP)
                .op(ROP_STORE_ACC, Iacc, nn(N), N, 0, jb.j0 > 0 ? RF_ADD : 0);
            const int rc = with_side ? run_row_side<ProgPropIntensityTTag>(N, b.p, b.n, stream)
                                     : run_row<ProgPropIntensityTag>(PS_F32, N, b.p, b.n, stream);
            if (rc) return rc;
            if (jb.j0 + jb.m >= n_lambda) {
                char *I = static_cast<char *>(I_out) + (size_t)jb.b0 * rb1;
                if (int rc2 = transpose(Iacc, I, N, jb.nb, 4, stream)) return rc2;
            }
        }
        if (!has_x && !has_y && has_t)
            if (int rc = transpose(W1[t % 2], W2[t % 2], N, (int64_t)jobs[t].nb * jobs[t].m, 8, stream)) return rc;
    }
    return PS_OK;
}

// Jobs of the pipelined propagation (FP32): up to 64 wavelengths and as many
// realisations per job as four complex buffers of the job's grids fit the
// budget; work that fits one job is split in two (realisations, else
// wavelengths): two pipelined jobs beat one plain job by ~10 % at 2048^2 and
// 4096^2 (8 realisations x 32 wavelengths), more jobs than the memory needs do
// not gain further.  False if the work does not make two jobs or one job does
// not fit.
static bool plan_poly_jobs(int N, int n_real, int n_lambda, size_t budget, std::vector<PolyJob> *jobs, int *Cp_out,
                           int *nbp_out) {
    const size_t cbytes = (size_t)nn(N) * 8, rb1 = (size_t)nn(N) * 4;
    auto need = [&](int Cq, int nbq) {
        return 4 * cbytes * (size_t)Cq * nbq + rb1 * nbq + 3 * (size_t)Cq * N * 8 + 4096;
    };
    int Cp = std::min(n_lambda, kRowMaxIter);
    while (Cp > 1 && need(Cp, 1) > budget) Cp = (Cp + 1) / 2;
    if (need(Cp, 1) > budget) return false;
    int nbp = 1;
    while (nbp < n_real && need(Cp, nbp + 1) <= budget) ++nbp;
    if (nbp >= n_real && Cp >= n_lambda) {
        if (n_real >= 2)
            nbp = (n_real + 1) / 2;
        else
            Cp = (n_lambda + 1) / 2;
    }
    jobs->clear();
    for (int b0 = 0; b0 < n_real; b0 += nbp)
        for (int j0 = 0; j0 < n_lambda; j0 += Cp)
            jobs->push_back({b0, std::min(nbp, n_real - b0), j0, std::min(Cp, n_lambda - j0)});
    *Cp_out = Cp;
    *nbp_out = nbp;
    return jobs->size() >= 2;
}

int fresnel_propagate(int N, double delta, double lambda, double z, const void *phi, double phase_scale, int n,
                      int dtype, void *I_out, void *hip_stream) {
    g_last_error.clear();
    g_last_warning.clear();
    if (int rc = check_common(N, dtype, n)) return rc;
    if (!phi || !I_out) return fail(PS_E_NULL, "phi and I_out must be non-NULL");
    if (int rc = check_aligned({phi, I_out})) return rc;
    if (!finite_pos(delta) || !finite_pos(lambda) || !finite_pos(z))
        return fail(PS_E_PARAM, "delta, lambda and z must be finite and > 0");
    if (!std::isfinite(phase_scale)) return fail(PS_E_PARAM, "phase_scale must be finite");
    const size_t rbytes = (size_t)nn(N) * real_bytes(dtype) * n;
    if (overlaps(phi, rbytes, I_out, rbytes)) return fail(PS_E_ALIAS, "I_out overlaps phi");
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    const double rho = std::sqrt(lambda * z / (2.0 * kPiD)) / delta;
    // FP32 from 2048 up with two or more realisations: the pipelined form
    // (one wavelength of phase scale s and weight 1)
    const SideCfg sc = side_cfg();
    if (dtype == PS_F32 && N >= 2048 && n >= 2 && sc.on) {
        std::vector<PolyJob> jobs;
        int Cp = 0, nbp = 0;
        if (plan_poly_jobs(N, n, 1, workspace_budget(), &jobs, &Cp, &nbp))
            return poly_pipelined(N, static_cast<const char *>(phi), jobs, Cp, nbp, 1, {rho}, {phase_scale}, {1.0},
                                  I_out, sc, stream);
    }
    const size_t cbytes = (size_t)nn(N) * 2 * real_bytes(dtype);
    const size_t tbytes = (size_t)N * 2 * real_bytes(dtype);
    const int nb_max = (int)std::max<size_t>(1, workspace_budget() / (2 * cbytes));
    for (int b0 = 0; b0 < n; b0 += nb_max) {
        const int nb = std::min(nb_max, n - b0);
        void *ws = nullptr;
        if (int rc = get_workspace(stream, 2 * cbytes * nb + tbytes + 1024, &ws)) return rc;
        Carver c;
        char *base = static_cast<char *>(ws);
        void *W1 = base + c.take(cbytes * nb);
        void *W2 = base + c.take(cbytes * nb);
        void *H = base + c.take(tbytes);
        const char *ph = static_cast<const char *>(phi) + (size_t)b0 * nn(N) * real_bytes(dtype);
        // W1 (complex) is free again once transposed into W2, so it holds the
        // transposed intensity
        if (int rc = poly_chunk(N, ph, nb, {rho}, {phase_scale}, {1.0}, dtype, W1, W2, H, W1, false, stream))
            return rc;
        char *I = static_cast<char *>(I_out) + (size_t)b0 * nn(N) * real_bytes(dtype);
        if (int rc = transpose(W1, I, N, nb, (int)real_bytes(dtype), stream)) return rc;
    }
    return PS_OK;
}

int fresnel_propagate_noalloc(int N, double delta, double lambda, double z, const void *phi, double phase_scale,
                              int n, int dtype, void *I_out, void *hip_stream) {
    g_last_error.clear();
    g_last_warning.clear();
    if (int rc = check_common(N, dtype, n)) return rc;
    if (!phi || !I_out) return fail(PS_E_NULL, "phi and I_out must be non-NULL");
    if (int rc = check_aligned({phi, I_out})) return rc;
    if (!finite_pos(delta) || !finite_pos(lambda) || !finite_pos(z))
        return fail(PS_E_PARAM, "delta, lambda and z must be finite and > 0");
    if (!std::isfinite(phase_scale)) return fail(PS_E_PARAM, "phase_scale must be finite");
    const size_t rb = real_bytes(dtype), cb = 2 * rb;
    const size_t rbytes = (size_t)nn(N) * rb * n;
    if (overlaps(phi, rbytes, I_out, rbytes)) return fail(PS_E_ALIAS, "I_out overlaps phi");
    TwiddleStages ts;
    if (!twiddle_stages(N, 0, &ts)) return fail(PS_E_SIZE, "no FFT plan for this size");
    // scratch: two complex fields per screen, the chirp table, the twiddles
    Carver c;
    const size_t oW1 = c.take(cb * (size_t)nn(N) * n), oW2 = c.take(cb * (size_t)nn(N) * n);
    const size_t oH = c.take(cb * (size_t)N), oT = c.take(cb * (size_t)std::max(ts.total, 1));
    if (c.used > kNoAllocScratchBytes)
        return fail(PS_E_SIZE, "fresnel_propagate_noalloc needs " + std::to_string(c.used) +
                                   " bytes of scratch for this size and batch, more than its " +
                                   std::to_string(kNoAllocScratchBytes) + "-byte array (4 N^2 n real elements "
                                   "plus tables); use fresnel_propagate");
    void *scr = nullptr;
    if (int rc = noalloc_scratch(&scr)) return rc;
    char *base = static_cast<char *>(scr);
    char *W1 = base + oW1, *W2 = base + oW2, *H = base + oH, *TW = base + oT;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    const bool f64 = dtype == PS_F64;
    HIP_TRY(launch_twiddle_table(TW, ts.n, ts.ns, ts.R, ts.off, ts.total, f64, stream));
    const double rho = std::sqrt(lambda * z / (2.0 * kPiD)) / delta;
    const double a = kPiD * rho * rho / ((double)N * (double)N);
    HIP_TRY(launch_chirp_tables(H, N, &a, 1, 1.0 / N, f64, stream));
    // x pass: exp(i s phi), DFT, chirp, inverse DFT; transpose; y pass:
    // DFT, chirp, inverse DFT, |.|^2 (into W1, transposed); transpose to I_out
    ProgBuilder x(N, (int64_t)n * N);
    x.op(ROP_LOOP)
        .op(ROP_LOAD_PHASE, phi, nn(N), N, 0, 0, phase_scale)
        .op(ROP_FFT_FWD)
        .op(ROP_MUL_TAB, H)
        .op(ROP_FFT_INV)
        .op(ROP_STORE_C, W1, nn(N), N)
        .op(ROP_ENDLOOP);
    if (int rc = launch_row_plan0<ProgPhasePropTag>(dtype, N, x.p, TW, stream)) return rc;
    HIP_TRY(launch_transpose(W1, W2, N, n, (int)cb, stream));
    ProgBuilder y(N, (int64_t)n * N);
    y.op(ROP_LOOP)
        .op(ROP_LOAD_C, W2, nn(N), N)
        .op(ROP_FFT_FWD)
        .op(ROP_MUL_TAB, H)
        .op(ROP_FFT_INV)
        .op(ROP_ACC_ABS2U)
        .op(ROP_ENDLOOP)
        .op(ROP_STORE_ACC, W1, nn(N), N);
    if (int rc = launch_row_plan0<ProgPropIntensityTag>(dtype, N, y.p, TW, stream)) return rc;
    HIP_TRY(launch_transpose(W1, I_out, N, n, (int)rb, stream));
    return PS_OK;
}

int fresnel_propagate_field(int N, double delta, double lambda, double z, const void *phi, double phase_scale, int n,
                            int dtype, void *I_out, void *field_out, void *hip_stream) {
    g_last_error.clear();
    g_last_warning.clear();
    if (int rc = check_common(N, dtype, n)) return rc;
    if (!phi || !I_out || !field_out) return fail(PS_E_NULL, "phi, I_out and field_out must be non-NULL");
    if (int rc = check_aligned({phi, I_out, field_out})) return rc;
    if (!finite_pos(delta) || !finite_pos(lambda) || !finite_pos(z))
        return fail(PS_E_PARAM, "delta, lambda and z must be finite and > 0");
    if (!std::isfinite(phase_scale)) return fail(PS_E_PARAM, "phase_scale must be finite");
    const size_t rbytes = (size_t)nn(N) * real_bytes(dtype) * n;
    if (overlaps(phi, rbytes, I_out, rbytes)) return fail(PS_E_ALIAS, "I_out overlaps phi");
    if (overlaps(field_out, 2 * rbytes, phi, rbytes) || overlaps(field_out, 2 * rbytes, I_out, rbytes))
        return fail(PS_E_ALIAS, "field_out overlaps phi or I_out");
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    const double rho = std::sqrt(lambda * z / (2.0 * kPiD)) / delta;
    const size_t cbytes = (size_t)nn(N) * 2 * real_bytes(dtype);
    const size_t tbytes = (size_t)N * 2 * real_bytes(dtype);
    const int nb_max = (int)std::max<size_t>(1, workspace_budget() / (2 * cbytes));
    for (int b0 = 0; b0 < n; b0 += nb_max) {
        const int nb = std::min(nb_max, n - b0);
        void *ws = nullptr;
        if (int rc = get_workspace(stream, 2 * cbytes * nb + tbytes + 1024, &ws)) return rc;
        Carver c;
        char *base = static_cast<char *>(ws);
        void *W1 = base + c.take(cbytes * nb);
        void *W2 = base + c.take(cbytes * nb);
        void *H = base + c.take(tbytes);
        if (int rc = chirp_tables(H, N, {rho}, dtype, true, stream)) return rc;
        const char *ph = static_cast<const char *>(phi) + (size_t)b0 * nn(N) * real_bytes(dtype);
        ProgBuilder a(N, (int64_t)nb * N);
        a.op(ROP_LOOP)
            .op(ROP_LOAD_PHASE, ph, nn(N), N, 0, 0, phase_scale)
            .op(ROP_FFT_FWD)
            .op(ROP_MUL_TAB, H)
            .op(ROP_FFT_INV)
            .op(ROP_STORE_C, W1, nn(N), N)
            .op(ROP_ENDLOOP);
        if (int rc = run_row<ProgPhasePropTag>(dtype, N, a.p, a.n, stream)) return rc;
        if (int rc = transpose(W1, W2, N, nb, 2 * (int)real_bytes(dtype), stream)) return rc;
        char *F = static_cast<char *>(field_out) + (size_t)b0 * cbytes;
        if (int rc = prop_y_pass(N, dtype, nb, W2, H, W1, F, stream)) return rc;
        char *I = static_cast<char *>(I_out) + (size_t)b0 * nn(N) * real_bytes(dtype);
        if (int rc = transpose(W1, I, N, nb, (int)real_bytes(dtype), stream)) return rc;
    }
    return PS_OK;
}

int fresnel_aperture(int N, double delta, double lambda, double z, const void *phi, double phase_scale,
                     double margin_rf, int n, int dtype, void *I_out, void *hip_stream) {
    g_last_error.clear();
    g_last_warning.clear();
    if (int rc = check_common(N, dtype, n)) return rc;
    if (!phi || !I_out) return fail(PS_E_NULL, "phi and I_out must be non-NULL");
    if (int rc = check_aligned({phi, I_out})) return rc;
    if (!finite_pos(delta) || !finite_pos(lambda) || !finite_pos(z))
        return fail(PS_E_PARAM, "delta, lambda and z must be finite and > 0");
    if (!std::isfinite(phase_scale)) return fail(PS_E_PARAM, "phase_scale must be finite");
    if (!(std::isfinite(margin_rf) && margin_rf >= 0.0)) return fail(PS_E_PARAM, "margin_rf must be finite and >= 0");
    const double rho = std::sqrt(lambda * z / (2.0 * kPiD)) / delta;
    const double two_pi_rho2 = 2.0 * kPiD * rho * rho;
    if ((double)N > two_pi_rho2 * (1.0 + 1e-9))
        return fail(PS_E_PARAM, "N delta^2 > lambda z: the Fresnel chirp is undersampled at the screen border");
    const double Lm = margin_rf * rho;
    if (2.0 * Lm > (double)N) return fail(PS_E_PARAM, "the window margins (2 margin_rf R_F) exceed the screen");
    const size_t rbytes = (size_t)nn(N) * real_bytes(dtype) * n;
    if (overlaps(phi, rbytes, I_out, rbytes)) return fail(PS_E_ALIAS, "I_out overlaps phi");
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    const size_t cbytes = (size_t)nn(N) * 2 * real_bytes(dtype);
    const size_t tbytes = (size_t)N * 2 * real_bytes(dtype);
    const int nb_max = (int)std::max<size_t>(1, workspace_budget() / (2 * cbytes));
    const double norm = 1.0 / (two_pi_rho2 * two_pi_rho2);
    for (int b0 = 0; b0 < n; b0 += nb_max) {
        const int nb = std::min(nb_max, n - b0);
        void *ws = nullptr;
        if (int rc = get_workspace(stream, 2 * cbytes * nb + tbytes + 1024, &ws)) return rc;
        Carver c;
        char *base = static_cast<char *>(ws);
        void *W1 = base + c.take(cbytes * nb);
        void *W2 = base + c.take(cbytes * nb);
        void *A = base + c.take(tbytes);
        HIP_TRY(launch_aperture_table(A, N, 1.0 / (4.0 * kPiD * rho * rho), Lm, dtype == PS_F64, stream));
        const char *ph = static_cast<const char *>(phi) + (size_t)b0 * nn(N) * real_bytes(dtype);
        // rows y: G = A[x] A[y] exp(i s phi), DFT along x
        ProgBuilder a(N, (int64_t)nb * N);
        a.op(ROP_LOAD_PHASE, ph, nn(N), N, 0, 0, phase_scale)
            .op(ROP_MUL_TAB, A)
            .op(ROP_MUL_ROWTAB, A)
            .op(ROP_FFT_FWD)
            .op(ROP_STORE_C, W1, nn(N), N);
        if (int rc = run_row<ProgApertureXTag>(dtype, N, a.p, a.n, stream)) return rc;
        if (int rc = transpose(W1, W2, N, nb, 2 * (int)real_bytes(dtype), stream)) return rc;
        // rows kx: DFT along y, |.|^2 / (2 pi rho^2)^2 (transposed intensity in W1)
        ProgBuilder d(N, (int64_t)nb * N);
        d.op(ROP_LOAD_C, W2, nn(N), N)
            .op(ROP_FFT_FWD)
            .op(ROP_ACC_ABS2, nullptr, 0, 0, 0, 0, norm)
            .op(ROP_STORE_ACC, W1, nn(N), N);
        if (int rc = run_row<ProgAbs2Tag>(dtype, N, d.p, d.n, stream)) return rc;
        char *I = static_cast<char *>(I_out) + (size_t)b0 * nn(N) * real_bytes(dtype);
        if (int rc = transpose(W1, I, N, nb, (int)real_bytes(dtype), stream)) return rc;
    }
    return PS_OK;
}

int ps_aperture_geometry(int N, double delta, double lambda, double z, double r_diff, double r_s,
                         double *observer_pixel, int *fiducial_margin) {
    g_last_error.clear();
    g_last_warning.clear();
    if (N < 2) return fail(PS_E_SIZE, "N must be >= 2");
    if (!observer_pixel || !fiducial_margin) return fail(PS_E_NULL, "observer_pixel and fiducial_margin must be non-NULL");
    if (!finite_pos(delta) || !finite_pos(lambda) || !finite_pos(z) || !finite_pos(r_diff))
        return fail(PS_E_PARAM, "delta, lambda, z and r_diff must be finite and > 0");
    if (!(std::isfinite(r_s) && r_s >= 0.0)) return fail(PS_E_PARAM, "r_s must be finite and >= 0");
    const double pix0 = lambda * z / ((double)N * delta);
    const double r_ref = lambda * z / r_diff;  // 2 pi R_F^2 / R_diff
    // the illuminated pattern is the screen's shadow, N delta wide, centred on
    // the observer grid (N pix0 wide, pix0 >= delta when fresnel_aperture runs)
    const double rim = std::max(0.0, 0.5 * (double)N * (1.0 - delta / pix0));
    const double m = std::ceil(rim + (0.5 * r_ref + r_s) / pix0 - 1e-9);
    *observer_pixel = pix0;
    *fiducial_margin = m > (double)N ? N : (int)m;
    if (2.0 * m >= (double)N) g_last_warning = "the fiducial zone is empty at this geometry";
    return PS_OK;
}

// The split of a polychromatic call (also reported by ps_plan_polychromatic):
// in FP32 from 2048 up, the pipelined jobs when four complex buffers of a
// job's grids fit (and there are two or more); otherwise chunks of C <= 64
// wavelengths and nb realisations such that two complex buffers of C nb
// grids plus the accumulator fit the budget.
struct PolyPlan {
    bool pipelined = false;
    int C = 1, nb = 1;
    std::vector<PolyJob> jobs;  // pipelined jobs (empty for the plain loop)
    size_t ws_bytes = 0;        // workspace it asks for
};
static PolyPlan plan_polychromatic(int N, int n_real, int n_lambda, int dtype, size_t budget, const SideCfg &sc) {
    PolyPlan pl;
    const size_t cbytes = (size_t)nn(N) * 2 * real_bytes(dtype);
    const size_t rb1 = (size_t)nn(N) * real_bytes(dtype);
    if (dtype == PS_F32 && N >= 2048 && sc.on &&
        plan_poly_jobs(N, n_real, n_lambda, budget, &pl.jobs, &pl.C, &pl.nb)) {
        pl.pipelined = true;
        pl.ws_bytes = 4 * cbytes * (size_t)pl.C * pl.nb + rb1 * pl.nb + 3 * (size_t)pl.C * N * 8 + 4096;
        return pl;
    }
    pl.jobs.clear();
    int C = std::min(n_lambda, kRowMaxIter);
    while (C > 1 && 2 * cbytes * (size_t)C + rb1 > budget) C = (C + 1) / 2;
    pl.C = C;
    pl.nb = std::min(n_real, (int)std::max<size_t>(1, budget / (2 * cbytes * (size_t)C + rb1)));
    pl.ws_bytes = 2 * cbytes * (size_t)C * pl.nb + rb1 * pl.nb + (size_t)C * N * 2 * real_bytes(dtype) + 2048;
    return pl;
}

int illumination_polychromatic(int N, double delta, double z, const void *phi_ref, double lambda_ref,
                               const double *lambdas, const double *weights, int n_lambda, int n_real, int dtype,
                               void *I_out, void *hip_stream) {
    g_last_error.clear();
    g_last_warning.clear();
    if (int rc = check_common(N, dtype, n_real)) return rc;
    if (!phi_ref || !I_out || !lambdas) return fail(PS_E_NULL, "phi_ref, lambdas and I_out must be non-NULL");
    if (int rc = check_aligned({phi_ref, I_out})) return rc;
    if (n_lambda < 1 || n_lambda > 4096) return fail(PS_E_SIZE, "n_lambda must lie in [1, 4096]");
    if (!finite_pos(delta) || !finite_pos(z) || !finite_pos(lambda_ref))
        return fail(PS_E_PARAM, "delta, z and lambda_ref must be finite and > 0");
    double wsum = 0.0;
    for (int j = 0; j < n_lambda; ++j) {
        if (!finite_pos(lambdas[j])) return fail(PS_E_PARAM, "every wavelength must be finite and > 0");
        const double w = weights ? weights[j] : 1.0;
        if (!std::isfinite(w) || w < 0.0) return fail(PS_E_PARAM, "weights must be finite and >= 0");
        wsum += w;
    }
    if (!(wsum > 0.0)) return fail(PS_E_PARAM, "weights must have a positive sum");
    const size_t rbytes = (size_t)nn(N) * real_bytes(dtype) * n_real;
    if (overlaps(phi_ref, rbytes, I_out, rbytes)) return fail(PS_E_ALIAS, "I_out overlaps phi_ref");
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    std::vector<double> rho(n_lambda), scale(n_lambda), weight(n_lambda);
    for (int j = 0; j < n_lambda; ++j) {
        rho[j] = std::sqrt(lambdas[j] * z / (2.0 * kPiD)) / delta;
        scale[j] = lambda_ref / lambdas[j];
        weight[j] = (weights ? weights[j] : 1.0) / wsum;
    }
    const size_t cbytes = (size_t)nn(N) * 2 * real_bytes(dtype);
    const size_t rb1 = (size_t)nn(N) * real_bytes(dtype);
    const SideCfg sc = side_cfg();
    const PolyPlan pl = plan_polychromatic(N, n_real, n_lambda, dtype, workspace_budget(), sc);
    if (pl.pipelined)
        return poly_pipelined(N, static_cast<const char *>(phi_ref), pl.jobs, pl.C, pl.nb, n_lambda, rho, scale, weight,
                              I_out, sc, stream);
    const int C = pl.C, nb_max = pl.nb;
    for (int b0 = 0; b0 < n_real; b0 += nb_max) {
        const int nb = std::min(nb_max, n_real - b0);
        void *ws = nullptr;
        const size_t tbytes = (size_t)C * N * 2 * real_bytes(dtype);
        if (int rc = get_workspace(stream, 2 * cbytes * (size_t)C * nb + rb1 * nb + tbytes + 2048, &ws)) return rc;
        Carver c;
        char *base = static_cast<char *>(ws);
        void *W1 = base + c.take(cbytes * (size_t)C * nb);
        void *W2 = base + c.take(cbytes * (size_t)C * nb);
        void *Iacc = base + c.take(rb1 * nb);
        void *H = base + c.take(tbytes);
        const char *ph = static_cast<const char *>(phi_ref) + (size_t)b0 * rb1;
        for (int j0 = 0; j0 < n_lambda; j0 += C) {
            const int m = std::min(C, n_lambda - j0);
            std::vector<double> r(rho.begin() + j0, rho.begin() + j0 + m);
            std::vector<double> s(scale.begin() + j0, scale.begin() + j0 + m);
            std::vector<double> w(weight.begin() + j0, weight.begin() + j0 + m);
            if (int rc = poly_chunk(N, ph, nb, r, s, w, dtype, W1, W2, H, Iacc, j0 > 0, stream)) return rc;
        }
        char *I = static_cast<char *>(I_out) + (size_t)b0 * rb1;
        if (int rc = transpose(Iacc, I, N, nb, (int)real_bytes(dtype), stream)) return rc;
    }
    return PS_OK;
}

int ps_plan_polychromatic(int N, int n_real, int n_lambda, int dtype, size_t budget_bytes, int *pipelined,
                          int *n_jobs, int *lambdas_per_job, int *real_per_job, size_t *workspace_bytes) {
    g_last_error.clear();
    if (int rc = check_common(N, dtype, n_real)) return rc;
    if (n_lambda < 1 || n_lambda > 4096) return fail(PS_E_SIZE, "n_lambda must lie in [1, 4096]");
    if (budget_bytes == 0) return fail(PS_E_PARAM, "budget_bytes must be > 0");
    const PolyPlan pl = plan_polychromatic(N, n_real, n_lambda, dtype, budget_bytes, side_cfg());
    const int jobs = pl.pipelined ? (int)pl.jobs.size()
                                  : ((n_real + pl.nb - 1) / pl.nb) * ((n_lambda + pl.C - 1) / pl.C);
    if (pipelined) *pipelined = pl.pipelined ? 1 : 0;
    if (n_jobs) *n_jobs = jobs;
    if (lambdas_per_job) *lambdas_per_job = pl.C;
    if (real_per_job) *real_per_job = pl.nb;
    if (workspace_bytes) *workspace_bytes = pl.ws_bytes;
    return PS_OK;
}

// Elements of one disk spectrum as kept: the quarter [0, N/2] x [0, N/2] of
// the N x N table (the disk, centred at the origin with minimum-image
// offsets, is even in x and in y, so its spectrum is even in kx' and ky').
static size_t disk_quarter_elems(int N) { return (size_t)(N / 2 + 1) * (N / 2 + 1); }

// Spectra of the normalised disks of radii Rpx[j] pixels, divided by N^2 (the
// inverse-transform normalisation), as n_r contiguous real tables of the
// quarter kx, ky in [0, N/2] of the spectrum indexed [kx][ky] (row length
// N/2 + 1; ROP_MUL_RTAB2D mirrors the rest); cached per (N, dtype, radii).
static int get_disk_spectra(int N, const std::vector<double> &Rpx, int dtype, hipStream_t stream,
                            const void **out) {
    int dev;
    if (int rc = current_device(&dev)) return rc;
    std::vector<uint64_t> bits(Rpx.size());
    for (size_t j = 0; j < Rpx.size(); ++j) std::memcpy(&bits[j], &Rpx[j], sizeof(uint64_t));
    auto key = std::make_pair(std::make_pair(N, dtype), bits);
    {
        std::lock_guard<std::mutex> lock(g_mutex);
        auto &dc = g_cache[dev];
        auto it = dc.disks.find(key);
        if (it != dc.disks.end()) {
            *out = it->second;
            return PS_OK;
        }
    }
    if (int rc = refuse_in_capture(stream, "building the disk spectra of these radii")) return rc;
    const size_t rb = (size_t)nn(N) * real_bytes(dtype);
    const size_t cb = 2 * rb;
    const size_t qb = disk_quarter_elems(N) * real_bytes(dtype);
    void *block = nullptr;
    if (hipMalloc(&block, qb * Rpx.size()) != hipSuccess) return fail(PS_E_ALLOC, "hipMalloc of disk spectra failed");
    void *tmp = nullptr;
    if (hipMalloc(&tmp, 2 * cb + rb) != hipSuccess) {
        (void)hipFree(block);
        return fail(PS_E_ALLOC, "hipMalloc of disk workspace failed");
    }
    char *W1 = static_cast<char *>(tmp), *W2 = W1 + cb, *tab = W2 + cb;  // tab: the full N x N table
    int rc = PS_OK;
    for (size_t j = 0; j < Rpx.size() && !rc; ++j) {
        // pixel count of the disk, same test as the disk image kernel
        const double r2 = Rpx[j] * Rpx[j];
        double count = 0.0;
        for (int y = 0; y < N; ++y) {
            const double dy = y < N / 2 ? y : y - N;
            if (dy * dy > r2) continue;
            for (int x = 0; x < N; ++x) {
                const double dx = x < N / 2 ? x : x - N;
                if (dx * dx + dy * dy <= r2) count += 1.0;
            }
        }
        hipError_t e = launch_disk_image(tab, N, r2, 1.0 / count, dtype == PS_F64, stream);
        if (e != hipSuccess) rc = fail(PS_E_DEVICE, std::string("disk image: ") + hipGetErrorString(e));
        if (!rc) {
            ProgBuilder a(N, N);
            a.op(ROP_LOAD_R, tab, 0, N).op(ROP_FFT_FWD).op(ROP_STORE_C, W1, 0, N);
            rc = run_row<ProgRealFwdTag>(dtype, N, a.p, a.n, stream);
        }
        if (!rc) rc = transpose(W1, W2, N, 1, 2 * (int)real_bytes(dtype), stream);
        if (!rc) {
            ProgBuilder b(N, N);
            b.op(ROP_LOAD_C, W2, 0, N).op(ROP_FFT_FWD).op(ROP_STORE_R, tab, 0, N, 0, 0, 1.0 / (double)nn(N));
            rc = run_row<ProgFwdReTag>(dtype, N, b.p, b.n, stream);
        }
        if (!rc) {
            // keep the quarter: rows kx <= N/2, their first N/2 + 1 entries
            const size_t w = (size_t)(N / 2 + 1) * real_bytes(dtype);
            hipError_t e2 = hipMemcpy2DAsync(static_cast<char *>(block) + j * qb, w, tab, (size_t)N * real_bytes(dtype), w,
                                             (size_t)(N / 2 + 1), hipMemcpyDeviceToDevice, stream);
            if (e2 != hipSuccess) rc = fail(PS_E_DEVICE, std::string("disk spectrum copy: ") + hipGetErrorString(e2));
        }
    }
    if (!rc) {
        hipError_t e = hipStreamSynchronize(stream);
        if (e != hipSuccess) rc = fail(PS_E_DEVICE, std::string("disk spectrum: ") + hipGetErrorString(e));
    }
    (void)hipFree(tmp);
    if (rc) {
        (void)hipFree(block);
        return rc;
    }
    std::lock_guard<std::mutex> lock(g_mutex);
    g_cache[dev].disks[key] = block;
    *out = block;
    return PS_OK;
}

// ------------------------------------------------------------ source smear
// One group of the smear: np complex transforms, each holding `step` (2: a
// pair, 1: a single) realisations; W1/W2 hold np complex grids, V1/V2
// np n_r.  The three row passes: the forward x pass of the real patterns,
// the middle pass (y forward, times each disk spectrum, y inverse), and per
// radius the inverse x pass to real patterns.
struct SmearJob {
    const char *Iin;
    char *Iout;
    int np, step;
    char *W1, *W2, *V1, *V2;
};
// transposes [u0, u1) of complex64 matrices in -> out, carried by a pass
struct SmearSide {
    const void *in;
    void *out;
    int64_t u0, u1;
};

static ProgBuilder smear_rf_prog(int N, const SmearJob &j, size_t rb1, bool side) {
    const bool pair = j.step == 2;
    ProgBuilder a(N, (int64_t)j.np * N);
    if (side) a.op(ROP_SIDE_T);
    a.op(ROP_LOAD_R, j.Iin, (int64_t)j.step * nn(N), N, 0, pair ? RF_PAIR : 0, 0.0,
         pair ? const_cast<char *>(j.Iin) + rb1 : nullptr)
        .op(ROP_FFT_FWD)
        .op(ROP_STORE_C, j.W1, nn(N), N);
    return a;
}
static ProgBuilder smear_mid_prog(int N, const SmearJob &j, const void *D, int n_r, bool side) {
    ProgBuilder b(N, (int64_t)j.np * N);
    b.p.n_iter = n_r;
    if (side) b.op(ROP_SIDE_T);
    b.op(ROP_LOAD_C, j.W2, nn(N), N)
        .op(ROP_FFT_FWD)
        .op(ROP_SAVE)
        .op(ROP_LOOP)
        .op(ROP_RESTORE)
        .op(ROP_MUL_RTAB2D, D, 0, N / 2 + 1, disk_quarter_elems(N))
        .op(ROP_FFT_INV)
        .op(ROP_STORE_C, j.V1, (int64_t)n_r * nn(N), N, nn(N))
        .op(ROP_ENDLOOP);
    return b;
}
static ProgBuilder smear_ir_prog(int N, const SmearJob &j, int r, int n_r, size_t rb1, bool side) {
    const bool pair = j.step == 2;
    const size_t cbytes = 2 * rb1;
    ProgBuilder d(N, (int64_t)j.np * N);
    char *dst = j.Iout + (size_t)r * rb1;
    if (side) d.op(ROP_SIDE_T);
    d.op(ROP_LOAD_C, j.V2 + (size_t)r * cbytes, (int64_t)n_r * nn(N), N)
        .op(ROP_FFT_INV)
        .op(ROP_STORE_R, dst, (int64_t)j.step * n_r * nn(N), N, 0, pair ? RF_PAIR : 0, 1.0,
            pair ? dst + (size_t)n_r * rb1 : nullptr);
    return d;
}
static void set_side(RowSide &sd, const SmearSide &t, const SideCfg &sc) {
    sd.in = t.in;
    sd.out = t.out;
    sd.u0 = t.u0;
    sd.u1 = t.u1;
    sd.fft_blocks = sc.fft_x;
    sd.side_blocks = sc.side_x;
}
// the passes in any precision, without side transposes
static int smear_rf_any(int N, int dtype, const SmearJob &j, hipStream_t stream) {
    ProgBuilder a = smear_rf_prog(N, j, (size_t)nn(N) * real_bytes(dtype), false);
    return run_row<ProgRealFwdTag>(dtype, N, a.p, a.n, stream);
}
static int smear_mid_any(int N, int dtype, const SmearJob &j, const void *D, int n_r, hipStream_t stream) {
    ProgBuilder b = smear_mid_prog(N, j, D, n_r, false);
    return run_row<ProgSmearMidTag>(dtype, N, b.p, b.n, stream);
}
static int smear_ir_any(int N, int dtype, const SmearJob &j, int r, int n_r, hipStream_t stream) {
    ProgBuilder d = smear_ir_prog(N, j, r, n_r, (size_t)nn(N) * real_bytes(dtype), false);
    return run_row<ProgInvReTag>(dtype, N, d.p, d.n, stream);
}
// FP32 passes carrying the transposes `t` (none if NULL)
static int smear_rf(int N, const SmearJob &j, const SmearSide *t, const SideCfg &sc, hipStream_t stream) {
    if (!t) return smear_rf_any(N, PS_F32, j, stream);
    ProgBuilder a = smear_rf_prog(N, j, (size_t)nn(N) * 4, true);
    set_side(a.p.side, *t, sc);
    return run_row_side<ProgRealFwdTTag>(N, a.p, a.n, stream);
}
static int smear_mid(int N, const SmearJob &j, const void *D, int n_r, const SmearSide *t, const SideCfg &sc,
                     hipStream_t stream) {
    if (!t) return smear_mid_any(N, PS_F32, j, D, n_r, stream);
    ProgBuilder b = smear_mid_prog(N, j, D, n_r, true);
    set_side(b.p.side, *t, sc);
    return run_row_side<ProgSmearMidTTag>(N, b.p, b.n, stream);
}
static int smear_ir(int N, const SmearJob &j, int r, int n_r, const SmearSide *t, const SideCfg &sc,
                    hipStream_t stream) {
    if (!t) return smear_ir_any(N, PS_F32, j, r, n_r, stream);
    ProgBuilder d = smear_ir_prog(N, j, r, n_r, (size_t)nn(N) * 4, true);
    set_side(d.p.side, *t, sc);
    return run_row_side<ProgInvReTTag>(N, d.p, d.n, stream);
}

int source_smear(int N, double delta, const void *I_in, const double *radii, int n_r, int n_real, int dtype,
                 void *I_out, void *hip_stream) {
    g_last_error.clear();
    g_last_warning.clear();
    if (int rc = check_common(N, dtype, n_real)) return rc;
    if (!I_in || !I_out || !radii) return fail(PS_E_NULL, "I_in, radii and I_out must be non-NULL");
    if (int rc = check_aligned({I_in, I_out})) return rc;
    if (n_r < 1 || n_r > kRowMaxIter) return fail(PS_E_SIZE, "n_r must lie in [1, 64]");
    if (!finite_pos(delta)) return fail(PS_E_PARAM, "delta must be finite and > 0");
    for (int j = 0; j < n_r; ++j)
        if (!std::isfinite(radii[j]) || radii[j] < 0.0) return fail(PS_E_PARAM, "radii must be finite and >= 0");
    const size_t rb1 = (size_t)nn(N) * real_bytes(dtype);
    if (overlaps(I_in, rb1 * n_real, I_out, rb1 * n_real * n_r) && !(n_r == 1 && I_in == I_out))
        return fail(PS_E_ALIAS, "I_out overlaps I_in (allowed only in place with n_r == 1)");
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    std::vector<double> rpx(n_r);
    for (int j = 0; j < n_r; ++j) rpx[j] = radii[j] / delta;
    const void *D = nullptr;
    if (int rc = get_disk_spectra(N, rpx, dtype, stream, &D)) return rc;
    const size_t cbytes = 2 * rb1;
    const size_t budget = workspace_budget();
    const int nb_max = (int)std::max<size_t>(1, budget / (cbytes * (2 + 2 * (size_t)n_r)));
    // The disk kernel is real, so two real patterns a and b ride in one
    // complex transform: (a + i b) * d = a * d + i (b * d).  Realisations are
    // paired; an odd last one goes alone (imaginary part zero).
    for (int b0 = 0; b0 < n_real; b0 += nb_max) {
        const int nb = std::min(nb_max, n_real - b0);
        void *ws = nullptr;
        if (int rc = get_workspace(stream, cbytes * nb * (2 + 2 * (size_t)n_r) + 4096, &ws)) return rc;
        Carver c;
        char *base = static_cast<char *>(ws);
        char *W1 = base + c.take(cbytes * nb);
        char *W2 = base + c.take(cbytes * nb);
        char *V1 = base + c.take(cbytes * nb * n_r);
        char *V2 = base + c.take(cbytes * nb * n_r);
        const SideCfg sc = side_cfg();
        for (int pb = 0; pb < nb;) {
            const bool pair = nb - pb >= 2;
            const int np = pair ? (nb - pb) / 2 : 1;  // complex transforms in this group
            const int step = pair ? 2 : 1;            // realisations per transform
            const char *Iin = static_cast<const char *>(I_in) + (size_t)(b0 + pb) * rb1;
            // I_out[b][r]: transform q holds realisations b0 + pb + step q (and + 1)
            char *Iout = static_cast<char *>(I_out) + (size_t)(b0 + pb) * n_r * rb1;
            SmearJob all{Iin, Iout, np, step, W1, W2, V1, V2};
            if (dtype == PS_F32 && N >= 2048 && np >= 2 && sc.on) {
                // two jobs, the transposes of each riding on the other's passes
                const int q0 = (np + 1) / 2;
                const SmearJob j0{Iin, Iout, q0, step, W1, W2, V1, V2};
                const size_t o = (size_t)q0 * cbytes;  // offset of job 1 in the complex buffers
                const SmearJob j1{Iin + (size_t)q0 * step * rb1, Iout + (size_t)q0 * step * n_r * rb1, np - q0, step,
                                  W1 + o, W2 + o, V1 + o * n_r, V2 + o * n_r};
                const int64_t upm = (int64_t)transpose_units_x(N) * transpose_units_y(N);
                const SmearSide t1_0{j0.W1, j0.W2, 0, upm * j0.np}, t1_1{j1.W1, j1.W2, 0, upm * j1.np};
                const SmearSide t2_0{j0.V1, j0.V2, 0, upm * j0.np * n_r};
                const int64_t U2 = upm * j1.np * n_r;
                if (int rc = smear_rf(N, j0, nullptr, sc, stream)) return rc;
                if (int rc = smear_rf(N, j1, &t1_0, sc, stream)) return rc;
                if (int rc = smear_mid(N, j0, D, n_r, &t1_1, sc, stream)) return rc;
                if (int rc = smear_mid(N, j1, D, n_r, &t2_0, sc, stream)) return rc;
                for (int r = 0; r < n_r; ++r) {
                    const SmearSide t2_1{j1.V1, j1.V2, U2 * r / n_r, U2 * (r + 1) / n_r};
                    if (int rc = smear_ir(N, j0, r, n_r, t2_1.u1 > t2_1.u0 ? &t2_1 : nullptr, sc, stream)) return rc;
                }
                for (int r = 0; r < n_r; ++r)
                    if (int rc = smear_ir(N, j1, r, n_r, nullptr, sc, stream)) return rc;
            } else {
                if (int rc = smear_rf_any(N, dtype, all, stream)) return rc;
                if (int rc = transpose(W1, W2, N, np, (int)(cbytes / nn(N)), stream)) return rc;
                if (int rc = smear_mid_any(N, dtype, all, D, n_r, stream)) return rc;
                if (int rc = transpose(V1, V2, N, (int64_t)np * n_r, (int)(cbytes / nn(N)), stream)) return rc;
                for (int r = 0; r < n_r; ++r)
                    if (int rc = smear_ir_any(N, dtype, all, r, n_r, stream)) return rc;
            }
            pb += np * step;
        }
    }
    return PS_OK;
}

int fresnel_propagate_vjp(int N, double delta, double lambda, double z, const void *phi, double phase_scale,
                          const void *grad_I, const void *field, int n, int dtype, void *grad_phi_out,
                          double *phi_dot_grad_out, void *hip_stream) {
    g_last_error.clear();
    g_last_warning.clear();
    if (int rc = check_common(N, dtype, n)) return rc;
    if (!phi || !grad_I || !grad_phi_out) return fail(PS_E_NULL, "phi, grad_I and grad_phi_out must be non-NULL");
    if (int rc = check_aligned({phi, grad_I, grad_phi_out, field})) return rc;
    if (!finite_pos(delta) || !finite_pos(lambda) || !finite_pos(z))
        return fail(PS_E_PARAM, "delta, lambda and z must be finite and > 0");
    if (!std::isfinite(phase_scale)) return fail(PS_E_PARAM, "phase_scale must be finite");
    const size_t rb1 = (size_t)nn(N) * real_bytes(dtype);
    if (overlaps(grad_phi_out, rb1 * n, phi, rb1 * n) || overlaps(grad_phi_out, rb1 * n, grad_I, rb1 * n) ||
        (field && overlaps(grad_phi_out, rb1 * n, field, 2 * rb1 * n)))
        return fail(PS_E_ALIAS, "grad_phi_out overlaps phi, grad_I or field");
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    if (phi_dot_grad_out)
        if (int rc = refuse_in_capture(stream, "returning phi_dot_grad_out to the host")) return rc;
    const double rho = std::sqrt(lambda * z / (2.0 * kPiD)) / delta;
    const size_t cbytes = 2 * rb1;
    const size_t tbytes = (size_t)N * 2 * real_bytes(dtype);
    const int nb_max = (int)std::max<size_t>(1, workspace_budget() / (2 * cbytes + rb1 + N * 8));
    std::vector<double> dots(n, 0.0);
    for (int b0 = 0; b0 < n; b0 += nb_max) {
        const int nb = std::min(nb_max, n - b0);
        void *ws = nullptr;
        if (int rc = get_workspace(stream, (2 * cbytes + rb1) * nb + tbytes + (size_t)nb * N * 8 + nb * 8 + 4096,
                                   &ws))
            return rc;
        Carver c;
        char *base = static_cast<char *>(ws);
        char *W1 = base + c.take(cbytes * nb);
        char *W2 = base + c.take(cbytes * nb);
        char *Gt = base + c.take(rb1 * nb);
        char *H = base + c.take(tbytes);
        double *rowdot = reinterpret_cast<double *>(base + c.take((size_t)nb * N * 8));
        double *bdot = reinterpret_cast<double *>(base + c.take((size_t)nb * 8));
        if (int rc = chirp_tables(H, N, {rho}, dtype, true, stream)) return rc;
        const char *ph = static_cast<const char *>(phi) + (size_t)b0 * rb1;
        const char *gI = static_cast<const char *>(grad_I) + (size_t)b0 * rb1;
        if (int rc = transpose(gI, Gt, N, nb, (int)real_bytes(dtype), stream)) return rc;
        if (field) {
            // from the checkpoint: g_A = 2 grad_I A, adjoint y-propagation
            ProgBuilder b(N, (int64_t)nb * N);
            b.op(ROP_LOAD_C, static_cast<const char *>(field) + (size_t)b0 * cbytes, nn(N), N)
                .op(ROP_MUL_RLOAD, Gt, nn(N), N, 0, 0, 2.0)
                .op(ROP_FFT_FWD)
                .op(ROP_MUL_TAB, H, 0, 0, 0, RF_CONJ)
                .op(ROP_FFT_INV)
                .op(ROP_STORE_C, W1, nn(N), N);
            if (int rc = run_row<ProgVjpYFieldTag>(dtype, N, b.p, b.n, stream)) return rc;
        } else {
            // forward x-propagation (recomputed from phi)
            ProgBuilder a(N, (int64_t)nb * N);
            a.op(ROP_LOOP)
                .op(ROP_LOAD_PHASE, ph, nn(N), N, 0, 0, phase_scale)
                .op(ROP_FFT_FWD)
                .op(ROP_MUL_TAB, H)
                .op(ROP_FFT_INV)
                .op(ROP_STORE_C, W1, nn(N), N)
                .op(ROP_ENDLOOP);
            if (int rc = run_row<ProgPhasePropTag>(dtype, N, a.p, a.n, stream)) return rc;
            if (int rc = transpose(W1, W2, N, nb, (int)(cbytes / nn(N)), stream)) return rc;
            // y-propagation to A (transposed), g_A = 2 grad_I A, adjoint y-propagation
            ProgBuilder b(N, (int64_t)nb * N);
            b.op(ROP_LOAD_C, W2, nn(N), N)
                .op(ROP_FFT_FWD)
                .op(ROP_MUL_TAB, H)
                .op(ROP_FFT_INV)
                .op(ROP_MUL_RLOAD, Gt, nn(N), N, 0, 0, 2.0)
                .op(ROP_FFT_FWD)
                .op(ROP_MUL_TAB, H, 0, 0, 0, RF_CONJ)
                .op(ROP_FFT_INV)
                .op(ROP_STORE_C, W1, nn(N), N);
            if (int rc = run_row<ProgVjpYTag>(dtype, N, b.p, b.n, stream)) return rc;
        }
        if (int rc = transpose(W1, W2, N, nb, (int)(cbytes / nn(N)), stream)) return rc;
        // adjoint x-propagation, dL/dphi = s Im(g_U conj U), and sum phi dL/dphi per row
        char *gphi = static_cast<char *>(grad_phi_out) + (size_t)b0 * rb1;
        ProgBuilder d(N, (int64_t)nb * N);
        d.op(ROP_LOAD_C, W2, nn(N), N)
            .op(ROP_FFT_FWD)
            .op(ROP_MUL_TAB, H, 0, 0, 0, RF_CONJ)
            .op(ROP_FFT_INV)
            .op(ROP_GRAD_PHI, ph, nn(N), N, 0, 0, phase_scale)
            .op(ROP_STORE_R, gphi, nn(N), N, 0, 0, 1.0)
            .op(ROP_DOT_R, ph, nn(N), N, 0, 0, 0.0, rowdot);
        if (int rc = run_row<ProgVjpXTag>(dtype, N, d.p, d.n, stream)) return rc;
        if (phi_dot_grad_out) {
            HIP_TRY(launch_finalize_sums(rowdot, N, nb, 1.0, bdot, stream));
            HIP_TRY(hipMemcpyAsync(dots.data() + b0, bdot, (size_t)nb * 8, hipMemcpyDeviceToHost, stream));
        }
    }
    if (phi_dot_grad_out) {
        HIP_TRY(hipStreamSynchronize(stream));
        std::memcpy(phi_dot_grad_out, dots.data(), (size_t)n * 8);
    }
    return PS_OK;
}

static int block_count(int64_t n) {
    const int64_t per = 256 * 16;
    return (int)std::max<int64_t>(1, std::min<int64_t>(1024, (n + per - 1) / per));
}

int ps_modulation_index(int N, const void *I, int n, int dtype, double *m_out, double *mean_out,
                        void *hip_stream) {
    g_last_error.clear();
    g_last_warning.clear();
    if (int rc = check_common(N, dtype, n)) return rc;
    if (!I || !m_out) return fail(PS_E_NULL, "I and m_out must be non-NULL");
    if (int rc = check_aligned({I})) return rc;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    if (int rc = refuse_in_capture(stream, "ps_modulation_index")) return rc;
    const int64_t per = nn(N);
    const int nblk = block_count(per);
    void *ws = nullptr;
    if (int rc = get_workspace(stream, (size_t)n * nblk * 8 + (size_t)n * 16 + 1024, &ws)) return rc;
    Carver c;
    char *base = static_cast<char *>(ws);
    double *part = reinterpret_cast<double *>(base + c.take((size_t)n * nblk * 8));
    double *mean = reinterpret_cast<double *>(base + c.take((size_t)n * 8));
    double *var = reinterpret_cast<double *>(base + c.take((size_t)n * 8));
    const bool f64 = dtype == PS_F64;
    HIP_TRY(launch_block_sums(I, per, n, nullptr, 1, nblk, f64, part, stream));
    HIP_TRY(launch_finalize_sums(part, nblk, n, 1.0 / (double)per, mean, stream));
    HIP_TRY(launch_block_sums(I, per, n, mean, 2, nblk, f64, part, stream));
    HIP_TRY(launch_finalize_sums(part, nblk, n, 1.0 / (double)per, var, stream));
    std::vector<double> hm(n), hv(n);
    HIP_TRY(hipMemcpyAsync(hm.data(), mean, (size_t)n * 8, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipMemcpyAsync(hv.data(), var, (size_t)n * 8, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    for (int b = 0; b < n; ++b) {
        m_out[b] = std::sqrt(hv[b]) / hm[b];
        if (mean_out) mean_out[b] = hm[b];
    }
    return PS_OK;
}

int ps_modulation_index_region(int N, const void *I, int n, int x0, int y0, int w, int h, int dtype, double *m_out,
                               double *mean_out, void *hip_stream) {
    g_last_error.clear();
    g_last_warning.clear();
    if (int rc = check_common(N, dtype, n)) return rc;
    if (!I || !m_out) return fail(PS_E_NULL, "I and m_out must be non-NULL");
    if (int rc = check_aligned({I})) return rc;
    if (x0 < 0 || y0 < 0 || w < 1 || h < 1 || w > N - x0 || h > N - y0)
        return fail(PS_E_PARAM, "the region must be non-empty and lie inside the N x N image");
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    if (int rc = refuse_in_capture(stream, "ps_modulation_index_region")) return rc;
    const int64_t count = (int64_t)w * h;
    const int nblk = block_count(count);
    void *ws = nullptr;
    if (int rc = get_workspace(stream, (size_t)n * nblk * 8 + (size_t)n * 16 + 1024, &ws)) return rc;
    Carver c;
    char *base = static_cast<char *>(ws);
    double *part = reinterpret_cast<double *>(base + c.take((size_t)n * nblk * 8));
    double *mean = reinterpret_cast<double *>(base + c.take((size_t)n * 8));
    double *var = reinterpret_cast<double *>(base + c.take((size_t)n * 8));
    const bool f64 = dtype == PS_F64;
    const char *first = static_cast<const char *>(I) + ((size_t)y0 * N + x0) * real_bytes(dtype);
    HIP_TRY(launch_region_sums(first, nn(N), w, h, N, n, nullptr, 1, nblk, f64, part, stream));
    HIP_TRY(launch_finalize_sums(part, nblk, n, 1.0 / (double)count, mean, stream));
    HIP_TRY(launch_region_sums(first, nn(N), w, h, N, n, mean, 2, nblk, f64, part, stream));
    HIP_TRY(launch_finalize_sums(part, nblk, n, 1.0 / (double)count, var, stream));
    std::vector<double> hm(n), hv(n);
    HIP_TRY(hipMemcpyAsync(hm.data(), mean, (size_t)n * 8, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipMemcpyAsync(hv.data(), var, (size_t)n * 8, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    for (int b = 0; b < n; ++b) {
        m_out[b] = std::sqrt(hv[b]) / hm[b];
        if (mean_out) mean_out[b] = hm[b];
    }
    return PS_OK;
}

int ps_light_curves(int N, const void *I, int n, const double *lines, int n_lines, int n_samples, int mode,
                    int dtype, void *curves_out, double *m_out, void *hip_stream) {
    g_last_error.clear();
    g_last_warning.clear();
    if (int rc = check_common(N, dtype, n)) return rc;
    if (!I || !lines || !curves_out) return fail(PS_E_NULL, "I, lines and curves_out must be non-NULL");
    if (int rc = check_aligned({I, curves_out})) return rc;
    if (n_lines < 1 || n_samples < 1) return fail(PS_E_SIZE, "n_lines and n_samples must be >= 1");
    if (mode != 0 && mode != 1) return fail(PS_E_PARAM, "mode must be 0 (nearest pixel) or 1 (bilinear)");
    for (int i = 0; i < 4 * n_lines; ++i)
        if (!std::isfinite(lines[i])) return fail(PS_E_PARAM, "line coordinates must be finite");
    const size_t ib = (size_t)nn(N) * real_bytes(dtype) * n;
    const size_t cb = (size_t)n * n_lines * n_samples * real_bytes(dtype);
    if (overlaps(I, ib, curves_out, cb)) return fail(PS_E_ALIAS, "curves_out overlaps I");
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    if (m_out)
        if (int rc = refuse_in_capture(stream, "returning m_out to the host")) return rc;
    double *stats = nullptr;
    if (m_out) {
        void *ws = nullptr;
        if (int rc = get_workspace(stream, (size_t)n * n_lines * 16 + 256, &ws)) return rc;
        stats = static_cast<double *>(ws);
    }
    HIP_TRY(launch_light_curves(I, N, n, lines, n_lines, n_samples, mode, dtype == PS_F64, curves_out, stats,
                                stream));
    if (m_out) {
        std::vector<double> h((size_t)2 * n * n_lines);
        HIP_TRY(hipMemcpyAsync(h.data(), stats, h.size() * 8, hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        for (size_t i = 0; i < (size_t)n * n_lines; ++i) m_out[i] = std::sqrt(h[2 * i + 1]) / h[2 * i];
    }
    return PS_OK;
}

int ps_m_theory(double r_diff, double r_f, double r_s, double *m_out) {
    g_last_error.clear();
    g_last_warning.clear();
    if (!m_out) return fail(PS_E_NULL, "m_out is NULL");
    if (!finite_pos(r_diff) || !finite_pos(r_f) || !finite_pos(r_s))
        return fail(PS_E_PARAM, "r_diff, r_f and r_s must be finite and > 0");
    const double r_ref = 2.0 * kPiD * r_f * r_f / r_diff;
    *m_out = std::pow(r_diff / r_f, 1.0 / 3.0) * std::pow(r_ref / (2.0 * kPiD * r_s), 7.0 / 6.0);
    if (!(r_s / r_f > r_f / r_diff && r_f / r_diff > 1.0))
        g_last_warning = "outside the strong, quenched regime R_s/R_F > R_F/R_diff > 1";
    return PS_OK;
}

int ps_structure_function(int N, double delta, const void *phi, int n, const double *radii, int n_r, int dtype,
                          double *S_out, double *D_out, double *rdiff_out, void *hip_stream) {
    g_last_error.clear();
    g_last_warning.clear();
    if (int rc = check_common(N, dtype, n)) return rc;
    if (!phi) return fail(PS_E_NULL, "phi is NULL");
    if (int rc = check_aligned({phi})) return rc;
    if (!finite_pos(delta)) return fail(PS_E_PARAM, "delta must be finite and > 0");
    if (n_r < 0 || (n_r > 0 && (!radii || !D_out))) return fail(PS_E_PARAM, "n_r >= 0, with radii and D_out when > 0");
    for (int j = 0; j < n_r; ++j)
        if (!(std::isfinite(radii[j]) && radii[j] >= 0.0)) return fail(PS_E_PARAM, "radii must be finite and >= 0");
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    if (int rc = refuse_in_capture(stream, "ps_structure_function")) return rc;
    const int nbins = N / 2 + 1;
    const size_t cbytes = (size_t)nn(N) * 2 * real_bytes(dtype);
    const int nb_max = (int)std::max<size_t>(1, workspace_budget() / (2 * cbytes));
    std::vector<double> rpx(n_r);
    for (int j = 0; j < n_r; ++j) rpx[j] = radii[j] / delta;
    for (int b0 = 0; b0 < n; b0 += nb_max) {
        const int nb = std::min(nb_max, n - b0);
        const size_t small = (size_t)nb * nbins * 8 + (size_t)nb * std::max(n_r, 1) * 8 + (size_t)nb * 8 + 1024;
        void *ws = nullptr;
        if (int rc = get_workspace(stream, 2 * cbytes * nb + small, &ws)) return rc;
        Carver c;
        char *base = static_cast<char *>(ws);
        void *W1 = base + c.take(cbytes * nb);
        void *W2 = base + c.take(cbytes * nb);
        double *S = reinterpret_cast<double *>(base + c.take((size_t)nb * nbins * 8));
        double *D = reinterpret_cast<double *>(base + c.take((size_t)nb * std::max(n_r, 1) * 8));
        double *R = reinterpret_cast<double *>(base + c.take((size_t)nb * 8));
        const char *ph = static_cast<const char *>(phi) + (size_t)b0 * nn(N) * real_bytes(dtype);
        // |DFT phi|^2 / N^2: DFT along x, transpose, DFT along y and |.|^2
        ProgBuilder a(N, (int64_t)nb * N);
        a.op(ROP_LOAD_R, ph, nn(N), N).op(ROP_FFT_FWD).op(ROP_STORE_C, W1, nn(N), N);
        if (int rc = run_row<ProgRealFwdTag>(dtype, N, a.p, a.n, stream)) return rc;
        if (int rc = transpose(W1, W2, N, nb, 2 * (int)real_bytes(dtype), stream)) return rc;
        ProgBuilder d(N, (int64_t)nb * N);
        d.op(ROP_LOAD_C, W2, nn(N), N)
            .op(ROP_FFT_FWD)
            .op(ROP_ACC_ABS2, nullptr, 0, 0, 0, 0, 1.0 / ((double)N * (double)N))
            .op(ROP_STORE_ACC, W1, nn(N), N);
        if (int rc = run_row<ProgAbs2Tag>(dtype, N, d.p, d.n, stream)) return rc;
        HIP_TRY(launch_ring_sums(W1, N, nb, dtype == PS_F64, S, nullptr, stream));
        if (n_r > 0 || rdiff_out)
            HIP_TRY(launch_hankel(S, N, nb, rpx.data(), n_r, D, rdiff_out ? R : nullptr, stream));
        std::vector<double> hS(S_out ? (size_t)nb * nbins : 0), hD((size_t)nb * n_r), hR(rdiff_out ? nb : 0);
        if (S_out) HIP_TRY(hipMemcpyAsync(hS.data(), S, hS.size() * 8, hipMemcpyDeviceToHost, stream));
        if (n_r > 0) HIP_TRY(hipMemcpyAsync(hD.data(), D, hD.size() * 8, hipMemcpyDeviceToHost, stream));
        if (rdiff_out) HIP_TRY(hipMemcpyAsync(hR.data(), R, hR.size() * 8, hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        // physical units: S in (length unit)^2 rad^2, R_diff^rec in the length unit
        for (size_t i = 0; i < hS.size(); ++i) S_out[(size_t)b0 * nbins + i] = hS[i] * delta * delta;
        for (size_t i = 0; i < hD.size(); ++i) D_out[(size_t)b0 * n_r + i] = hD[i];
        for (int i = 0; i < (int)hR.size(); ++i) {
            rdiff_out[b0 + i] = hR[i] * delta;
            if (!std::isfinite(hR[i])) g_last_warning = "D_rec = 1 is not reached between 1e-3 and N/2 pixels";
        }
    }
    return PS_OK;
}

int ps_l2_loss(int N, const void *I, const void *I_target, int n, int dtype, void *grad_out, double *loss_out,
               void *hip_stream) {
    g_last_error.clear();
    g_last_warning.clear();
    if (int rc = check_common(N, dtype, n)) return rc;
    if (!I || !I_target) return fail(PS_E_NULL, "I and I_target must be non-NULL");
    if (int rc = check_aligned({I, I_target, grad_out})) return rc;
    const size_t rb = (size_t)nn(N) * real_bytes(dtype) * n;
    if (grad_out && (overlaps(grad_out, rb, I, rb) || overlaps(grad_out, rb, I_target, rb)))
        return fail(PS_E_ALIAS, "grad_out overlaps I or I_target");
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    if (loss_out)
        if (int rc = refuse_in_capture(stream, "returning loss_out to the host")) return rc;
    const int64_t per = nn(N);
    const int nblk = block_count(per);
    void *ws = nullptr;
    if (int rc = get_workspace(stream, (size_t)n * nblk * 8 + (size_t)n * 8 + 1024, &ws)) return rc;
    Carver c;
    char *base = static_cast<char *>(ws);
    double *part = reinterpret_cast<double *>(base + c.take((size_t)n * nblk * 8));
    double *tot = reinterpret_cast<double *>(base + c.take((size_t)n * 8));
    HIP_TRY(launch_l2_loss(I, I_target, grad_out, per, n, nblk, dtype == PS_F64, part, stream));
    if (loss_out) {
        HIP_TRY(launch_finalize_sums(part, nblk, n, 1.0, tot, stream));
        std::vector<double> h(n);
        HIP_TRY(hipMemcpyAsync(h.data(), tot, (size_t)n * 8, hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        std::memcpy(loss_out, h.data(), (size_t)n * 8);
    }
    return PS_OK;
}

}  // extern "C"

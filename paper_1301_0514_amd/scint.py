"""ctypes binding of libscint.so (the C ABI in include/scint.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of libscint.so.  PyTorch supplies device memory and the current HIP
stream.  If the library has not been built this module raises on import of
the library (no CPU fallback exists).

Function names and argument order follow the C ABI; arrays are torch tensors
on the current GPU, contiguous, float32 (PS_F32) or float64 (PS_F64).
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libscint.so")

PS_F32, PS_F64 = 0, 1
PS_OK = 0
STATUS_NAMES = {0: "PS_OK", -1: "PS_E_NULL", -2: "PS_E_SIZE", -3: "PS_E_PARAM", -4: "PS_E_DTYPE",
                -5: "PS_E_ALLOC", -6: "PS_E_DEVICE", -7: "PS_E_ALIAS", -8: "PS_E_UNIMPLEMENTED",
                -9: "PS_E_CAPTURE"}
PS_E_CAPTURE = -9

# Every symbol include/scint.h declares, with its ctypes signature.
_c_int, _c_dbl, _c_u32, _c_u64, _vp = ctypes.c_int, ctypes.c_double, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
SIGNATURES = {
    "ps_supported_size": (_c_int, [_c_int, _c_int]),
    "ps_num_supported_sizes": (_c_int, [_c_int]),
    "ps_supported_size_at": (_c_int, [_c_int, _c_int]),
    "ps_generate": (_c_int, [_c_int, _c_dbl, _c_dbl, _c_dbl, _c_u64, _c_u32, _c_int, _c_int, _vp, _vp]),
    "fresnel_propagate": (_c_int, [_c_int, _c_dbl, _c_dbl, _c_dbl, _vp, _c_dbl, _c_int, _c_int, _vp, _vp]),
    "fresnel_propagate_noalloc": (_c_int, [_c_int, _c_dbl, _c_dbl, _c_dbl, _vp, _c_dbl, _c_int, _c_int, _vp,
                                           _vp]),
    "ps_screen_fresnel": (_c_int, [_c_int, _c_dbl, _c_dbl, _c_dbl, _c_u64, _c_u32, _c_int, _c_dbl, _c_dbl,
                                   _c_int, _vp, _vp, _vp, _vp]),
    "fresnel_propagate_field": (_c_int, [_c_int, _c_dbl, _c_dbl, _c_dbl, _vp, _c_dbl, _c_int, _c_int, _vp, _vp,
                                         _vp]),
    "illumination_polychromatic": (_c_int, [_c_int, _c_dbl, _c_dbl, _vp, _c_dbl, _dp, _dp, _c_int, _c_int,
                                            _c_int, _vp, _vp]),
    "source_smear": (_c_int, [_c_int, _c_dbl, _vp, _dp, _c_int, _c_int, _c_int, _vp, _vp]),
    "fresnel_propagate_vjp": (_c_int, [_c_int, _c_dbl, _c_dbl, _c_dbl, _vp, _c_dbl, _vp, _vp, _c_int, _c_int,
                                       _vp, _dp, _vp]),
    "ps_modulation_index": (_c_int, [_c_int, _vp, _c_int, _c_int, _dp, _dp, _vp]),
    "fresnel_aperture": (_c_int, [_c_int, _c_dbl, _c_dbl, _c_dbl, _vp, _c_dbl, _c_dbl, _c_int, _c_int, _vp, _vp]),
    "ps_aperture_geometry": (_c_int, [_c_int, _c_dbl, _c_dbl, _c_dbl, _c_dbl, _c_dbl, _dp,
                                      ctypes.POINTER(_c_int)]),
    "ps_modulation_index_region": (_c_int, [_c_int, _vp, _c_int, _c_int, _c_int, _c_int, _c_int, _c_int, _dp, _dp,
                                            _vp]),
    "ps_light_curves": (_c_int, [_c_int, _vp, _c_int, _dp, _c_int, _c_int, _c_int, _c_int, _vp, _dp, _vp]),
    "ps_m_theory": (_c_int, [_c_dbl, _c_dbl, _c_dbl, _dp]),
    "ps_structure_function": (_c_int, [_c_int, _c_dbl, _vp, _c_int, _dp, _c_int, _c_int, _dp, _dp, _dp, _vp]),
    "ps_l2_loss": (_c_int, [_c_int, _vp, _vp, _c_int, _c_int, _vp, _dp, _vp]),
    "ps_last_error": (ctypes.c_char_p, []),
    "ps_last_warning": (ctypes.c_char_p, []),
    "ps_release_cache": (_c_int, []),
    "ps_version": (_c_int, []),
    "ps_num_plan_variants": (_c_int, [_c_int, _c_int]),
    "ps_plan_variant": (_c_int, [_c_int, _c_int, ctypes.POINTER(_c_int), ctypes.POINTER(ctypes.c_float)]),
    "ps_set_plan_variant": (_c_int, [_c_int, _c_int, _c_int]),
    "ps_tune_plans": (_c_int, [_c_int, _c_int]),
    "ps_set_workspace_budget": (_c_int, [ctypes.c_size_t]),
    "ps_plan_polychromatic": (_c_int, [_c_int, _c_int, _c_int, _c_int, ctypes.c_size_t, ctypes.POINTER(_c_int),
                                       ctypes.POINTER(_c_int), ctypes.POINTER(_c_int), ctypes.POINTER(_c_int),
                                       ctypes.POINTER(ctypes.c_size_t)]),
    "ps_timing_enable": (_c_int, [_c_int]),
    "ps_timing_count": (_c_int, []),
    "ps_timing_entry": (_c_int, [_c_int, ctypes.c_char_p, _c_int, _dp, ctypes.POINTER(ctypes.c_longlong), _dp,
                                 _dp, _dp]),
}

_lock = threading.Lock()
_lib = None


class ScintError(RuntimeError):
    """A libscint entry point returned a non-OK status."""

    def __init__(self, fn: str, code: int, msg: str):
        super().__init__("%s returned %s (%d): %s" % (fn, STATUS_NAMES.get(code, "?"), code, msg))
        self.code = code


def load_library(path: str | None = None) -> ctypes.CDLL:
    """Load libscint.so (built by paper_1301_0514_amd.build) and bind every
    symbol of include/scint.h.  Raises FileNotFoundError if it is not built."""
    global _lib
    with _lock:
        if _lib is not None and path is None:
            return _lib
        p = path or LIB_PATH
        if not os.path.exists(p):
            raise FileNotFoundError("libscint.so not built: run `python -m paper_1301_0514_amd.build` (%s)" % p)
        lib = ctypes.CDLL(p)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        if path is None:
            _lib = lib
        return lib


def _check(fn: str, rc: int) -> None:
    if rc != PS_OK:
        raise ScintError(fn, rc, load_library().ps_last_error().decode())


def _dtype_code(t: torch.dtype) -> int:
    if t == torch.float32:
        return PS_F32
    if t == torch.float64:
        return PS_F64
    raise TypeError("libscint works on float32 or float64 tensors, got %s" % t)


def _ptr(t: torch.Tensor | None):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream(device: torch.device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _host_doubles(vals):
    arr = (ctypes.c_double * len(vals))(*[float(v) for v in vals])
    return arr


def _batch_of(t: torch.Tensor, N: int) -> int:
    if t.dim() < 2 or t.shape[-1] != N or t.shape[-2] != N:
        raise ValueError("expected a [..., N, N] tensor with N=%d, got %s" % (N, tuple(t.shape)))
    return t.numel() // (N * N)


def _check_like(name: str, t: torch.Tensor, shape, dtype: torch.dtype, device: torch.device) -> None:
    """Raise ValueError unless t has exactly the shape, dtype and device the
    library will write or read through it (the C ABI trusts the sizes it is
    given, so a smaller or differently typed buffer would be overrun)."""
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch.Tensor" % name)
    if tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))
    if t.dtype != dtype:
        raise ValueError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if t.device != device:
        raise ValueError("%s must be on %s, got %s" % (name, device, t.device))


# ------------------------------------------------------------------ queries
def supported_size(N: int, dtype: torch.dtype = torch.float32) -> bool:
    return bool(load_library().ps_supported_size(int(N), _dtype_code(dtype)))


def supported_sizes(dtype: torch.dtype = torch.float32) -> list[int]:
    lib = load_library()
    code = _dtype_code(dtype)
    return [lib.ps_supported_size_at(code, i) for i in range(lib.ps_num_supported_sizes(code))]


def last_warning() -> str:
    return load_library().ps_last_warning().decode()


def release_cache() -> None:
    _check("ps_release_cache", load_library().ps_release_cache())


def version() -> int:
    return load_library().ps_version()


def num_plan_variants(N: int, dtype: torch.dtype = torch.float32) -> int:
    return load_library().ps_num_plan_variants(int(N), _dtype_code(dtype))


def plan_variant(N: int, dtype: torch.dtype = torch.float32):
    """(plan in use, tuner times in ms per plan or -1) -- tunes N now if needed."""
    lib = load_library()
    nv = max(1, lib.ps_num_plan_variants(int(N), _dtype_code(dtype)))
    v = _c_int()
    ms = (ctypes.c_float * nv)()
    _check("ps_plan_variant", lib.ps_plan_variant(int(N), _dtype_code(dtype), ctypes.byref(v), ms))
    return v.value, [ms[i] for i in range(nv)]


def set_plan_variant(N: int, variant: int, dtype: torch.dtype = torch.float32) -> None:
    """Pin FFT plan `variant` for size N (-1: back to the tuner's choice)."""
    _check("ps_set_plan_variant", load_library().ps_set_plan_variant(int(N), _dtype_code(dtype), int(variant)))


def tune_plans(N: int, dtype: torch.dtype = torch.float32) -> None:
    """Choose (tuning if needed) the FFT plan of size N and build its tables on
    the current device, so that a later graph capture of size-N calls finds
    nothing to allocate or time."""
    _check("ps_tune_plans", load_library().ps_tune_plans(int(N), _dtype_code(dtype)))


def set_workspace_budget(nbytes: int, device=None) -> None:
    """Cap the workspace the library plans for on `device` (default: the
    current one) at nbytes; 0 restores the default."""
    if int(nbytes) < 0:
        raise ValueError("nbytes must be >= 0")
    with torch.cuda.device(torch.device("cuda") if device is None else torch.device(device)):
        _check("ps_set_workspace_budget", load_library().ps_set_workspace_budget(int(nbytes)))


def plan_polychromatic(N: int, n_real: int, n_lambda: int, budget_bytes: int, dtype=torch.float32) -> dict:
    """The split illumination_polychromatic would use for these sizes under
    the given workspace budget (host arithmetic; no GPU needed)."""
    if int(budget_bytes) <= 0:
        raise ValueError("budget_bytes must be > 0")
    out = [_c_int() for _ in range(4)]
    ws = ctypes.c_size_t()
    _check("ps_plan_polychromatic", load_library().ps_plan_polychromatic(
        int(N), int(n_real), int(n_lambda), _dtype_code(dtype), int(budget_bytes), *[ctypes.byref(o) for o in out],
        ctypes.byref(ws)))
    return {"pipelined": bool(out[0].value), "n_jobs": out[1].value, "lambdas_per_job": out[2].value,
            "real_per_job": out[3].value, "workspace_bytes": ws.value}


def timing_enable(on: bool = True) -> None:
    """Start (clearing totals) or stop per-kernel event timing in the library."""
    _check("ps_timing_enable", load_library().ps_timing_enable(1 if on else 0))


def timing_report() -> dict:
    """{kernel name: {"ms": total, "launches": n, "bytes": algorithmic bytes,
    "schedule_bytes": operand bytes as scheduled, "flops": ...}} for the
    kernels launched while timing was enabled (waits for them)."""
    lib = load_library()
    out = {}
    for i in range(lib.ps_timing_count()):
        buf = ctypes.create_string_buffer(256)
        ms, n = ctypes.c_double(), ctypes.c_longlong()
        b, sb, f = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check("ps_timing_entry", lib.ps_timing_entry(i, buf, 256, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(b),
                                                      ctypes.byref(sb), ctypes.byref(f)))
        out[buf.value.decode()] = {"ms": ms.value, "launches": n.value, "bytes": b.value,
                                   "schedule_bytes": sb.value, "flops": f.value}
    return out


# ------------------------------------------------------------------ entry points
def ps_generate(N, delta, r_diff, beta, seed, first_realisation=0, n_real=1, dtype=torch.float32,
                out: torch.Tensor | None = None, device=None) -> torch.Tensor:
    """Phase screens [n_real, N, N] (radians); see ps_generate in scint.h."""
    device = torch.device(device or "cuda")
    if out is None:
        out = torch.empty((n_real, N, N), dtype=dtype, device=device)
    else:
        _check_like("out", out, (n_real, N, N), out.dtype, out.device)
        _dtype_code(out.dtype)
    rc = load_library().ps_generate(int(N), float(delta), float(r_diff), float(beta), int(seed),
                                    int(first_realisation), int(n_real), _dtype_code(out.dtype),
                                    _ptr(out), _stream(out.device))
    _check("ps_generate", rc)
    return out


def fresnel_propagate(phi: torch.Tensor, delta, lam, z, phase_scale=1.0,
                      out: torch.Tensor | None = None) -> torch.Tensor:
    """Point-source illumination I = |A|^2 of each screen; see scint.h."""
    N = phi.shape[-1]
    n = _batch_of(phi, N)
    if out is None:
        out = torch.empty_like(phi)
    else:
        _check_like("out", out, phi.shape, phi.dtype, phi.device)
    rc = load_library().fresnel_propagate(int(N), float(delta), float(lam), float(z), _ptr(phi),
                                          float(phase_scale), n, _dtype_code(phi.dtype), _ptr(out),
                                          _stream(phi.device))
    _check("fresnel_propagate", rc)
    return out


def fresnel_propagate_noalloc(phi: torch.Tensor, delta, lam, z, phase_scale=1.0,
                              out: torch.Tensor | None = None) -> torch.Tensor:
    """fresnel_propagate through the entry point that allocates no device
    memory (its intermediates live in the library's fixed scratch array);
    see scint.h.  With `out` given, the call itself allocates nothing."""
    N = phi.shape[-1]
    n = _batch_of(phi, N)
    if out is None:
        out = torch.empty_like(phi)
    else:
        _check_like("out", out, phi.shape, phi.dtype, phi.device)
    rc = load_library().fresnel_propagate_noalloc(int(N), float(delta), float(lam), float(z), _ptr(phi),
                                                  float(phase_scale), n, _dtype_code(phi.dtype), _ptr(out),
                                                  _stream(phi.device))
    _check("fresnel_propagate_noalloc", rc)
    return out


def fresnel_aperture(phi: torch.Tensor, delta, lam, z, phase_scale=1.0, margin_rf=10.0,
                     out: torch.Tensor | None = None) -> torch.Tensor:
    """Aperture mode: one-FFT Fresnel pattern of the windowed screen on the
    observer grid of pixel lam z / (N delta); see scint.h."""
    N = phi.shape[-1]
    n = _batch_of(phi, N)
    if out is None:
        out = torch.empty_like(phi)
    else:
        _check_like("out", out, phi.shape, phi.dtype, phi.device)
    rc = load_library().fresnel_aperture(int(N), float(delta), float(lam), float(z), _ptr(phi), float(phase_scale),
                                         float(margin_rf), n, _dtype_code(phi.dtype), _ptr(out), _stream(phi.device))
    _check("fresnel_aperture", rc)
    return out


def aperture_geometry(N, delta, lam, z, r_diff, r_s=0.0):
    """(observer pixel, fiducial margin in observer pixels) of the aperture
    mode; host arithmetic, see scint.h."""
    pix = ctypes.c_double(0.0)
    margin = _c_int(0)
    rc = load_library().ps_aperture_geometry(int(N), float(delta), float(lam), float(z), float(r_diff), float(r_s),
                                             ctypes.byref(pix), ctypes.byref(margin))
    _check("ps_aperture_geometry", rc)
    return pix.value, margin.value


def ps_screen_fresnel(N, delta, r_diff, beta, seed, lam, z, first_realisation=0, n_real=1,
                      dtype=torch.float32, want_phi=False, want_field=False, device=None):
    """Screen generation and propagation fused; returns I, then phi and the
    adjoint's field checkpoint [n_real, N, N, 2] ([b][x][y], re/im) if asked."""
    device = torch.device(device or "cuda")
    I = torch.empty((n_real, N, N), dtype=dtype, device=device)
    phi = torch.empty_like(I) if want_phi else None
    field = torch.empty((n_real, N, N, 2), dtype=dtype, device=device) if want_field else None
    rc = load_library().ps_screen_fresnel(int(N), float(delta), float(r_diff), float(beta), int(seed),
                                          int(first_realisation), int(n_real), float(lam), float(z),
                                          _dtype_code(dtype), _ptr(phi), _ptr(I), _ptr(field), _stream(device))
    _check("ps_screen_fresnel", rc)
    out = (I,) + ((phi,) if want_phi else ()) + ((field,) if want_field else ())
    return out if len(out) > 1 else I


def fresnel_propagate_field(phi: torch.Tensor, delta, lam, z, phase_scale=1.0):
    """(I, field): the pattern and the complex field A kept as the adjoint's
    checkpoint, [..., N, N, 2] in the [b][x][y] layout; see scint.h."""
    N = phi.shape[-1]
    n = _batch_of(phi, N)
    out = torch.empty_like(phi)
    field = torch.empty(tuple(phi.shape) + (2,), dtype=phi.dtype, device=phi.device)
    rc = load_library().fresnel_propagate_field(int(N), float(delta), float(lam), float(z), _ptr(phi),
                                                float(phase_scale), n, _dtype_code(phi.dtype), _ptr(out), _ptr(field),
                                                _stream(phi.device))
    _check("fresnel_propagate_field", rc)
    return out, field


def illumination_polychromatic(phi_ref: torch.Tensor, delta, z, lam_ref, lambdas, weights=None,
                               out: torch.Tensor | None = None) -> torch.Tensor:
    """Co-added illumination over the wavelengths; see scint.h."""
    N = phi_ref.shape[-1]
    n = _batch_of(phi_ref, N)
    if out is None:
        out = torch.empty_like(phi_ref)
    else:
        _check_like("out", out, phi_ref.shape, phi_ref.dtype, phi_ref.device)
    lam = _host_doubles(lambdas)
    w = None if weights is None else _host_doubles(weights)
    if w is not None and len(weights) != len(lambdas):
        raise ValueError("weights and lambdas differ in length")
    rc = load_library().illumination_polychromatic(int(N), float(delta), float(z), _ptr(phi_ref), float(lam_ref),
                                                   lam, w, len(lambdas), n, _dtype_code(phi_ref.dtype),
                                                   _ptr(out), _stream(phi_ref.device))
    _check("illumination_polychromatic", rc)
    return out


def source_smear(I: torch.Tensor, delta, radii, out: torch.Tensor | None = None) -> torch.Tensor:
    """Extended-source patterns [n_real, n_r, N, N]; see scint.h."""
    N = I.shape[-1]
    n = _batch_of(I, N)
    if out is None:
        out = torch.empty((n, len(radii), N, N), dtype=I.dtype, device=I.device)
    else:
        _check_like("out", out, (n, len(radii), N, N), I.dtype, I.device)
    rc = load_library().source_smear(int(N), float(delta), _ptr(I), _host_doubles(radii), len(radii), n,
                                     _dtype_code(I.dtype), _ptr(out), _stream(I.device))
    _check("source_smear", rc)
    return out


def fresnel_propagate_vjp(phi: torch.Tensor, delta, lam, z, grad_I: torch.Tensor, phase_scale=1.0,
                          out: torch.Tensor | None = None, want_dot=False, field: torch.Tensor | None = None):
    """dL/dphi for dL/dI = grad_I, from the forward's field checkpoint if
    given (else the forward is recomputed); optionally also
    sum(phi * dL/dphi) per screen."""
    N = phi.shape[-1]
    n = _batch_of(phi, N)
    _check_like("grad_I", grad_I, phi.shape, phi.dtype, phi.device)
    if field is not None:
        _check_like("field", field, tuple(phi.shape) + (2,), phi.dtype, phi.device)
    if out is None:
        out = torch.empty_like(phi)
    else:
        _check_like("out", out, phi.shape, phi.dtype, phi.device)
    dots = (ctypes.c_double * n)() if want_dot else None
    rc = load_library().fresnel_propagate_vjp(int(N), float(delta), float(lam), float(z), _ptr(phi),
                                              float(phase_scale), _ptr(grad_I), _ptr(field), n,
                                              _dtype_code(phi.dtype), _ptr(out), dots, _stream(phi.device))
    _check("fresnel_propagate_vjp", rc)
    return (out, [dots[i] for i in range(n)]) if want_dot else out


def ps_modulation_index(I: torch.Tensor, want_mean=False):
    """m = sigma_I / mean(I) per pattern (FP64 accumulation); synchronises."""
    N = I.shape[-1]
    n = _batch_of(I, N)
    m = (ctypes.c_double * n)()
    mean = (ctypes.c_double * n)()
    rc = load_library().ps_modulation_index(int(N), _ptr(I), n, _dtype_code(I.dtype), m, mean,
                                            _stream(I.device))
    _check("ps_modulation_index", rc)
    ms = [m[i] for i in range(n)]
    return (ms, [mean[i] for i in range(n)]) if want_mean else ms


def ps_modulation_index_region(I: torch.Tensor, x0: int, y0: int, w: int, h: int, want_mean=False):
    """m (and the mean) over the w x h rectangle starting at pixel (x0, y0) of
    each pattern, e.g. a fiducial zone; synchronises."""
    N = I.shape[-1]
    n = _batch_of(I, N)
    m = (ctypes.c_double * n)()
    mean = (ctypes.c_double * n)()
    rc = load_library().ps_modulation_index_region(int(N), _ptr(I), n, int(x0), int(y0), int(w), int(h),
                                                   _dtype_code(I.dtype), m, mean, _stream(I.device))
    _check("ps_modulation_index_region", rc)
    ms = [m[i] for i in range(n)]
    return (ms, [mean[i] for i in range(n)]) if want_mean else ms


def light_curves(I: torch.Tensor, lines, n_samples: int, mode: int = 0, want_m: bool = True):
    """Samples of each pattern along straight lines (x0, y0, dx, dy) in pixels
    (Sect. 3.3): returns curves [n, n_lines, n_samples] and, if asked, m of
    each curve as a nested list [n][n_lines] (synchronises); see scint.h."""
    N = I.shape[-1]
    n = _batch_of(I, N)
    flat = [float(v) for line in lines for v in line]
    n_lines = len(flat) // 4
    if n_lines * 4 != len(flat) or n_lines < 1:
        raise ValueError("lines must be a non-empty list of (x0, y0, dx, dy)")
    arr = (ctypes.c_double * len(flat))(*flat)
    curves = torch.empty((n, n_lines, int(n_samples)), dtype=I.dtype, device=I.device)
    m = (ctypes.c_double * (n * n_lines))() if want_m else None
    rc = load_library().ps_light_curves(int(N), _ptr(I), n, arr, n_lines, int(n_samples), int(mode),
                                        _dtype_code(I.dtype), _ptr(curves), m, _stream(I.device))
    _check("ps_light_curves", rc)
    if not want_m:
        return curves
    return curves, [[m[b * n_lines + l] for l in range(n_lines)] for b in range(n)]


def structure_function(phi: torch.Tensor, delta, radii=(), want_spectrum=False):
    """Recomputed structure function of each screen (Sect. 3.1.1, Eq. crec):
    returns (D [n][len(radii)], R_diff^rec [n]) and, if asked, the ring
    spectrum S_rec [n][N/2 + 1] (q_b = b / (N delta)); synchronises."""
    N = phi.shape[-1]
    n = _batch_of(phi, N)
    nr = len(radii)
    r = (ctypes.c_double * max(nr, 1))(*[float(v) for v in radii])
    D = (ctypes.c_double * max(n * nr, 1))()
    R = (ctypes.c_double * n)()
    S = (ctypes.c_double * (n * (N // 2 + 1)))() if want_spectrum else None
    rc = load_library().ps_structure_function(int(N), float(delta), _ptr(phi), n, r if nr else None, nr,
                                              _dtype_code(phi.dtype), S, D if nr else None, R, _stream(phi.device))
    _check("ps_structure_function", rc)
    Ds = [[D[b * nr + j] for j in range(nr)] for b in range(n)]
    Rs = [R[b] for b in range(n)]
    if want_spectrum:
        return Ds, Rs, [[S[b * (N // 2 + 1) + k] for k in range(N // 2 + 1)] for b in range(n)]
    return Ds, Rs


def m_theory(r_diff, r_f, r_s) -> float:
    """Expected m of an extended source (Sect. 4.1, Eq. xparam); host only."""
    m = ctypes.c_double(0.0)
    _check("ps_m_theory", load_library().ps_m_theory(float(r_diff), float(r_f), float(r_s), ctypes.byref(m)))
    return m.value


def ps_l2_loss(I: torch.Tensor, I_target: torch.Tensor, want_grad=True):
    """L = sum (I - I_t)^2 per pattern and dL/dI = 2 (I - I_t)."""
    N = I.shape[-1]
    n = _batch_of(I, N)
    _check_like("I_target", I_target, I.shape, I.dtype, I.device)
    grad = torch.empty_like(I) if want_grad else None
    loss = (ctypes.c_double * n)()
    rc = load_library().ps_l2_loss(int(N), _ptr(I), _ptr(I_target), n, _dtype_code(I.dtype), _ptr(grad), loss,
                                   _stream(I.device))
    _check("ps_l2_loss", rc)
    return [loss[i] for i in range(n)], grad


# ------------------------------------------------------------------ graphs
def capture_graph(fn, warmup: int = 1, stream: torch.cuda.Stream | None = None):
    """Capture fn() (a sequence of libscint calls on the current stream) into
    a HIP graph.  fn runs `warmup` times first on the capture stream, so that
    the library's per-stream workspace and its cached tables exist and the
    captured calls allocate nothing.  Returns (graph, stream); replay with
    graph.replay() under `with torch.cuda.stream(stream)`."""
    stream = stream or torch.cuda.Stream()
    with torch.cuda.stream(stream):
        for _ in range(max(1, warmup)):
            fn()
    stream.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        fn()
    stream.synchronize()
    return g, stream


# ------------------------------------------------------------------ autograd
class FresnelIntensity(torch.autograd.Function):
    """I = fresnel_propagate(phi) with the hand-written adjoint as backward;
    the forward keeps the complex field as the adjoint's checkpoint, so the
    backward runs the adjoint passes only."""

    @staticmethod
    def forward(ctx, phi, delta, lam, z, phase_scale):
        phi = phi.contiguous()
        I, field = fresnel_propagate_field(phi, delta, lam, z, phase_scale)
        ctx.save_for_backward(phi, field)
        ctx.args = (delta, lam, z, phase_scale)
        return I

    @staticmethod
    def backward(ctx, grad_I):
        phi, field = ctx.saved_tensors
        delta, lam, z, s = ctx.args
        g = fresnel_propagate_vjp(phi, delta, lam, z, grad_I.contiguous(), s, field=field)
        return g, None, None, None, None


def fresnel_intensity(phi, delta, lam, z, phase_scale=1.0):
    """Differentiable propagation: gradients flow to phi through the adjoint kernels."""
    return FresnelIntensity.apply(phi, delta, lam, z, phase_scale)

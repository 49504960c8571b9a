"""FP64 CPU oracle for the phase-screen + Fresnel propagation method.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only users.  The GPU library never imports this
module and this module never imports the GPU library.

The arithmetic lives in ``scint_oracle.c`` (plain C99, double precision, its
own Philox generator and its own mixed-radix DFT); this file only builds it
with gcc and marshals numpy arrays through ctypes.

Each function cites the passage of Habibi et al. (A&A 2013, arXiv:1301.0514)
that it follows.  All lengths are in pixels unless the name says otherwise.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "scint_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile scint_oracle.c into liboracle.so with gcc (-O2, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall",
               "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            dp = ctypes.POINTER(ctypes.c_double)
            u32p = ctypes.POINTER(ctypes.c_uint32)
            u64p = ctypes.POINTER(ctypes.c_uint64)
            c_int, c_dbl, c_u32, c_u64 = ctypes.c_int, ctypes.c_double, ctypes.c_uint32, ctypes.c_uint64
            sig = {
                "oracle_philox4x32_10": (None, [u32p, u32p, u32p]),
                "oracle_philox4x64_10": (None, [u64p, u64p, u64p]),
                "oracle_normals": (None, [c_int, c_u64, c_u32, dp]),
                "oracle_dft1": (None, [c_int, dp, dp, c_int]),
                "oracle_dft2": (None, [c_int, dp, c_int]),
                "oracle_f_beta": (c_dbl, [c_dbl]),
                "oracle_spectrum": (c_dbl, [c_dbl, c_dbl, c_dbl]),
                "oracle_spectrum_coeffs": (None, [c_int, c_dbl, c_dbl, c_u64, c_u32, dp]),
                "oracle_screen": (None, [c_int, c_dbl, c_dbl, c_u64, c_u32, dp]),
                "oracle_propagate": (None, [c_int, c_dbl, c_dbl, dp, dp, dp]),
                "oracle_fresnel": (None, [c_int, c_dbl, c_dbl, c_dbl, c_dbl, dp, dp]),
                "oracle_fresnel_radius_px": (c_dbl, [c_dbl, c_dbl, c_dbl]),
                "oracle_fresnel_direct": (None, [c_int, c_dbl, dp, dp]),
                "oracle_fresnel_onefft": (None, [c_int, c_dbl, dp, dp]),
                "oracle_polychromatic": (None, [c_int, c_dbl, c_dbl, dp, c_dbl, dp, dp, c_int, dp]),
                "oracle_smear": (None, [c_int, dp, c_dbl, dp]),
                "oracle_smear_direct": (None, [c_int, dp, c_dbl, dp]),
                "oracle_disk_count": (c_dbl, [c_int, c_dbl]),
                "oracle_modulation_index": (c_dbl, [c_int, dp]),
                "oracle_sf_window": (None, [c_int, c_dbl, dp]),
                "oracle_fresnel_aperture": (None, [c_int, c_dbl, c_dbl, c_dbl, dp, dp]),
                "oracle_fresnel_aperture_direct": (None, [c_int, c_dbl, c_dbl, c_dbl, dp, dp]),
                "oracle_modulation_index_region": (c_dbl, [c_int, dp, c_int, c_int, c_int, c_int, dp]),
                "oracle_light_curves": (None, [c_int, dp, c_int, dp, c_int, c_int, dp, dp]),
                "oracle_propagate_line": (None, [c_int, c_dbl, c_dbl, dp, dp]),
                "oracle_ring_spectrum": (None, [c_int, dp, dp, dp]),
                "oracle_structure_from_spectrum": (c_dbl, [c_int, dp, c_dbl]),
                "oracle_rdiff_rec": (c_dbl, [c_int, dp]),
                "oracle_m_theory": (c_dbl, [c_dbl, c_dbl, c_dbl]),
                "oracle_propagate_vjp": (None, [c_int, c_dbl, c_dbl, dp, dp, dp]),
                "oracle_propagate_adjoint_field": (None, [c_int, c_dbl, dp, dp]),
                "oracle_propagate_field": (None, [c_int, c_dbl, dp, dp]),
                "oracle_num_threads": (c_int, []),
                "oracle_set_num_threads": (None, [c_int]),
            }
            for name, (res, args) in sig.items():
                fn = getattr(lib, name)
                fn.restype = res
                fn.argtypes = args
            _lib = lib
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _c128(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.complex128)


# ---------------------------------------------------------------- generators
def philox4x32_10(counter, key) -> np.ndarray:
    """Philox4x32-10 block (Salmon et al. SC'11) for one counter and key."""
    c = np.ascontiguousarray(counter, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    p = ctypes.POINTER(ctypes.c_uint32)
    _load().oracle_philox4x32_10(c.ctypes.data_as(p), k.ctypes.data_as(p), out.ctypes.data_as(p))
    return out


def philox4x64_10(counter, key) -> np.ndarray:
    """Philox4x64-10 block; the same round structure with 64-bit words."""
    c = np.ascontiguousarray(counter, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    p = ctypes.POINTER(ctypes.c_uint64)
    _load().oracle_philox4x64_10(c.ctypes.data_as(p), k.ctypes.data_as(p), out.ctypes.data_as(p))
    return out


def normals(N: int, seed: int, r: int = 0) -> np.ndarray:
    """Complex standard normals g[ky, kx] (unit variance per part) of one
    realisation: one random complex number per Fourier pixel (Sect. 3.1)."""
    g = np.zeros((N, N, 2), dtype=np.float64)
    _load().oracle_normals(N, seed, r, _dp(g))
    return g[..., 0] + 1j * g[..., 1]


# ---------------------------------------------------------------------- DFT
def dft1(x, sign: int = -1) -> np.ndarray:
    """Own unnormalised 1-D DFT, out[k] = sum_j x[j] exp(sign 2 pi i j k / n)."""
    x = _c128(x)
    out = np.zeros_like(x)
    _load().oracle_dft1(x.size, _dp(x.view(np.float64)), _dp(out.view(np.float64)), int(sign))
    return out


def dft2(a, sign: int = -1) -> np.ndarray:
    """Own unnormalised 2-D DFT of an N x N array."""
    a = _c128(a).copy()
    N = a.shape[0]
    assert a.shape == (N, N)
    _load().oracle_dft2(N, _dp(a.view(np.float64)), int(sign))
    return a


# ----------------------------------------------------------------- spectrum
def f_beta(beta: float) -> float:
    """f(beta) = 2^-beta beta Gamma(-beta/2)/Gamma(beta/2) (Sect. 2, Eq. spectre)."""
    return _load().oracle_f_beta(beta)


def spectrum(q: float, R: float, beta: float) -> float:
    """Phase spectral density S(q), q in cycles per pixel (Sect. 2, Eq. spectre)."""
    return _load().oracle_spectrum(q, R, beta)


def spectrum_coeffs(N: int, R: float, beta: float, seed: int, r: int = 0) -> np.ndarray:
    """Random phase spectrum c = F_phi/(L_x L_y) on the FFT grid (Sect. 3.1, Eq. densite)."""
    c = np.zeros((N, N), dtype=np.complex128)
    _load().oracle_spectrum_coeffs(N, R, beta, seed, r, _dp(c.view(np.float64)))
    return c


def screen(N: int, R: float, beta: float, seed: int, r: int = 0) -> np.ndarray:
    """Phase screen phi (radians), the inverse Fourier transform of the random
    spectrum, phi = sqrt(2) Re(...) (Sect. 3.1)."""
    phi = np.zeros((N, N), dtype=np.float64)
    _load().oracle_screen(N, R, beta, seed, r, _dp(phi))
    return phi


# -------------------------------------------------------------- propagation
def fresnel_radius_px(delta: float, lam: float, z: float) -> float:
    """R_F = sqrt(lambda z / 2 pi) in pixels of side delta (Sect. 2, Eq. Rfresnel)."""
    return _load().oracle_fresnel_radius_px(delta, lam, z)


def propagate(phi, rho: float, s: float = 1.0, return_field: bool = False):
    """Illumination I = |A|^2 of a unit plane wave through the periodic screen
    s*phi at Fresnel radius rho pixels (Sect. 2, Eq. hxy, transfer-function form)."""
    phi = _f64(phi)
    N = phi.shape[0]
    out = np.zeros((N, N), dtype=np.float64)
    if return_field:
        A = np.zeros((N, N), dtype=np.complex128)
        _load().oracle_propagate(N, rho, s, _dp(phi), _dp(out), _dp(A.view(np.float64)))
        return out, A
    _load().oracle_propagate(N, rho, s, _dp(phi), _dp(out), None)
    return out


def fresnel(phi, delta: float, lam: float, z: float, s: float = 1.0) -> np.ndarray:
    """propagate() with physical arguments (one length unit for delta, lambda, z)."""
    phi = _f64(phi)
    N = phi.shape[0]
    out = np.zeros((N, N), dtype=np.float64)
    _load().oracle_fresnel(N, delta, lam, z, s, _dp(phi), _dp(out))
    return out


def fresnel_direct(phi, rho: float) -> np.ndarray:
    """Direct O(N^4) sum of Eq. hxy over the finite screen (Sect. 2)."""
    phi = _f64(phi)
    N = phi.shape[0]
    out = np.zeros((N, N), dtype=np.float64)
    _load().oracle_fresnel_direct(N, rho, _dp(phi), _dp(out))
    return out


def fresnel_onefft(phi, rho: float) -> np.ndarray:
    """The paper's one-FFT numerics without the smoothing window (Sect. 3.2,
    Eqs. intens and Gxy), valid on the screen grid when N = 2 pi rho^2."""
    phi = _f64(phi)
    N = phi.shape[0]
    out = np.zeros((N, N), dtype=np.float64)
    _load().oracle_fresnel_onefft(N, rho, _dp(phi), _dp(out))
    return out


def sf_window(N: int, margin_px: float) -> np.ndarray:
    """The smoothing window SF at the N pixel centres for a margin of
    margin_px pixels on each border (Sect. 3.2.1); margin 0 = no window."""
    out = np.zeros(N, dtype=np.float64)
    _load().oracle_sf_window(N, margin_px, _dp(out))
    return out


def fresnel_aperture(phi, rho: float, s: float = 1.0, margin_rf: float = 10.0) -> np.ndarray:
    """Aperture mode (Sect. 3.2, Eqs. intens and Gxy, with the window of
    Sect. 3.2.1): |FT[SF SF G]|^2 / (2 pi rho^2)^2 on the observer grid of
    pixel 2 pi rho^2 / N, centred (observer pixel N/2 faces screen pixel N/2).
    margin_rf = L_m / R_F (the paper uses 10; 0 = no window)."""
    phi = _f64(phi)
    N = phi.shape[0]
    out = np.zeros((N, N), dtype=np.float64)
    _load().oracle_fresnel_aperture(N, rho, s, margin_rf, _dp(phi), _dp(out))
    return out


def fresnel_aperture_direct(phi, rho: float, s: float = 1.0, margin_rf: float = 10.0) -> np.ndarray:
    """The aperture-mode intensity from the Fresnel sum (Eq. hxy) at each
    observer point, O(N^4): for small N only."""
    phi = _f64(phi)
    N = phi.shape[0]
    out = np.zeros((N, N), dtype=np.float64)
    _load().oracle_fresnel_aperture_direct(N, rho, s, margin_rf, _dp(phi), _dp(out))
    return out


def modulation_index_region(I, x0: int, y0: int, w: int, h: int):
    """(m, mean) over the w x h rectangle starting at pixel (x0, y0): the
    statistics inside a fiducial zone (Sect. 3.2.1, Sect. 4)."""
    I = _f64(I)
    mean = ctypes.c_double(0.0)
    m = _load().oracle_modulation_index_region(I.shape[0], _dp(I), x0, y0, w, h, ctypes.byref(mean))
    return m, mean.value


def light_curves(I, lines, n_samples: int, mode: int = 0):
    """Light curves (Sect. 3.3): samples of the periodic pattern I along
    straight lines, lines[l] = (x0, y0, dx, dy) in pixels (pixel (ix, iy) at the
    integer point), mode 0 nearest pixel, 1 bilinear.  Returns (curves
    [n_lines, n_samples], m per curve)."""
    I = _f64(I)
    L = _f64(np.atleast_2d(lines))
    n_lines = L.shape[0]
    curves = np.zeros((n_lines, n_samples), dtype=np.float64)
    m = np.zeros(n_lines, dtype=np.float64)
    _load().oracle_light_curves(I.shape[0], _dp(I), n_lines, _dp(L), n_samples, mode, _dp(curves), _dp(m))
    return curves, m


def m_theory(r_diff: float, r_f: float, r_s: float) -> float:
    """Expected m of an extended source, strong quenched regime, Kolmogorov
    (Sect. 4.1, Eq. xparam): (R_diff/R_F)^(1/3) (R_ref/(2 pi R_s))^(7/6)."""
    return _load().oracle_m_theory(r_diff, r_f, r_s)


def ring_spectrum(phi):
    """(S_rec[b], count[b]) for b = 0..N/2: the ring-averaged spectral density
    |DFT phi|^2 / N^2 of a screen (Sect. 3.1.1), pixel units."""
    phi = _f64(phi)
    N = phi.shape[0]
    S = np.zeros(N // 2 + 1)
    c = np.zeros(N // 2 + 1)
    _load().oracle_ring_spectrum(N, _dp(phi), _dp(S), _dp(c))
    return S, c


def structure_from_spectrum(N: int, S, r: float) -> float:
    """D_rec(r) = 2 (xi(0) - xi(r)) from a ring spectrum (Eq. crec), pixels."""
    S = _f64(S)
    return _load().oracle_structure_from_spectrum(N, _dp(S), float(r))


def rdiff_rec(N: int, S) -> float:
    """R_diff^rec (pixels): D_rec(R) = 1, by bisection (NaN if not bracketed)."""
    S = _f64(S)
    return _load().oracle_rdiff_rec(N, _dp(S))


def propagate_line(phi_1d, rho: float, s: float = 1.0) -> np.ndarray:
    """Field a = N^-1 IDFT[H1 DFT exp(i s phi)] along one line of N pixels;
    for phi(x, y) = f(x) + g(y) the 2-D intensity is |a_g(y)|^2 |a_f(x)|^2."""
    phi = _f64(phi_1d)
    out = np.zeros(phi.shape[0], dtype=np.complex128)
    _load().oracle_propagate_line(phi.shape[0], rho, s, _dp(phi), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out


def propagate_field(field, rho: float) -> np.ndarray:
    """The linear propagation alone applied to a complex field."""
    f = _c128(field)
    N = f.shape[0]
    out = np.zeros_like(f)
    _load().oracle_propagate_field(N, rho, _dp(f.view(np.float64)), _dp(out.view(np.float64)))
    return out


def propagate_adjoint_field(field, rho: float) -> np.ndarray:
    """Adjoint of the linear propagation (conjugate transfer function)."""
    f = _c128(field)
    N = f.shape[0]
    out = np.zeros_like(f)
    _load().oracle_propagate_adjoint_field(N, rho, _dp(f.view(np.float64)), _dp(out.view(np.float64)))
    return out


def polychromatic(phi_ref, delta: float, z: float, lam_ref: float, lambdas, weights=None) -> np.ndarray:
    """Co-added illumination over wavelengths for one screen (Sect. 3.2.4); the
    phase scales as lambda_ref/lambda (Sect. 2, Eq. phiNl)."""
    phi = _f64(phi_ref)
    N = phi.shape[0]
    lam = _f64(lambdas)
    out = np.zeros((N, N), dtype=np.float64)
    w = None if weights is None else _f64(weights)
    _load().oracle_polychromatic(N, delta, z, _dp(phi), lam_ref, _dp(lam),
                                 None if w is None else _dp(w), lam.size, _dp(out))
    return out


def smear(I, Rs_px: float) -> np.ndarray:
    """Extended-source pattern I_ext = P_r * I with a uniform disk of radius
    Rs_px pixels, by DFT (Sect. 3.2.3, Eq. iprh)."""
    I = _f64(I)
    N = I.shape[0]
    out = np.zeros((N, N), dtype=np.float64)
    _load().oracle_smear(N, _dp(I), Rs_px, _dp(out))
    return out


def smear_direct(I, Rs_px: float) -> np.ndarray:
    """Direct circular convolution with the same disk (Sect. 3.2.3)."""
    I = _f64(I)
    N = I.shape[0]
    out = np.zeros((N, N), dtype=np.float64)
    _load().oracle_smear_direct(N, _dp(I), Rs_px, _dp(out))
    return out


def disk_count(N: int, Rs_px: float) -> int:
    return int(_load().oracle_disk_count(N, Rs_px))


def modulation_index(I) -> float:
    """m = sigma_I / mean(I), population sigma (Sect. 4)."""
    I = _f64(I)
    return _load().oracle_modulation_index(I.shape[0], _dp(I))


def propagate_vjp(phi, rho: float, s: float, grad_I) -> np.ndarray:
    """dL/dphi for a loss L(I) with dL/dI = grad_I (adjoint of the propagation)."""
    phi = _f64(phi)
    g = _f64(grad_I)
    N = phi.shape[0]
    out = np.zeros((N, N), dtype=np.float64)
    _load().oracle_propagate_vjp(N, rho, s, _dp(phi), _dp(g), _dp(out))
    return out


def num_threads() -> int:
    return _load().oracle_num_threads()


def set_num_threads(n: int) -> None:
    _load().oracle_set_num_threads(int(n))

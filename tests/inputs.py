"""Seeded synthetic inputs shared by the GPU tests and the oracle calls.

Holds no arithmetic of the method: only random fields drawn with numpy's
generator from a seed.  (The method's own noise, Philox4x32-10, is drawn by
each side from its own implementation of the published generator.)
"""
import numpy as np


def phase_field(N, seed, sigma=3.0, n=1):
    """Gaussian random phases (radians), shape [n, N, N], float64."""
    rng = np.random.default_rng(seed)
    return sigma * rng.standard_normal((n, N, N))


def smooth_phase_field(N, seed, sigma=6.0, corr=4.0, n=1):
    """Gaussian random phases with a Gaussian correlation of `corr` pixels
    (low-pass filtered white noise, normalised to rms sigma)."""
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((n, N, N))
    k = np.fft.fftfreq(N)
    filt = np.exp(-0.5 * (2 * np.pi * corr) ** 2 * (k[None, :] ** 2 + k[:, None] ** 2))
    f = np.real(np.fft.ifft2(np.fft.fft2(w) * filt))
    return sigma * f / f.std()


def intensity_field(N, seed, n=1):
    """Positive speckle-like intensities (unit exponential), [n, N, N]."""
    rng = np.random.default_rng(seed)
    return rng.exponential(1.0, (n, N, N))


def line_phase(N, seed, sigma=3.0, corr=4.0):
    """One line of Gaussian random phases with a Gaussian correlation of
    `corr` pixels (periodic), float64 [N]."""
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(N)
    k = np.fft.fftfreq(N)
    f = np.real(np.fft.ifft(np.fft.fft(w) * np.exp(-0.5 * (2 * np.pi * corr * k) ** 2)))
    return sigma * f / f.std()

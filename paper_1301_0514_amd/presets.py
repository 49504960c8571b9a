"""Named workloads in pixel units (pixel side delta = 1).

Lengths: lambda and z enter only through the Fresnel radius
rho = sqrt(lambda z / 2 pi) pixels, so each preset fixes lambda (a label in
metres) and sets z = 2 pi rho^2 / lambda.  R is the diffraction radius
R_diff in pixels and beta the spectral exponent of the phase spectrum.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field


def z_for_rho(rho: float, lam: float, delta: float = 1.0) -> float:
    """Screen-observer distance giving a Fresnel radius of rho pixels."""
    return 2.0 * math.pi * (rho * delta) ** 2 / lam


@dataclass
class Mono:
    N: int
    rho: float
    R: float
    beta: float = 11.0 / 3.0
    lam: float = 5e-7
    seeds: tuple = (1,)
    dtype: str = "float32"

    @property
    def z(self) -> float:
        return z_for_rho(self.rho, self.lam)


@dataclass
class Poly:
    """Polychromatic + extended source: the screen is given at lam_ref."""
    N: int = 8192
    rho_ref: float = 90.0
    R_ref: float = 30.0
    beta: float = 11.0 / 3.0
    lam_ref: float = 650e-9
    lambdas: list = field(default_factory=lambda: [400e-9 + j * 500e-9 / 31 for j in range(32)])
    n_real: int = 8
    seed: int = 1
    smear_radii_over_rf: tuple = (0.5, 1.0, 2.0, 4.0)

    @property
    def z(self) -> float:
        return z_for_rho(self.rho_ref, self.lam_ref)

    @property
    def smear_radii(self) -> list:
        return [f * self.rho_ref for f in self.smear_radii_over_rf]


# Plain method in FP64 on a 256^2 grid, R_F = 32 px, R_diff = 4 px.
PLAIN_FP64 = Mono(N=256, rho=32.0, R=4.0, lam=500e-9, seeds=(1,), dtype="float64")
# Single wavelength, 4096^2, R_F = 64 px, R_diff in {8, 32, 128}, seeds 1..4.
SINGLE_4096 = [Mono(N=4096, rho=64.0, R=R, lam=600e-9, seeds=(1, 2, 3, 4)) for R in (8.0, 32.0, 128.0)]
# Paper-scale grids, R_F = 100 px, R_diff = 30 px.
PAPER_SCALE = [Mono(N=N, rho=100.0, R=30.0, beta=b, lam=500e-9) for N in (10000, 16384)
               for b in (3.2, 11.0 / 3.0, 3.9, 3.1)]
# Batched polychromatic + extended source, 8192^2, 32 wavelengths in 400-900 nm, 8 realisations.
POLY_8192 = Poly()
# Differentiation: 16 realisations of 2048^2, R_F = 48 px, R_diff = 24 px.
GRAD_2048 = Mono(N=2048, rho=48.0, R=24.0, lam=500e-9, seeds=(1,))
GRAD_N_REAL = 16
GRAD_TARGET_SEED0 = 1000


# The paper's own scale (Sect. 3.2.4, Figs. pattern and multypoint): 20000^2
# pixels of 22.6 km, R_diff = 100 km at 2.16 um, screen at 160 pc (R_F = 1300 km
# = 57.5 px, R_diff = 4.42 px), the K_s passband as 21 wavelengths regularly
# spaced in [2.08, 2.28] um with equal weights.
PC_M = 3.0856775814913673e16


@dataclass(frozen=True)
class KsBand:
    N: int = 20000
    delta: float = 22.6e3  # m
    r_diff: float = 100e3  # m, at lam_ref
    z: float = 160 * PC_M  # m
    lam_ref: float = 2.16e-6
    band: tuple = (2.08e-6, 2.28e-6)
    n_lambda: int = 21
    seed: int = 1

    def lambdas(self, n=None):
        n = self.n_lambda if n is None else n
        lo, hi = self.band
        return [0.5 * (lo + hi)] if n == 1 else [lo + (hi - lo) * j / (n - 1) for j in range(n)]


PAPER_KS_20000 = KsBand()

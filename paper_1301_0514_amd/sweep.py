"""Modulation index of simulated extended-source patterns against its expected
value (Sect. 4.1, Eq. xparam and Fig. mx).

For each diffraction radius a series of screens is generated and propagated
on the GPU, each pattern is smeared by the projected disks of the stellar
radii, and m is taken over the pattern (periodic mode) or inside its
fiducial zone (aperture mode, Sect. 3.2.1).  Every step runs in libscint;
this module only chooses the configurations and collects the numbers.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import torch

from . import scint

PC = 3.0856775814913673e16  # m
R_SUN = 6.957e8  # m (IAU nominal solar radius)


@dataclass
class SweepPoint:
    r_diff_km: float
    r_s_rsun: float
    R_s_km: float  # projected source radius r_s z0 / z1
    realisation: int
    m: float
    m_theory: float
    n_ref: float  # (fiducial size / R_ref)^2, the number of refractive domains


def m_versus_theory(N: int, delta_km: float, lam_m: float, z0_m: float, z1_m: float, r_diffs_km, radii_rsun,
                    n_real: int = 2, seed: int = 1, beta: float = 11.0 / 3.0, mode: str = "periodic",
                    margin_rf: float = 10.0, dtype=torch.float32, device="cuda") -> list[SweepPoint]:
    """Runs the sweep; lengths in km unless named otherwise.  mode
    "periodic": transfer-function propagation, m over the whole pattern
    (no borders on the torus; the disk must be smaller than the grid);
    "aperture": one-FFT propagation with the window and m inside the
    fiducial zone (margin R_ref/2 + R_s)."""
    if mode not in ("periodic", "aperture"):
        raise ValueError("mode must be 'periodic' or 'aperture'")
    delta = delta_km * 1e3
    r_f = math.sqrt(lam_m * z0_m / (2 * math.pi))
    Rs_km = [r * R_SUN * z0_m / z1_m / 1e3 for r in radii_rsun]
    Rs_px = [r / delta_km for r in Rs_km]
    if mode == "periodic" and 2 * max(Rs_px) >= N:
        raise ValueError("a source disk is wider than the periodic grid")
    out: list[SweepPoint] = []
    for r_diff_km in r_diffs_km:
        phi = scint.ps_generate(N, delta, r_diff_km * 1e3, beta, seed, 0, n_real, dtype, device=device)
        if mode == "periodic":
            I = scint.fresnel_propagate(phi, delta, lam_m, z0_m)
        else:
            I = scint.fresnel_aperture(phi, delta, lam_m, z0_m, margin_rf=margin_rf)
        del phi
        Is = scint.source_smear(I, 1.0, Rs_px)  # [n_real, n_r, N, N], radii in pixels
        del I
        r_ref_km = 2 * math.pi * (r_f / 1e3) ** 2 / r_diff_km
        for j, (r_s, R_s) in enumerate(zip(radii_rsun, Rs_km)):
            pats = Is[:, j].contiguous()
            if mode == "periodic":
                ms = scint.ps_modulation_index(pats)
                d_km = N * delta_km
            else:
                pix, margin = scint.aperture_geometry(N, delta, lam_m, z0_m, r_diff_km * 1e3, R_s * 1e3)
                w = N - 2 * margin
                if w < 1:
                    continue
                ms = scint.ps_modulation_index_region(pats, margin, margin, w, w)
                d_km = w * pix / 1e3
            mt = scint.m_theory(r_diff_km, r_f / 1e3, R_s)
            for b, m in enumerate(ms):
                out.append(SweepPoint(r_diff_km, r_s, R_s, b, m, mt, (d_km / r_ref_km) ** 2))
        del Is
    return out

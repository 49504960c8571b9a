"""Pins of the oracle's structure-function check of a screen (Sect. 3.1.1,
Eq. crec): ring-averaged spectrum, Hankel transform with J0, D = 2(xi(0) -
xi(r)), and R_diff^rec from D = 1."""
import math

import numpy as np
import pytest
from scipy import integrate, optimize, special

from tests._golden import paper_values


def test_single_mode_closed_form(oracle):
    # phi = A cos(2 pi (3x + 4y)/N): all power sits at k' = +-(3, 4), |k'| = 5,
    # so S_rec[5] = 2 (A N^2 / 2)^2 / N^2 / count_5 and
    # D(r) = 2 * 2 pi (5/N) S_5 (1/N) (1 - J0(2 pi 5 r / N))
    N, A = 64, 0.7
    y, x = np.mgrid[0:N, 0:N]
    phi = A * np.cos(2 * np.pi * (3 * x + 4 * y) / N)
    S, count = oracle.ring_spectrum(phi)
    k = np.arange(N)
    k = np.where(k < N // 2, k, k - N)
    rad = np.sqrt(k[:, None] ** 2 + k[None, :] ** 2)
    count5 = np.sum(np.floor(rad + 0.5) == 5)  # brute-force ring count
    assert count[5] == count5
    S5 = 2 * (A * N * N / 2) ** 2 / N ** 2 / count5
    assert S[5] == pytest.approx(S5, rel=1e-12)
    assert np.abs(np.delete(S, 5)).max() < 1e-20 * S5 + 1e-24
    for r in (0.5, 3.0, 7.3):
        D = 2 * 2 * np.pi * (5 / N) * S5 / N * (1 - special.j0(2 * np.pi * 5 * r / N))
        assert oracle.structure_from_spectrum(N, S, r) == pytest.approx(D, rel=1e-12)


def test_ring_counts_partition_the_plane(oracle):
    N = 50
    S, count = oracle.ring_spectrum(np.zeros((N, N)))
    k = np.arange(N)
    k = np.where(k < N // 2, k, k - N)
    rad = np.sqrt(k[:, None] ** 2 + k[None, :] ** 2)
    assert count.sum() == np.sum(np.floor(rad + 0.5) <= N // 2)
    assert count[0] == 1 and count[1] == 8  # |k'| = 1 and sqrt(2) both round to 1


def test_theoretical_spectrum_gives_the_papers_540_km(oracle):
    # the paper's check (Sect. 3.1.1): 14000^2 pixels of 28.85 km, R_diff =
    # 500 km input, about 540 km recovered from the sampled spectrum; here the
    # theoretical spectrum sampled on the same rings
    pv = paper_values()
    N, dkm = int(pv["rdiff_rec_pixels"]), pv["rdiff_rec_delta_km"]
    R = pv["rdiff_rec_input_km"] / dkm
    q = np.arange(N // 2 + 1) / N
    S = np.array([oracle.spectrum(qq, R, 11 / 3) if qq > 0 else 0.0 for qq in q])
    r_rec = oracle.rdiff_rec(N, S) * dkm
    assert r_rec == pytest.approx(pv["rdiff_rec_km"], rel=0.01)
    # the continuous integral over the same limits (scipy quadrature) lies
    # within the discretisation of the first rings
    def D(r):
        f = lambda qq: 2 * math.pi * qq * oracle.spectrum(qq, R, 11 / 3) * (1 - special.j0(2 * math.pi * qq * r))
        return 2 * integrate.quad(f, 1.0 / N, 0.5, limit=4000)[0]
    r_cont = optimize.brentq(lambda r: D(r) - 1, 1.0, 100.0) * dkm
    assert r_rec == pytest.approx(r_cont, rel=0.025)
    # and with infinite limits D(R_diff) = 1 exactly (Eq. dphi), so the
    # sampled value exceeds the input: the lost large and small scales
    assert r_rec > pv["rdiff_rec_input_km"] * 1.05


def ring_mean_of_theory(oracle, N, R, beta):
    """The theoretical spectrum averaged over the Fourier pixels of each ring
    (the expectation of the realised ring spectrum)."""
    k = np.arange(N)
    k = np.where(k < N // 2, k, k - N).astype(np.float64)
    rad = np.sqrt(k[:, None] ** 2 + k[None, :] ** 2)
    b = np.floor(rad + 0.5).astype(np.int64)
    A = oracle.spectrum(1.0, R, beta)  # S(q) = A q^-beta
    with np.errstate(divide="ignore"):
        s = np.where(rad > 0, A * (rad / N) ** (-beta), 0.0)
    keep = b <= N // 2
    tot = np.bincount(b[keep], weights=s[keep], minlength=N // 2 + 1)
    cnt = np.bincount(b[keep], minlength=N // 2 + 1)
    return tot / np.maximum(cnt, 1)


def test_screens_recover_their_sampled_spectrum(oracle):
    # oracle screens: D_rec(r) is linear in the ring spectrum, so its mean over
    # realisations must equal D of the ring-averaged theoretical spectrum
    # (within 4 standard errors of the realisation scatter)
    N, R, n = 256, 4.0, 16
    S_th = ring_mean_of_theory(oracle, N, R, 11 / 3)
    spectra = [oracle.ring_spectrum(oracle.screen(N, R, 11 / 3, 3, r))[0] for r in range(n)]
    for r in (0.5 * R, R, 2 * R):
        d = np.array([oracle.structure_from_spectrum(N, S, r) for S in spectra])
        d_th = oracle.structure_from_spectrum(N, S_th, r)
        assert abs(d.mean() - d_th) < 4 * d.std(ddof=1) / np.sqrt(n) + 1e-3 * d_th
    # R_diff^rec of single screens scatters a few percent around that of S_th
    r_th = oracle.rdiff_rec(N, S_th)
    vals = np.array([oracle.rdiff_rec(N, S) for S in spectra])
    assert np.all(np.abs(vals / r_th - 1) < 0.2)

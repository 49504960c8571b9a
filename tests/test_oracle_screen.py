"""Pins of the oracle's phase spectrum and phase screen (Sect. 2 and 3.1).

* f(beta) against the Bessel-integral closed form that makes Eq. spectre and
  Eq. dphi consistent; the continuous structure function D(R_diff) = 1.
* the random spectrum has <|c_k|^2> = S(q_k)/N^2 (Eq. densite with c = F/L^2).
* the realised structure function of the screen equals the exact discrete
  expectation E[D(r)] = 2 sum_k S_k/N^2 (1 - cos 2 pi k_x r / N).
* the paper's printed figure: about 540 km recovered for an input of 500 km on
  a 14000^2 grid of 28.85 km pixels (Sect. 3.1.1).
"""
import numpy as np
import pytest
from scipy import integrate, optimize, special

from _golden import paper_values

BETAS = [3.1, 3.2, 11 / 3, 3.9]


@pytest.mark.parametrize("beta", BETAS)
def test_f_beta_equals_bessel_integral(oracle, beta):
    # D(r) = (r/R)^(beta-2) requires int_0^inf u^(1-beta) (1 - J0(u)) du = f(beta)
    g = lambda u: u ** (1 - beta) * (1 - special.j0(u))
    head, _ = integrate.quad(g, 0, 50, limit=500)
    tail_one = 50 ** (2 - beta) / (beta - 2)
    tail_j0, _ = integrate.quad(lambda u: u ** (1 - beta) * special.j0(u), 50, 5000, limit=5000)
    assert oracle.f_beta(beta) == pytest.approx(head + tail_one - tail_j0, rel=1e-7)


@pytest.mark.parametrize("beta", BETAS)
@pytest.mark.parametrize("r_over_R", [0.5, 1.0, 2.0])
def test_continuous_structure_function(oracle, beta, r_over_R):
    # D(r) = 2 int d^2q S(q) (1 - cos 2 pi q.r) = 2 int 2 pi q S(q) (1 - J0(2 pi q r)) dq
    R = 7.0
    r = r_over_R * R
    integrand = lambda q: 2 * 2 * np.pi * q * oracle.spectrum(q, R, beta) * (1 - special.j0(2 * np.pi * q * r))
    # split at the first zeros region; S decays as q^-beta so the tail is analytic
    qmax = 200.0 / r
    body, _ = integrate.quad(integrand, 0, qmax, limit=2000)
    A = oracle.spectrum(1.0, R, beta)
    tail = 2 * 2 * np.pi * A * qmax ** (2 - beta) / (beta - 2)
    tail_j0, _ = integrate.quad(lambda q: 2 * 2 * np.pi * q * oracle.spectrum(q, R, beta) * special.j0(2 * np.pi * q * r),
                                qmax, 100 * qmax, limit=5000)
    D = body + tail - tail_j0
    assert D == pytest.approx(r_over_R ** (beta - 2), rel=2e-6)


def test_spectrum_is_power_law(oracle):
    R, beta = 5.0, 11 / 3
    for q in (0.01, 0.1, 0.3):
        assert oracle.spectrum(2 * q, R, beta) / oracle.spectrum(q, R, beta) == pytest.approx(2 ** -beta, rel=1e-13)
    # R enters as R^(2-beta)
    assert oracle.spectrum(0.1, 2 * R, beta) / oracle.spectrum(0.1, R, beta) == pytest.approx(2 ** (2 - beta), rel=1e-13)


def _signed(N):
    k = np.arange(N)
    return np.where(k < N // 2, k, k - N)


def test_spectrum_coefficient_variance(oracle):
    N, R, beta, nreal = 32, 3.0, 11 / 3, 64
    acc = np.zeros((N, N))
    for r in range(nreal):
        c = oracle.spectrum_coeffs(N, R, beta, seed=11, r=r)
        assert c[0, 0] == 0
        acc += np.abs(c) ** 2
    k = _signed(N)
    q = np.sqrt(k[None, :] ** 2 + k[:, None] ** 2) / N
    q[0, 0] = 1
    S = np.vectorize(lambda x: oracle.spectrum(x, R, beta))(q)
    ratio = (acc / nreal) * N * N / S
    ratio[0, 0] = np.nan
    # |c|^2 N^2/S is a unit exponential per pixel: mean 1, sd 1/sqrt(count)
    m = np.nanmean(ratio)
    assert abs(m - 1) < 4 / np.sqrt(nreal * (N * N - 1))


def expected_D(oracle, N, R, beta, lags, with_sd=False):
    """Exact discrete expectation of the structure function along x and, if
    asked, the standard deviation of its one-realisation estimate (each
    Fourier mode's power is exponential, so its variance is its mean squared;
    the modes k and -k of the real screen carry the same power)."""
    A = oracle.spectrum(1.0, R, beta)  # S(q) = A q^-beta
    k = _signed(N).astype(np.float64)
    k2 = k[None, :] ** 2 + k[:, None] ** 2
    k2[0, 0] = np.inf
    S = A * (np.sqrt(k2) / N) ** (-beta)
    sigma2 = S / N ** 2
    E, SD = [], []
    for lag in lags:
        w = 2 * (1 - np.cos(2 * np.pi * k[None, :] * lag / N))
        E.append((w * sigma2).sum())
        SD.append(np.sqrt(2 * (w ** 2 * sigma2 ** 2).sum()))
    return (np.array(E), np.array(SD)) if with_sd else np.array(E)


def test_screen_structure_function(oracle):
    N, R, beta, nreal = 64, 4.0, 11 / 3, 48
    lags = np.array([1, 2, 4, 8, 16])
    Dx = np.zeros(len(lags))
    Dy = np.zeros(len(lags))
    for r in range(nreal):
        phi = oracle.screen(N, R, beta, seed=3, r=r)
        assert abs(phi.mean()) < 1e-12 * np.abs(phi).max()
        for i, lag in enumerate(lags):
            Dx[i] += np.mean((np.roll(phi, -lag, axis=1) - phi) ** 2)
            Dy[i] += np.mean((np.roll(phi, -lag, axis=0) - phi) ** 2)
    E, SD = expected_D(oracle, N, R, beta, lags, with_sd=True)
    tol = 5 * SD / np.sqrt(nreal)
    assert np.all(np.abs(Dx / nreal - E) < tol)
    assert np.all(np.abs(Dy / nreal - E) < tol)
    # a screen that dropped the sqrt(2) of phi = sqrt(2) Re(...) would sit at E/2
    assert np.all(tol[:4] < 0.25 * E[:4])


def test_discrete_expectation_approaches_power_law(oracle):
    # Sect. 3.1.1: with a wider frequency range (q_min -> 0, q_max -> inf) the
    # sampled structure function approaches Eq. dphi; D(R_diff) -> 1.
    beta = 11 / 3
    vals = []
    for N, R in ((64, 4.0), (256, 4.0), (1024, 4.0), (4096, 4.0)):
        vals.append(expected_D(oracle, N, R, beta, [R])[0])
    assert all(a < b < 1.0 for a, b in zip(vals, vals[1:]))
    gaps = [1 - v for v in vals]
    assert all(g2 < 0.8 * g1 for g1, g2 in zip(gaps, gaps[1:]))
    assert vals[-1] > 0.85


def test_paper_recovered_rdiff(oracle):
    """Sect. 3.1.1: N ~ 14000, pixel 28.85 km, R_diff = 500 km -> ~540 km."""
    pv = paper_values()
    N = int(pv["rdiff_rec_pixels"])
    delta = pv["rdiff_rec_delta_km"]
    R = pv["rdiff_rec_input_km"] / delta
    beta = pv["beta_kolmogorov"]
    A = oracle.spectrum(1.0, R, beta)
    k = _signed(N).astype(np.float64)
    Sx = np.zeros(N)
    for i0 in range(0, N, 1000):
        kx = k[i0:i0 + 1000]
        k2 = kx[:, None] ** 2 + k[None, :] ** 2
        with np.errstate(divide="ignore"):
            s = A * (np.sqrt(k2) / N) ** (-beta)
        s[~np.isfinite(s)] = 0.0
        Sx[i0:i0 + 1000] = s.sum(axis=1)
    D = lambda lag: 2 * (Sx * (1 - np.cos(2 * np.pi * k * lag / N))).sum() / N ** 2
    r_rec = optimize.brentq(lambda lag: D(lag) - 1.0, 1.0, 60.0)
    assert r_rec * delta == pytest.approx(pv["rdiff_rec_km"], rel=0.02)

"""Pins of the oracle's light-curve sampler (Sect. 3.3) and of the expected
modulation index of Eq. xparam (Sect. 4.1)."""
import numpy as np
import pytest

from tests._golden import paper_values

KPC = 3.0856775814913673e19  # m
R_SUN = 6.957e8  # m (IAU nominal solar radius)


@pytest.mark.parametrize("mode", [0, 1])
def test_axis_aligned_lines_are_rows_and_columns(oracle, mode):
    N = 24
    I = np.random.default_rng(1).exponential(1.0, (N, N))
    lines = [(0.0, 5.0, 1.0, 0.0), (3.0, 0.0, 0.0, 1.0), (7.0, 11.0, -1.0, 0.0), (2.0, 9.0, 0.0, -1.0)]
    n = 2 * N + 3  # wraps around the periodic pattern twice
    c, _ = oracle.light_curves(I, lines, n, mode)
    k = np.arange(n)
    assert np.array_equal(c[0], I[5, k % N])
    assert np.array_equal(c[1], I[k % N, 3])
    assert np.array_equal(c[2], I[11, (7 - k) % N])
    assert np.array_equal(c[3], I[(9 - k) % N, 2])


def test_bilinear_is_exact_on_a_linear_field(oracle):
    N = 40
    y, x = np.mgrid[0:N, 0:N].astype(np.float64)
    I = 2.0 + 0.3 * x - 0.17 * y
    line = (1.3, 2.7, 0.37, 0.21)  # stays inside [0, N - 1) for 80 samples
    c, _ = oracle.light_curves(I, [line], 80, 1)
    k = np.arange(80)
    px, py = line[0] + k * line[2], line[1] + k * line[3]
    assert px.max() < N - 1 and py.max() < N - 1
    assert np.abs(c[0] - (2.0 + 0.3 * px - 0.17 * py)).max() < 1e-12


def test_nearest_pixel_is_within_half_a_pixel(oracle):
    N = 32
    y, x = np.mgrid[0:N, 0:N]
    I = (y * N + x).astype(np.float64)  # each pixel holds its own index
    line = (-3.3, 40.6, 0.731, -0.419)
    n = 300
    c, _ = oracle.light_curves(I, [line], n, 0)
    k = np.arange(n)
    px, py = line[0] + k * line[2], line[1] + k * line[3]
    iy, ix = np.divmod(c[0].astype(np.int64), N)
    dx = (ix - px + N / 2) % N - N / 2  # minimum-image offsets
    dy = (iy - py + N / 2) % N - N / 2
    assert np.all(np.abs(dx) <= 0.5) and np.all(np.abs(dy) <= 0.5)


def test_curve_modulation_index(oracle):
    N = 64
    I = np.random.default_rng(3).gamma(2.0, 0.5, (N, N))
    lines = [(0.5, 1.5, 0.9, 0.1), (10.0, 3.0, 0.2, 1.1)]
    for mode in (0, 1):
        c, m = oracle.light_curves(I, lines, 500, mode)
        for l in range(2):
            assert m[l] == pytest.approx(c[l].std() / c[l].mean(), rel=1e-12)


def test_m_theory_matches_the_papers_numeric_form(oracle):
    # first form of Eq. xparam (oracle) against the second, numeric form, in
    # which the paper rounds the constant to 0.035: the ratio must be the same
    # for every configuration (same exponents) and within 1 % of one
    pv = paper_values()
    ratios = []
    for lam_um, z0_kpc, rdiff_km, rs_rsun, z1_kpc in [(2.162, 0.16, 100.0, 0.5, 1.0), (1.0, 1.0, 1000.0, 1.0, 10.0),
                                                      (0.5, 0.08, 300.0, 0.25, 8.0), (2.2, 10.0, 50.0, 1.5, 62.0)]:
        lam, z0, rdiff, z1 = lam_um * 1e-6, z0_kpc * KPC, rdiff_km * 1e3, z1_kpc * KPC
        r_s = rs_rsun * R_SUN
        rf = np.sqrt(lam * z0 / (2 * np.pi))
        R_s = r_s * z0 / z1  # projected source radius
        m1 = oracle.m_theory(rdiff, rf, R_s)
        m2 = pv["m_theory_coeff"] * lam_um * z0_kpc ** (-1 / 6) * (rdiff_km / 1000) ** (-5 / 6) * \
            ((r_s / z1) / (R_SUN / (10 * KPC))) ** (-7 / 6)
        ratios.append(m1 / m2)
    assert np.ptp(ratios) < 1e-12 * max(ratios)
    assert ratios[0] == pytest.approx(1.0, abs=0.01)

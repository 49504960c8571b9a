"""Pins of the oracle's aperture mode (Sect. 3.2, Eqs. intens and Gxy, with
the screen regularisation of Sect. 3.2.1) and of the fiducial-zone statistics.

Each pin is independent of the oracle's own arithmetic: the direct Fresnel
sum is computed here in numpy, the conjugate-plane identity compares with the
periodic two-FFT propagation, the window is checked through properties that
its definition implies (not by re-typing it), and the flatness figure is the
paper's own (< 1 % for a uniform screen)."""
import numpy as np
import pytest

from tests._golden import paper_values


def direct_aperture_numpy(phi, rho, s, sf):
    """Eq. hxy summed over the screen pixels at every observer point: the
    screen pixel j sits at x1 = j - N/2, observer pixel m at
    x0 = (m - N/2) 2 pi rho^2 / N (pixel units)."""
    N = phi.shape[0]
    pix0 = 2 * np.pi * rho ** 2 / N
    x1 = np.arange(N) - N // 2
    x0 = (np.arange(N) - N // 2) * pix0
    w = np.outer(sf, sf) * np.exp(1j * s * phi)
    # separable kernel: e^{i |x0 - x1|^2 / 2 rho^2} = kx(x0, x1) ky(y0, y1)
    k = np.exp(1j * (x0[:, None] - x1[None, :]) ** 2 / (2 * rho ** 2))  # [observer, screen]
    field = k @ w @ k.T / (2 * np.pi * rho ** 2)  # [y0, x0]
    return np.abs(field) ** 2


@pytest.mark.parametrize("Lm", [9.0, 10.0, 6.0])
def test_sf_window_properties(oracle, Lm):
    N = 64
    sf = oracle.sf_window(N, Lm)
    centres = np.arange(N) + 0.5
    # mirror symmetry about the screen centre
    assert np.abs(sf - sf[::-1]).max() < 1e-15
    # flat (=1) strictly inside the margins, rising from 0 at the border
    inner = (centres > Lm) & (centres < N - Lm)
    assert np.all(sf[inner] == 1.0)
    assert 0.0 < sf[0] < 0.05 and np.all(np.diff(sf[centres < Lm]) > 0)
    # the raised sine is odd about its half point: SF(x) + SF(Lm - x) = 1
    left = np.flatnonzero(centres < Lm)
    for j in left:
        x = centres[j]
        jm = int(round(Lm - x - 0.5))
        if 0 <= jm < N and abs(centres[jm] - (Lm - x)) < 1e-12:
            assert sf[j] + sf[jm] == pytest.approx(1.0, abs=1e-15)
    if Lm == 9.0:  # a pixel centre at Lm/2 = 4.5: the half-height point
        assert sf[4] == pytest.approx(0.5, abs=1e-15)
    # no window
    assert np.all(oracle.sf_window(N, 0.0) == 1.0)


@pytest.mark.parametrize("N,rho,s,margin", [(16, 1.596, 1.0, 0.0), (16, 2.0, 0.8, 1.5), (16, 2.5, 1.2, 3.0),
                                            (12, 1.4, 1.0, 2.0), (20, 1.7, 0.6, 0.0)])
def test_aperture_equals_direct_fresnel_sum(oracle, N, rho, s, margin):
    phi = np.random.default_rng(N + int(10 * rho)).uniform(-3, 3, (N, N))
    sf = oracle.sf_window(N, margin * rho)
    ref = direct_aperture_numpy(phi, rho, s, sf)
    got = oracle.fresnel_aperture(phi, rho, s, margin)
    assert np.abs(got - ref).max() < 1e-12 * max(1.0, ref.max())
    # and the oracle's own O(N^4) form
    assert np.abs(oracle.fresnel_aperture_direct(phi, rho, s, margin) - ref).max() < 1e-12 * max(1.0, ref.max())


@pytest.mark.parametrize("N", [16, 64, 100])
def test_aperture_without_window_is_periodic_form_at_conjugate_planes(oracle, N):
    # N Delta^2 = 2 pi R_F^2 (Sect. 3.4): observer pixel = screen pixel, and
    # the one-FFT aperture form equals the periodic propagation pixel by pixel
    rho = np.sqrt(N / (2 * np.pi))
    phi = oracle.screen(N, 2.0, 11 / 3, seed=3, r=0)
    for s in (1.0, 0.7):
        a = oracle.fresnel_aperture(phi, rho, s, 0.0)
        b = oracle.propagate(phi, rho, s)
        assert np.abs(a - b).max() < 1e-11


@pytest.mark.parametrize("N,f", [(256, 1.0), (256, 1.3), (512, 1.0)])
def test_uniform_screen_is_flat_inside_the_window(oracle, N, f):
    # the paper's check of the regularisation: a point source through a
    # uniform screen gives a uniform pattern to better than 1 %
    pv = paper_values()
    rho = f * np.sqrt(N / (2 * np.pi))
    I = oracle.fresnel_aperture(np.zeros((N, N)), rho, 1.0, 10.0)
    pix0 = 2 * np.pi * rho ** 2 / N
    x0 = (np.arange(N) - N // 2) * pix0
    inner = np.abs(x0) < N / 2 - 12 * rho  # more than L_m + 2 R_F inside the border
    assert inner.sum() > 20
    assert np.abs(I[np.ix_(inner, inner)] - 1).max() < pv["uniform_flatness"]
    outside = np.abs(x0) > N / 2 + 3 * rho  # beyond the screen's shadow
    if outside.any():
        assert I[np.ix_(outside, outside)].max() < 1e-10
    # without the window the diaphragm's fringes reach the same zone's edge
    I0 = oracle.fresnel_aperture(np.zeros((N, N)), rho, 1.0, 0.0)
    if f > 1.0:
        near = np.abs(x0) < N / 2 - 2 * rho
        assert np.abs(I0[np.ix_(near, near)] - 1).max() > pv["uniform_flatness"]


@pytest.mark.parametrize("N,f,margin", [(64, 1.0, 10.0), (64, 1.4, 3.0), (80, 1.2, 0.0)])
def test_aperture_energy_conservation(oracle, N, f, margin):
    # Parseval in physical units: sum(h) * observer pixel area equals the
    # power through the windowed screen, sum(SF_x^2 SF_y^2) * screen pixel area
    rho = f * np.sqrt(N / (2 * np.pi))
    if 2 * margin * rho > N:
        pytest.skip("window wider than the screen")
    phi = oracle.screen(N, 1.5, 11 / 3, seed=9, r=1)
    I = oracle.fresnel_aperture(phi, rho, 1.0, margin)
    pix0 = 2 * np.pi * rho ** 2 / N
    sf = oracle.sf_window(N, margin * rho)
    assert I.sum() * pix0 ** 2 == pytest.approx(np.sum(sf ** 2) ** 2, rel=1e-12)


def test_region_statistics(oracle):
    rng = np.random.default_rng(4)
    I = rng.gamma(2.0, 0.5, (48, 48))
    for (x0, y0, w, h) in [(0, 0, 48, 48), (5, 7, 30, 20), (47, 0, 1, 48), (10, 10, 1, 1)]:
        sub = I[y0:y0 + h, x0:x0 + w]
        m, mean = oracle.modulation_index_region(I, x0, y0, w, h)
        assert mean == pytest.approx(sub.mean(), rel=1e-14)
        assert m == pytest.approx(sub.std() / sub.mean(), rel=1e-12, abs=1e-15)
    m_all, _ = oracle.modulation_index_region(I, 0, 0, 48, 48)
    assert m_all == pytest.approx(oracle.modulation_index(I), rel=1e-14)

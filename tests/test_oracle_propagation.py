"""Pins of the oracle's Fresnel propagation (Sect. 2, Eq. hxy; Sect. 3.2).

* at N = 2 pi rho^2 (the conjugate-plane relation of Sect. 3.4) the periodic
  transfer-function result equals a direct O(N^4) sum of Eq. hxy over the
  finite screen and the paper's one-FFT form (Eqs. intens, Gxy) without the
  smoothing window; both are computed here with numpy, not by the oracle.
* a uniform screen gives I = 1 (Sect. 3.2.1); so does a linear phase ramp;
  <I> = 1 for any screen (Parseval).
* a sinusoidal phase grating has the Jacobi-Anger closed form; at the Talbot
  distances the pattern is uniform.
* weak phase: I - 1 = 2 IDFT(sin(theta_k) phi_k)/N^2 to first order, which
  fixes the sign of the chirp (a phase bump focuses light).
* strong regime point source: m ~ 1 (Sect. 4.1).
"""
import numpy as np
import pytest
from scipy import special

from _golden import paper_values


def _signed(N):
    k = np.arange(N)
    return np.where(k < N // 2, k, k - N)


def direct_fresnel_numpy(phi, rho):
    N = phi.shape[0]
    y, x = np.mgrid[0:N, 0:N]
    u = np.exp(1j * phi).ravel()
    out = np.zeros((N, N))
    for y0 in range(N):
        for x0 in range(N):
            d2 = (x0 - x) ** 2 + (y0 - y) ** 2
            acc = (u * np.exp(1j * d2.ravel() / (2 * rho ** 2))).sum() / (2 * np.pi * rho ** 2)
            out[y0, x0] = abs(acc) ** 2
    return out


@pytest.mark.parametrize("N", [8, 16])
def test_conjugate_plane_equals_direct_fresnel_sum(oracle, N):
    rho = np.sqrt(N / (2 * np.pi))
    rng = np.random.default_rng(N)
    phi = rng.uniform(-3, 3, (N, N))
    I_tf = oracle.propagate(phi, rho)
    I_direct = direct_fresnel_numpy(phi, rho)
    assert np.abs(I_tf - I_direct).max() < 1e-12
    # the oracle's own direct sum and one-FFT variants agree too
    assert np.abs(oracle.fresnel_direct(phi, rho) - I_direct).max() < 1e-12
    # the paper's one-FFT numerics: |FT[G]|^2 / (2 pi rho^2)^2, G = exp(i(phi + r^2/2rho^2))
    y, x = np.mgrid[0:N, 0:N]
    G = np.exp(1j * (phi + (x ** 2 + y ** 2) / (2 * rho ** 2)))
    I_onefft = np.abs(np.fft.fft2(G) / (2 * np.pi * rho ** 2)) ** 2
    assert np.abs(I_tf - I_onefft).max() < 1e-12
    assert np.abs(oracle.fresnel_onefft(phi, rho) - I_onefft).max() < 1e-12


def test_away_from_conjugate_plane_differs_from_aperture_sum(oracle):
    # sanity: the identity above is special to N = 2 pi rho^2
    N = 16
    rho = 0.8 * np.sqrt(N / (2 * np.pi))
    phi = np.random.default_rng(1).uniform(-3, 3, (N, N))
    assert np.abs(oracle.propagate(phi, rho) - direct_fresnel_numpy(phi, rho)).max() > 1e-3


@pytest.mark.parametrize("N,rho", [(64, 5.0), (40, 3.3), (100, 9.0)])
def test_uniform_screen_and_ramp(oracle, N, rho):
    pv = paper_values()
    I = oracle.propagate(np.full((N, N), 1.234), rho)
    assert np.abs(I - 1).max() < 1e-13 < pv["uniform_flatness"]
    m = np.arange(N)
    ramp = 2 * np.pi * (3 * m[None, :] + 5 * m[:, None]) / N
    assert np.abs(oracle.propagate(ramp, rho) - 1).max() < 1e-12


@pytest.mark.parametrize("N,rho,s", [(64, 6.0, 1.0), (80, 11.0, 0.7), (128, 20.0, 1.3)])
def test_parseval_mean_intensity(oracle, N, rho, s):
    phi = oracle.screen(N, 2.0, 11 / 3, seed=5, r=0)
    I = oracle.propagate(phi, rho, s)
    assert I.mean() == pytest.approx(1.0, abs=1e-13)


@pytest.mark.parametrize("a,p,rho", [(1.3, 3, 7.0), (2.5, 1, 11.0), (0.4, 5, 4.0)])
def test_phase_grating_jacobi_anger(oracle, a, p, rho):
    N = 64
    m = np.arange(N)
    phi = np.tile(a * np.cos(2 * np.pi * p * m / N), (N, 1))
    I = oracle.propagate(phi, rho)
    # A(m) = sum_n i^n J_n(a) H1(n p) exp(2 pi i n p m / N), H1(k) = exp(-i 2 pi^2 rho^2 k'^2/N^2)
    A = np.zeros(N, dtype=complex)
    for n in range(-40, 41):
        k = n * p
        kk = ((k + N // 2) % N) - N // 2
        H1 = np.exp(-1j * 2 * np.pi ** 2 * rho ** 2 * kk ** 2 / N ** 2)
        A += (1j ** n) * special.jv(n, a) * H1 * np.exp(2j * np.pi * n * p * m / N)
    assert np.abs(I - np.abs(A)[None, :] ** 2).max() < 1e-12


@pytest.mark.parametrize("talbot", [1, 2])
def test_talbot_self_imaging(oracle, talbot):
    N, p = 64, 4
    # theta(p) = 2 pi^2 rho^2 p^2 / N^2 = pi * talbot
    rho = np.sqrt(talbot * N ** 2 / (2 * np.pi * p ** 2))
    m = np.arange(N)
    phi = np.tile(1.7 * np.cos(2 * np.pi * p * m / N), (N, 1))
    I = oracle.propagate(phi, rho)
    assert np.abs(I - 1).max() < 1e-12
    # and between Talbot planes it is not uniform
    assert np.abs(oracle.propagate(phi, rho * 0.8) - 1).max() > 0.1


def test_weak_phase_linear_response_fixes_chirp_sign(oracle):
    N, rho, eps = 64, 6.0, 1e-5
    y, x = np.mgrid[0:N, 0:N]
    bump = np.exp(-((x - 20) ** 2 + (y - 30) ** 2) / (2 * 3.0 ** 2))
    phi = eps * bump
    I = oracle.propagate(phi, rho)
    k = _signed(N)
    theta = 2 * np.pi ** 2 * rho ** 2 * (k[None, :] ** 2 + k[:, None] ** 2) / N ** 2
    pred = 2 * np.real(np.fft.ifft2(np.sin(theta) * np.fft.fft2(phi)))
    assert np.abs((I - 1) - pred).max() < 20 * eps ** 2
    assert np.abs(pred).max() > 1e3 * eps ** 2
    # a positive phase bump (a converging lens for exp(+i|x|^2/2 R_F^2)) brightens its centre
    assert I[30, 20] > 1


def test_strong_regime_point_source_modulation(oracle):
    pv = paper_values()
    N, R, rho = 256, 4.0, 32.0
    ms = [oracle.modulation_index(oracle.propagate(oracle.screen(N, R, 11 / 3, seed=1, r=r), rho))
          for r in range(3)]
    # m ~ 1 for a point source in the strong regime; the paper's pattern gave 1.18
    assert pv["m_point_strong"] * 0.85 < np.mean(ms) < pv["m_point_tlc"] * 1.15


def test_physical_arguments(oracle):
    N, delta, lam, z = 64, 2.0, 5e-7, 3e5
    rho = np.sqrt(lam * z / (2 * np.pi)) / delta
    assert oracle.fresnel_radius_px(delta, lam, z) == pytest.approx(rho, rel=1e-15)
    phi = oracle.screen(N, 3.0, 11 / 3, seed=2, r=0)
    assert np.array_equal(oracle.fresnel(phi, delta, lam, z), oracle.propagate(phi, rho))


@pytest.mark.parametrize("N,rho,s", [(16, None, 1.0), (64, None, 0.7), (40, 7.0, 0.8), (64, 3.0, 1.3),
                                     (100, 20.0, 1.0)])
def test_separable_screen_factorises(oracle, N, rho, s):
    conjugate = rho is None
    if conjugate:
        rho = np.sqrt(N / (2 * np.pi))
    # phi(x, y) = f(x) + g(y): the 2-D propagation is the outer product of two
    # 1-D propagations (the DFT and H = H1(kx) H1(ky) both factorise)
    rng = np.random.default_rng(N)
    f, g = rng.uniform(-3, 3, N), rng.uniform(-3, 3, N)
    I2 = oracle.propagate(g[:, None] + f[None, :], rho, s)
    af, ag = oracle.propagate_line(f, rho, s), oracle.propagate_line(g, rho, s)
    I1 = np.outer(np.abs(ag) ** 2, np.abs(af) ** 2)
    assert np.abs(I2 - I1).max() < 1e-12 * I2.max()
    # and at the conjugate planes the 1-D line equals the direct 1-D Fresnel sum
    if conjugate:
        m = np.arange(N)
        k = np.exp(1j * np.pi * ((m[:, None] - m[None, :]) ** 2) / N)  # e^{i (x0-x1)^2 / 2 rho^2}
        a_direct = k @ np.exp(1j * s * f) / np.sqrt(N) * np.exp(-1j * np.pi / 4)
        assert np.abs(np.abs(a_direct) ** 2 - np.abs(af) ** 2).max() < 1e-12

"""Pins of the oracle's polychromatic sum (Sect. 3.2.4), extended-source smear
(Sect. 3.2.3, Eq. iprh) and modulation index (Sect. 4)."""
import numpy as np
import pytest


def test_modulation_index_matches_numpy(oracle):
    rng = np.random.default_rng(0)
    I = rng.exponential(1.0, (64, 64)) + 0.1
    assert oracle.modulation_index(I) == pytest.approx(I.std() / I.mean(), rel=1e-13)
    assert oracle.modulation_index(np.full((8, 8), 3.0)) == 0.0


def test_polychromatic_single_wavelength_is_monochromatic(oracle):
    N, delta, z = 64, 1.0, 2 * np.pi * 36.0 / 6e-7
    phi = oracle.screen(N, 3.0, 11 / 3, seed=4, r=0)
    lam = 6e-7
    I1 = oracle.polychromatic(phi, delta, z, lam, [lam])
    assert np.array_equal(I1, oracle.propagate(phi, oracle.fresnel_radius_px(delta, lam, z), 1.0))


def test_polychromatic_is_weighted_sum(oracle):
    N, delta, lam_ref = 48, 1.0, 6.5e-7
    z = 2 * np.pi * 20.0 ** 2 / lam_ref
    phi = oracle.screen(N, 3.0, 11 / 3, seed=4, r=1)
    lams = np.array([4e-7, 6.5e-7, 9e-7])
    w = np.array([1.0, 3.0, 2.0])
    I = oracle.polychromatic(phi, delta, z, lam_ref, lams, w)
    parts = [oracle.propagate(phi, np.sqrt(l * z / (2 * np.pi)) / delta, lam_ref / l) for l in lams]
    expect = sum(wi * p for wi, p in zip(w / w.sum(), parts))
    assert np.abs(I - expect).max() < 1e-13
    # weights are normalised: scaling them changes nothing; <I> = 1
    assert np.abs(oracle.polychromatic(phi, delta, z, lam_ref, lams, 7 * w) - I).max() < 1e-13
    assert I.mean() == pytest.approx(1.0, abs=1e-13)
    # the phase scales as 1/lambda (Eq. phiNl): the part at lambda is the
    # monochromatic pattern of the screen lambda_ref/lambda * phi
    assert np.abs(parts[0] - oracle.propagate(phi * lam_ref / lams[0], np.sqrt(lams[0] * z / (2 * np.pi)))).max() < 1e-12


def test_polychromatic_reduces_modulation(oracle):
    # Sect. 3.2.4: co-adding a passband attenuates the speckle
    N, delta, lam_ref = 128, 1.0, 6.5e-7
    z = 2 * np.pi * 24.0 ** 2 / lam_ref
    phi = oracle.screen(N, 3.0, 11 / 3, seed=9, r=0)
    lams = np.linspace(4e-7, 9e-7, 12)
    m_poly = oracle.modulation_index(oracle.polychromatic(phi, delta, z, lam_ref, lams))
    m_mono = oracle.modulation_index(oracle.polychromatic(phi, delta, z, lam_ref, [lam_ref]))
    assert m_poly < 0.8 * m_mono


@pytest.mark.parametrize("N,Rs", [(16, 2.5), (20, 3.0), (32, 5.2), (40, 0.99)])
def test_smear_equals_direct_convolution(oracle, N, Rs):
    I = np.random.default_rng(N).exponential(1.0, (N, N))
    a = oracle.smear(I, Rs)
    # direct circular convolution with the binary disk, written here with numpy
    k = np.arange(N)
    k = np.where(k < N // 2, k, k - N)
    disk = (k[None, :] ** 2 + k[:, None] ** 2) <= Rs ** 2
    P = disk / disk.sum()
    direct = np.zeros((N, N))
    for dy, dx in zip(*np.nonzero(P)):
        direct += P[dy, dx] * np.roll(np.roll(I, dy, axis=0), dx, axis=1)
    assert np.abs(a - direct).max() < 1e-13 * I.max()
    assert np.abs(oracle.smear_direct(I, Rs) - direct).max() < 1e-13 * I.max()
    assert a.mean() == pytest.approx(I.mean(), rel=1e-13)


def test_smear_small_radius_is_identity(oracle):
    I = np.random.default_rng(3).exponential(1.0, (32, 32))
    assert np.abs(oracle.smear(I, 0.5) - I).max() < 1e-13
    assert oracle.disk_count(32, 0.5) == 1
    assert oracle.disk_count(32, 1.0) == 5


def test_smear_disk_spectrum_is_real(oracle):
    N, Rs = 64, 7.3
    k = np.arange(N)
    k = np.where(k < N // 2, k, k - N)
    disk = ((k[None, :] ** 2 + k[:, None] ** 2) <= Rs ** 2).astype(float)
    D = oracle.dft2(disk, -1)
    assert np.abs(D.imag).max() < 1e-11


def test_modulation_shrinks_with_source_radius(oracle):
    # Sect. 4.1: an extended source always has m < 1 and m decreases as R_s grows
    N, R, rho = 256, 4.0, 32.0
    I = oracle.propagate(oracle.screen(N, R, 11 / 3, seed=1, r=0), rho)
    ms = [oracle.modulation_index(oracle.smear(I, Rs)) for Rs in (0.0, 2.0, 8.0, 16.0, 32.0)]
    assert all(b < a for a, b in zip(ms, ms[1:]))
    assert ms[-1] < 0.5

"""Pins of the oracle's adjoint (vector-Jacobian product) of the propagation:
dot-product test, central finite differences on phi and on log R_diff."""
import numpy as np
import pytest


def test_adjoint_dot_product(oracle):
    N, rho = 40, 5.5
    rng = np.random.default_rng(0)
    x = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    y = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    lhs = np.vdot(y, oracle.propagate_field(x, rho))
    rhs = np.vdot(oracle.propagate_adjoint_field(y, rho), x)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    # the propagation is unitary: the adjoint inverts it
    assert np.abs(oracle.propagate_adjoint_field(oracle.propagate_field(x, rho), rho) - x).max() < 1e-12


def _loss(oracle, phi, rho, s, It):
    return ((oracle.propagate(phi, rho, s) - It) ** 2).sum()


def test_vjp_finite_differences(oracle):
    # FP64 subproblem: 256^2, rho = 6, R_diff = 3, h = 1e-4 central
    N, rho, R, beta, s = 256, 6.0, 3.0, 11 / 3, 1.0
    phi = oracle.screen(N, R, beta, seed=1, r=0)
    It = oracle.propagate(oracle.screen(N, R, beta, seed=1000, r=0), rho, s)
    I = oracle.propagate(phi, rho, s)
    g = oracle.propagate_vjp(phi, rho, s, 2 * (I - It))
    rng = np.random.default_rng(5)
    h = 1e-4
    pix = rng.integers(0, N, size=(16, 2))
    for (py, px) in pix:
        p1 = phi.copy(); p1[py, px] += h
        p0 = phi.copy(); p0[py, px] -= h
        fd = (_loss(oracle, p1, rho, s, It) - _loss(oracle, p0, rho, s, It)) / (2 * h)
        assert fd == pytest.approx(g[py, px], rel=1e-6, abs=1e-7 * np.abs(g).max())


def test_vjp_phase_scale(oracle):
    N, rho, s = 32, 4.0, 0.6
    phi = oracle.screen(N, 2.0, 11 / 3, seed=3, r=0)
    It = np.random.default_rng(2).exponential(1.0, (N, N))
    I = oracle.propagate(phi, rho, s)
    g = oracle.propagate_vjp(phi, rho, s, 2 * (I - It))
    h = 1e-5
    for (py, px) in ((0, 0), (5, 17), (31, 2)):
        p1 = phi.copy(); p1[py, px] += h
        p0 = phi.copy(); p0[py, px] -= h
        fd = (_loss(oracle, p1, rho, s, It) - _loss(oracle, p0, rho, s, It)) / (2 * h)
        assert fd == pytest.approx(g[py, px], rel=1e-6)


def test_log_rdiff_gradient(oracle):
    # phi scales as R_diff^((2-beta)/2) for fixed noise, so
    # dL/dlog R_diff = ((2 - beta)/2) sum phi dL/dphi
    N, rho, R, beta = 256, 6.0, 3.0, 11 / 3
    It = oracle.propagate(oracle.screen(N, R, beta, seed=1000, r=0), rho)
    phi = oracle.screen(N, R, beta, seed=1, r=0)
    g = oracle.propagate_vjp(phi, rho, 1.0, 2 * (oracle.propagate(phi, rho) - It))
    analytic = (2 - beta) / 2 * (phi * g).sum()
    h = 1e-4
    Lp = _loss(oracle, oracle.screen(N, R * np.exp(h), beta, seed=1, r=0), rho, 1.0, It)
    Lm = _loss(oracle, oracle.screen(N, R * np.exp(-h), beta, seed=1, r=0), rho, 1.0, It)
    assert (Lp - Lm) / (2 * h) == pytest.approx(analytic, rel=1e-6)
    # and the screen really scales that way
    ratio = oracle.screen(N, 2 * R, beta, seed=1, r=0) / np.where(phi == 0, 1, phi)
    assert np.nanmax(np.abs(ratio[phi != 0] - 2 ** ((2 - beta) / 2))) < 1e-9

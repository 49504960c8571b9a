"""Pins of the oracle's noise generator and of its own DFT.

Noise: Philox4x32-10 against the published known-answer vectors, the 64-bit
instance of the same round structure against numpy's Philox, and the
distribution of the Box-Muller normals (one complex Gaussian per Fourier
pixel, Sect. 3.1).  DFT: numpy.fft and direct O(n^2) sums.
"""
import numpy as np
import pytest

from _golden import kat_rows


def test_philox4x32_kat(oracle):
    for row in kat_rows("philox4x32_10_kat.txt"):
        ctr, key, want = row[:4], row[4:6], row[6:10]
        got = oracle.philox4x32_10(ctr, key)
        assert [int(x) for x in got] == want


def test_philox4x64_kat(oracle):
    for row in kat_rows("philox4x64_10_kat.txt"):
        ctr, key, want = row[:4], row[4:6], row[6:10]
        got = oracle.philox4x64_10(ctr, key)
        assert [int(x) for x in got] == want


@pytest.mark.parametrize("key,ctr", [((0, 0), (0, 0, 0, 0)), ((123, 456), (5, 7, 9, 11)),
                                      ((2**64 - 1, 2**63 + 5), (2**64 - 3, 1, 0, 2**40))])
def test_philox4x64_matches_numpy(oracle, key, ctr):
    # numpy's Philox increments its 256-bit counter before each block
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(ctr, dtype=np.uint64))
    raw = bg.random_raw(8)
    c = list(ctr)
    blocks = []
    for _ in range(2):
        # add one with carry over the four 64-bit words
        for i in range(4):
            c[i] = (c[i] + 1) % 2**64
            if c[i] != 0:
                break
        blocks.extend(int(x) for x in oracle.philox4x64_10(c, key))
    assert blocks == [int(x) for x in raw]


def test_normals_distribution(oracle):
    N = 128
    g = np.concatenate([oracle.normals(N, seed=7, r=r).ravel() for r in range(4)])
    n = g.size
    for part in (g.real, g.imag):
        assert abs(part.mean()) < 5 / np.sqrt(n)
        assert abs(part.var() - 1) < 5 * np.sqrt(2 / n)
        # fourth moment of a unit normal is 3
        assert abs((part ** 4).mean() - 3) < 5 * np.sqrt(96 / n)
    assert abs(np.mean(g.real * g.imag)) < 5 / np.sqrt(n)
    # |g|^2/2 is a unit exponential: chi-square on 20 equiprobable bins
    from scipy import stats
    e = np.abs(g) ** 2 / 2
    edges = stats.expon.ppf(np.linspace(0, 1, 21))
    counts, _ = np.histogram(e, bins=edges)
    chi2 = ((counts - n / 20) ** 2 / (n / 20)).sum()
    assert chi2 < stats.chi2.ppf(0.9999, 19)


def test_normals_depend_on_all_counter_words(oracle):
    a = oracle.normals(16, seed=1, r=0)
    assert not np.allclose(a, oracle.normals(16, seed=2, r=0))
    assert not np.allclose(a, oracle.normals(16, seed=1, r=1))
    assert not np.allclose(a, oracle.normals(16, seed=1 + 2**32, r=0))
    assert not np.allclose(a, a.T)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 8, 10, 16, 20, 25, 40, 50, 56, 64, 100, 125, 250, 256,
                               1000, 1024, 2000, 4096, 10000])
def test_dft1_matches_numpy(oracle, n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    scale = np.abs(x).sum()
    assert np.abs(oracle.dft1(x, -1) - np.fft.fft(x)).max() <= 1e-14 * scale
    assert np.abs(oracle.dft1(x, +1) - np.fft.ifft(x) * n).max() <= 1e-14 * scale


@pytest.mark.parametrize("n", [2, 5, 6, 10, 12, 40])
def test_dft1_matches_direct_sum(oracle, n):
    rng = np.random.default_rng(100 + n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    j = np.arange(n)
    for sign in (-1, 1):
        direct = np.array([(x * np.exp(sign * 2j * np.pi * j * k / n)).sum() for k in range(n)])
        assert np.abs(oracle.dft1(x, sign) - direct).max() <= 1e-13 * np.abs(x).sum()


@pytest.mark.parametrize("N", [8, 10, 40, 64, 160, 256])
def test_dft2_matches_numpy(oracle, N):
    rng = np.random.default_rng(N)
    a = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    scale = np.abs(a).sum()
    assert np.abs(oracle.dft2(a, -1) - np.fft.fft2(a)).max() <= 1e-14 * scale
    assert np.abs(oracle.dft2(a, +1) - np.fft.ifft2(a) * N * N).max() <= 1e-14 * scale
    back = oracle.dft2(oracle.dft2(a, -1), +1) / (N * N)
    assert np.abs(back - a).max() <= 1e-13 * np.abs(a).max()

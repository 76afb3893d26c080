"""Pins for the transforms the oracle uses (numpy rfftn / irfftn).

The oracle's forward transform must be the unnormalised DFT with kernel exp(-i k.x) over all
axes, halved along the last axis, and its inverse the 1/N transform with exp(+i k.x)
(Eq. (9)).  These tests compare against the O(N^2) definition summed explicitly, and
check Parseval, delta -> flat spectrum, and Hermitian input -> real output.
"""

import itertools

import numpy as np
import pytest


def brute_dft(x, sign=-1):
    """Explicit sum over every grid point for every mode (no FFT)."""
    dims = x.shape
    N = x.size
    out = np.zeros(dims, dtype=np.complex128)
    pts = list(itertools.product(*[range(n) for n in dims]))
    for m in pts:
        acc = 0j
        for xi in pts:
            ph = sum(m[a] * xi[a] / dims[a] for a in range(len(dims)))
            acc += x[xi] * np.exp(sign * 2j * np.pi * ph)
        out[m] = acc
    return out


SHAPES = [(8, 8), (4, 4, 4), (6, 6, 6), (12, 8), (6, 10), (4, 6, 8)]


@pytest.mark.parametrize("dims", SHAPES)
def test_rfftn_is_the_forward_dft(dims):
    rng = np.random.default_rng(1)
    x = rng.standard_normal(dims)
    full = brute_dft(x, -1)
    half = full[..., : dims[-1] // 2 + 1]
    np.testing.assert_allclose(np.fft.rfftn(x), half, rtol=0, atol=1e-11 * np.sqrt(x.size))


@pytest.mark.parametrize("dims", SHAPES)
def test_irfftn_is_the_inverse_dft(dims):
    rng = np.random.default_rng(2)
    x = rng.standard_normal(dims)
    X = brute_dft(x, -1)
    back = brute_dft(X, +1).real / x.size
    np.testing.assert_allclose(back, x, atol=1e-11)
    np.testing.assert_allclose(np.fft.irfftn(X[..., : dims[-1] // 2 + 1], s=dims, axes=tuple(range(len(dims)))), x, atol=1e-12)


def test_parseval_and_delta():
    rng = np.random.default_rng(3)
    for dims in [(16, 12), (8, 6, 10)]:
        x = rng.standard_normal(dims)
        X = np.fft.fftn(x)
        assert np.isclose(np.sum(x ** 2), np.sum(np.abs(X) ** 2) / x.size, rtol=1e-12)
        d = np.zeros(dims)
        d[(0,) * len(dims)] = 1.0
        np.testing.assert_allclose(np.abs(np.fft.rfftn(d)), 1.0, rtol=1e-15)


def test_hermitian_input_gives_real_output():
    # the spectrum of a real field times a lattice-even real weight is Hermitian,
    # so the full complex inverse must come back real
    rng = np.random.default_rng(4)
    dims = (8, 6, 10)
    x = rng.standard_normal(dims)
    d2 = 0.0
    for i, n in enumerate(dims):
        m = np.arange(n)
        sh = [1] * 3
        sh[i] = n
        d2 = d2 + (np.minimum(m, n - m) ** 2).reshape(sh)
    y = np.fft.ifftn(np.fft.fftn(x) * np.exp(-d2 / 7.0))
    assert np.max(np.abs(y.imag)) < 1e-14 * np.max(np.abs(y.real))


def test_shift_theorem_fixes_the_sign():
    # x shifted by one cell along the last axis multiplies mode m by exp(-2 pi i m / n)
    rng = np.random.default_rng(5)
    x = rng.standard_normal((6, 8))
    X = np.fft.rfftn(x)
    Xs = np.fft.rfftn(np.roll(x, 1, axis=1))
    m = np.arange(5)
    np.testing.assert_allclose(Xs, X * np.exp(-2j * np.pi * m / 8), atol=1e-12)

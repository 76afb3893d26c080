"""Pins of the level cut and two-point oracle (CPU).

* S_2 by FFT equals its definition by brute force (2D and 3D, non-square, 3 * 2^k);
* S_2(0) is the volume fraction, the mean over r is its square, S_2(r) = S_2(-r);
* closed forms: a uniform map (S_2 = 1), a checkerboard (1/2 on even-parity shifts, else 0);
* the level threshold inverts the normal CDF (checked with erfc), t(1/2) = 0, t(phi) = -t(1 - phi),
  and a large Gaussian sample cut at t_phi has volume fraction phi within sampling error.
"""

import math

import numpy as np
import pytest

from oracle import twopoint as TP


@pytest.mark.parametrize("shape", [(6, 10), (12, 8), (4, 6, 8), (3, 4, 6)])
def test_s2_fft_equals_brute_force(shape):
    rng = np.random.default_rng(sum(shape))
    g = np.where(rng.random(shape) < 0.37, 1, -1).astype(np.int8)
    np.testing.assert_allclose(TP.s2_map(g), TP.s2_brute(g), rtol=0, atol=1e-12)


def test_s2_identities():
    rng = np.random.default_rng(2)
    g = np.where(rng.random((32, 48)) < 0.3, 1, -1).astype(np.int8)
    S = TP.s2_map(g)
    phi = float(np.mean(g == 1))
    assert S[0, 0] == pytest.approx(phi, abs=1e-12)
    assert float(np.mean(S)) == pytest.approx(phi ** 2, abs=1e-12)
    Sm = np.roll(np.flip(S, axis=(0, 1)), shift=(1, 1), axis=(0, 1))   # S(-r)
    np.testing.assert_allclose(S, Sm, atol=1e-12)


def test_s2_closed_forms():
    np.testing.assert_allclose(TP.s2_map(np.ones((8, 6), np.int8)), 1.0, atol=1e-12)
    y, x = np.meshgrid(np.arange(8), np.arange(6), indexing="ij")
    cb = np.where((x + y) % 2 == 0, 1, -1).astype(np.int8)
    ref = np.where((x + y) % 2 == 0, 0.5, 0.0)
    np.testing.assert_allclose(TP.s2_map(cb), ref, atol=1e-12)


@pytest.mark.parametrize("phi", [0.5, 0.3, 0.05, 0.9, 1e-6])
def test_level_threshold_inverts_the_normal_cdf(phi):
    t = TP.level_threshold(phi, sigma_f=2.0)
    # P(f >= t) for f ~ N(0, 4) is erfc(t / (2 sqrt 2)) / 2
    assert 0.5 * math.erfc(t / (2.0 * math.sqrt(2.0))) == pytest.approx(phi, rel=1e-12, abs=0.0)
    # oddness about 1/2: q = 1 - phi rounds, so compare with the exact tail of the value passed
    q = 1.0 - phi
    assert TP.level_threshold(q, sigma_f=2.0) == pytest.approx(-TP.level_threshold(1.0 - q, sigma_f=2.0),
                                                              rel=1e-13, abs=0.0 if phi != 0.5 else 1e-300)
    if phi == 0.5:
        assert t == 0.0


def test_level_cut_volume_fraction():
    rng = np.random.default_rng(5)
    f = rng.standard_normal(2_000_000)
    for phi in (0.2, 0.5, 0.75):
        g = TP.level_cut(f, TP.level_threshold(phi))
        assert float(np.mean(g == 1)) == pytest.approx(phi, abs=2e-3)

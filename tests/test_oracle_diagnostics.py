"""Pins of the hyperuniformity diagnostics oracle (CPU).

* the window form factor against direct quadrature of exp(i k.y) over a disk / ball;
* single Fourier modes: sigma^2(R) = W^2 / 2 (and W^2 for a Nyquist mode, whose interpolant is
  cos(pi x));
* R = 0 gives the population variance (Parseval);
* a small random field: the variance over all lattice centres of the ball average of its
  trigonometric interpolant, by quadrature, equals the spectral sum;
* the small-k exponent of an exact power law, and of the expected spectrum of a wide-band filter
  (slope -> alpha, Eq. (13) at small K);
* the class table of Eqs. (6)-(7).
"""

import math

import numpy as np
import pytest

from oracle import diagnostics as D
from oracle import FilterParams
from oracle.loss import target_bins


def _disk_average(fun, R, nr=40, nt=96):
    """Mean of fun(y) over |y| < R in 2D (Gauss-Legendre in r with the Jacobian r, trapezoid in
    angle)."""
    g, w = np.polynomial.legendre.leggauss(nr)
    r = 0.5 * R * (g + 1.0)
    wr = 0.5 * R * w * r / (0.5 * R * R)      # / (R^2 / 2): the radial weights sum to 1
    th = 2.0 * math.pi * np.arange(nt) / nt
    y0 = r[:, None] * np.cos(th)[None, :]
    y1 = r[:, None] * np.sin(th)[None, :]
    return float(np.sum(wr[:, None] * fun(y0, y1)) / nt)


def _ball_average(fun, R, nr=24, nc=24, nphi=48):
    """Mean of fun(y) over |y| < R in 3D (Gauss-Legendre in r with the Jacobian r^2 and in
    cos(theta), trapezoid in phi)."""
    g, w = np.polynomial.legendre.leggauss(nr)
    r = 0.5 * R * (g + 1.0)
    wr = 0.5 * R * w * r * r / (R ** 3 / 3.0)
    gc, wc = np.polynomial.legendre.leggauss(nc)
    phi = 2.0 * math.pi * np.arange(nphi) / nphi
    st = np.sqrt(1.0 - gc ** 2)
    y0 = r[:, None, None] * st[None, :, None] * np.cos(phi)[None, None, :]
    y1 = r[:, None, None] * st[None, :, None] * np.sin(phi)[None, None, :]
    y2 = r[:, None, None] * gc[None, :, None] * np.ones_like(phi)[None, None, :]
    wt = wr[:, None, None] * (0.5 * wc)[None, :, None]
    return float(np.sum(wt * fun(y0, y1, y2)) / nphi)


@pytest.mark.parametrize("u", [0.3, 1.0, 2.4048, 3.8317, 7.5, 12.0])
def test_form_factor_2d_matches_disk_quadrature(u):
    k = np.array([0.6, 0.8])                 # unit direction
    got = D.form_factor(np.array([u]), 2)[0]
    ref = _disk_average(lambda a, b: np.cos(u * (k[0] * a + k[1] * b)), 1.0)
    assert abs(got - ref) < 1e-10


@pytest.mark.parametrize("u", [0.3, 1.0, 4.4934, 7.0, 11.0])
def test_form_factor_3d_matches_ball_quadrature(u):
    k = np.array([2.0, -1.0, 2.0]) / 3.0
    got = D.form_factor(np.array([u]), 3)[0]
    ref = _ball_average(lambda a, b, c: np.cos(u * (k[0] * a + k[1] * b + k[2] * c)), 1.0)
    assert abs(got - ref) < 1e-9


def test_single_modes_closed_form():
    n = (24, 32)
    y, x = np.meshgrid(np.arange(n[0]), np.arange(n[1]), indexing="ij")
    m = (3, -5)
    k = 2 * math.pi * np.array([m[0] / n[0], m[1] / n[1]])
    f = np.cos(k[0] * y + k[1] * x + 0.4)
    radii = [0.0, 1.5, 3.0, 7.25]
    got = D.window_variance(f, radii)
    W = D.form_factor(np.linalg.norm(k) * np.array(radii), 2)
    np.testing.assert_allclose(got, 0.5 * W ** 2, rtol=1e-12, atol=1e-15)
    # the Nyquist mode along x: interpolant cos(pi x), variance W(pi R)^2
    g = np.cos(math.pi * x).astype(float)
    got = D.window_variance(g, radii)
    np.testing.assert_allclose(got, D.form_factor(math.pi * np.array(radii), 2) ** 2, rtol=1e-12, atol=1e-15)


def test_zero_radius_is_the_variance():
    rng = np.random.default_rng(1)
    for shape in [(16, 12), (6, 8, 10)]:
        x = rng.standard_normal(shape) + 3.0
        assert D.window_variance(x, [0.0])[0] == pytest.approx(np.var(x), rel=1e-12)


def _interp_window_variance_2d(x, R):
    """Brute force: ball average of the real trigonometric interpolant at every lattice centre."""
    n = x.shape
    X = np.fft.fftn(x) / x.size
    m0 = np.where(np.arange(n[0]) < n[0] // 2, np.arange(n[0]), np.arange(n[0]) - n[0])
    m1 = np.where(np.arange(n[1]) < n[1] // 2, np.arange(n[1]), np.arange(n[1]) - n[1])
    vals = []
    for c0 in range(n[0]):
        for c1 in range(n[1]):
            def fun(a, b):
                ph = (2 * math.pi * m0[:, None, None, None] * (c0 + a)[None, None] / n[0]
                      + 2 * math.pi * m1[None, :, None, None] * (c1 + b)[None, None] / n[1])
                return np.real(np.sum(X[:, :, None, None] * np.exp(1j * ph), axis=(0, 1)))
            vals.append(_disk_average(fun, R, nr=16, nt=40))
    return float(np.var(np.array(vals)))


def test_random_field_matches_interpolant_brute_force_2d():
    rng = np.random.default_rng(7)
    x = rng.standard_normal((6, 8))
    for R in (0.7, 1.9):
        assert D.window_variance(x, [R])[0] == pytest.approx(_interp_window_variance_2d(x, R), rel=1e-7)


def test_random_field_matches_interpolant_brute_force_3d():
    rng = np.random.default_rng(8)
    x = rng.standard_normal((4, 4, 6))
    n = x.shape
    X = np.fft.fftn(x) / x.size
    ms = [np.where(np.arange(k) < k // 2, np.arange(k), np.arange(k) - k) for k in n]
    R = 1.3
    vals = []
    for c in np.ndindex(*n):
        def fun(a, b, d):
            tot = np.zeros_like(a)
            for i0, j0 in enumerate(ms[0]):
                for i1, j1 in enumerate(ms[1]):
                    for i2, j2 in enumerate(ms[2]):
                        ph = 2 * math.pi * (j0 * (c[0] + a) / n[0] + j1 * (c[1] + b) / n[1] + j2 * (c[2] + d) / n[2])
                        tot += np.real(X[i0, i1, i2] * np.exp(1j * ph))
            return tot
        vals.append(_ball_average(fun, R, nr=10, nc=10, nphi=20))
    assert D.window_variance(x, [R])[0] == pytest.approx(float(np.var(vals)), rel=1e-6)


def test_small_k_exponent_of_a_power_law():
    nr, beta = 64, 1.7
    r = np.arange(nr)
    cnt = np.full(nr + 1, 10.0)
    s = np.zeros(nr + 1)
    s[:nr] = cnt[:nr] * (((r + 0.5) / nr) ** beta)
    assert D.small_k_exponent(s, cnt, nr, 8) == pytest.approx(beta, rel=1e-12)


def test_small_k_exponent_of_a_wide_band_filter_is_alpha():
    # H^2 = K^alpha exp(-(K - k0)^2 / w^2): with k0 = 0 and a wide band the small-K slope is alpha.
    # Bins 4 lattice units wide: the bin mean of k^alpha exceeds the centre value by a relative
    # amount ~ alpha^2 (w/c)^2 / 24 that falls as 1/r^2, which flattens the fitted slope by under 3 %
    # here (measured: 1.98 for alpha 2, 3.92 for alpha 4).
    for alpha in (2.0, 4.0):
        filt = FilterParams(p=2, semi=(1, 1, 1), alpha=alpha, k0=0.0, width=5.0)
        T, c = target_bins((512, 512), filt, 64)
        s = T * c
        got = D.small_k_exponent(np.append(s, 0.0), np.append(c, 0), 64, 12)
        assert got == pytest.approx(alpha, rel=0.03)


def test_class_table():
    assert D.CLASSES[D.hyperuniformity_class(2.0, 2)] == "hyperuniform class I"
    assert D.CLASSES[D.hyperuniformity_class(1.0, 3)] == "hyperuniform class II"
    assert D.CLASSES[D.hyperuniformity_class(0.5, 2)] == "hyperuniform class III"
    assert D.CLASSES[D.hyperuniformity_class(0.0, 2)] == "nonhyperuniform (standard)"
    assert D.CLASSES[D.hyperuniformity_class(-1.0, 2)] == "antihyperuniform"
    assert D.CLASSES[D.hyperuniformity_class(-2.5, 2)] == "outside the classified range"


def test_alpha_zero_spectrum_is_flat_at_small_k():
    # alpha = 0 (standard nonhyperuniform, Eq. (7)): chi(k -> 0) > 0, small-k slope 0
    filt = FilterParams(p=2, semi=(1, 1, 1), alpha=0.0, k0=0.0, width=2.0)
    T, c = target_bins((512, 512), filt, 64)
    a = D.small_k_exponent(np.append(T * c, 0.0), np.append(c, 0), 64, 12)
    assert abs(a) < 0.02
    assert D.CLASSES[D.hyperuniformity_class(a, 2, tol=0.02)] == "nonhyperuniform (standard)"


def test_negative_alpha_spectrum_slope_is_alpha():
    # -d < alpha < 0 (antihyperuniform, Eq. (7)): chi ~ |k|^alpha diverges at small k
    filt = FilterParams(p=2, semi=(1, 1, 1), alpha=-1.0, k0=0.0, width=2.0)
    T, c = target_bins((512, 512), filt, 64)
    a = D.small_k_exponent(np.append(T * c, 0.0), np.append(c, 0), 64, 12)
    assert a == pytest.approx(-1.0, rel=0.03)
    assert D.CLASSES[D.hyperuniformity_class(a, 2)] == "antihyperuniform"

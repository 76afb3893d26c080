"""Pins for the oracle's spectral density and amplitude (Eqs. (8), (12)-(14)).

Each test checks a property fixed by the paper or by mathematics, not the formula retyped:
* the peak of chi is 1 (C normalises max chi = 1, the sentence after Eq. (13)), found by a
  dense numerical search rather than the closed form;
* chi(0) = 0 and the small-k log-log slope is alpha (Eq. (4), Eq. (14));
* Eq. (12) reduces to the Euclidean norm at p = 2, a = b, to the L1 norm at p = 1 and to the
  max norm as p -> infinity (the sentence after Eq. (12));
* the amplitude is even, rotating the mask by 90 degrees swaps a and b, and with k0 = 0 the
  band reduces to Eq. (13)'s exp(alpha ln K - K^2 / (2 sigma^2)) up to the constant C;
* a tabulated radial form sampled from a smooth closed form reproduces it within the linear
  interpolation bound, a constant profile gives a flat amplitude, and K past the table takes
  the last sample.
"""

import numpy as np
import pytest

import oracle as O
from oracle.spectral import superellipse_K


def F(**kw):
    base = dict(p=2.0, semi=(1.0, 1.0, 1.0), rot=0.0, alpha=2.0, k0=0.2, width=0.05)
    base.update(kw)
    return O.FilterParams(**base)


@pytest.mark.parametrize("kw", [dict(), dict(alpha=4, k0=0.0, width=0.06217), dict(alpha=20, k0=0.0),
                                dict(alpha=0.5, k0=0.3, width=0.02), dict(alpha=100, k0=0.0, width=0.06)])
def test_peak_is_one(kw):
    f = F(**kw)
    K = np.linspace(1e-6, 3.0, 2_000_001)
    lc = O.ln_chi_rel(K, f)
    assert abs(np.max(lc)) < 1e-9
    assert np.all(lc <= 1e-12)


def test_chi_zero_at_origin_and_slope_alpha():
    for alpha in (0.5, 2.0, 4.0, 6.0):
        f = F(alpha=alpha, k0=0.2, width=0.05)
        assert np.exp(O.ln_chi_rel(np.array([0.0]), f))[0] == 0.0
        K1, K2 = 1e-9, 2e-9
        slope = (O.ln_chi_rel(np.array([K2]), f) - O.ln_chi_rel(np.array([K1]), f)) / np.log(K2 / K1)
        assert abs(slope[0] - alpha) < 1e-5


def _grid(n=40):
    k = np.linspace(-1, 1, n)
    return [k.reshape(-1, 1), k.reshape(1, -1)]          # (ky, kx) axis order


def test_norm_special_cases():
    ky, kx = _grid()
    K2, _, _ = superellipse_K([ky, kx], F(p=2.0))
    np.testing.assert_allclose(K2, np.hypot(kx, ky), rtol=1e-14, atol=1e-15)
    K1, _, _ = superellipse_K([ky, kx], F(p=1.0))
    np.testing.assert_allclose(K1, np.abs(kx) + np.abs(ky), rtol=1e-14, atol=1e-15)
    Kinf, _, _ = superellipse_K([ky, kx], F(p=400.0))
    m = np.maximum(np.abs(kx), np.abs(ky))
    assert np.all(np.abs(Kinf - m) <= 0.01 * m + 1e-15)
    # anisotropy: a = 2 halves the x contribution
    Ka, _, _ = superellipse_K([ky, kx], F(p=2.0, semi=(2.0, 1.0, 1.0)))
    np.testing.assert_allclose(Ka, np.hypot(kx / 2, ky), rtol=1e-14, atol=1e-15)
    # 3D: a third term (|kz|/c)^p
    kz = np.linspace(-1, 1, 7).reshape(-1, 1, 1)
    K3, _, _ = superellipse_K([kz, ky[None], kx[None]], F(p=2.0, semi=(1.0, 1.0, 3.0)))
    np.testing.assert_allclose(K3, np.sqrt(kx[None] ** 2 + ky[None] ** 2 + (kz / 3) ** 2), rtol=1e-14)


def test_amplitude_even_and_rotation_swaps_axes():
    f = F(p=3.0, semi=(2.0, 1.0, 1.0), rot=0.37)
    ky, kx = _grid(33)
    Kp, _, _ = superellipse_K([ky, kx], f)
    Km, _, _ = superellipse_K([-ky, -kx], f)
    np.testing.assert_allclose(Kp, Km, rtol=1e-14)
    g1 = F(p=3.0, semi=(2.0, 1.0, 1.0), rot=np.pi / 2)
    g2 = F(p=3.0, semi=(1.0, 2.0, 1.0), rot=0.0)
    K1, _, _ = superellipse_K([ky, kx], g1)
    K2, _, _ = superellipse_K([ky, kx], g2)
    np.testing.assert_allclose(K1, K2, rtol=1e-12)


def test_k0_zero_reduces_to_eq13():
    f = F(p=1.0, alpha=20.0, k0=0.0, width=0.06)
    K = np.linspace(1e-3, 1.5, 5001)
    raw = np.exp(f.alpha * np.log(K) - K ** 2 / (2 * f.width ** 2))
    chi = np.exp(O.ln_chi_rel(K, f))
    ratio = chi / raw
    np.testing.assert_allclose(ratio, ratio[0], rtol=1e-9)


def test_hsym_only_differs_on_rotated_nyquist_planes():
    dims = (12, 16)
    f0 = F(p=3.0, semi=(2.0, 1.0, 1.0), rot=0.0, k0=0.6, width=0.3)
    np.testing.assert_array_equal(O.amplitude_sym(dims, f0), O.amplitude_half(dims, f0))
    f1 = f0.replace(rot=0.4)
    Hs, H = O.amplitude_sym(dims, f1), O.amplitude_half(dims, f1)
    diff = Hs != H
    diff[6, :] = False          # m_y = n_y / 2
    diff[:, 8] = False          # m_x = n_x / 2
    assert not diff.any()
    assert (Hs[6, 1:8] != H[6, 1:8]).any()


def test_degenerate_filter_raises():
    # a band far narrower than the lattice step, centred between lattice shells
    # (|kappa| = 0.5303 and 0.5590 on a 16^2 grid): every mode has ln chi < -80
    f = F(p=2.0, alpha=2.0, k0=0.545, width=1e-4)
    with pytest.raises(O.DegenerateFilter):
        O.amplitude_half((16, 16), f)
    O.amplitude_half((16, 16), f.replace(width=0.02))


# ---- mask variants: alpha = 0 (standard nonhyperuniform) and the offset regularisation --------
FilterParams, DegenerateFilter, amplitude_half = O.FilterParams, O.DegenerateFilter, O.amplitude_half


def test_alpha_zero_is_the_gaussian_band():
    from oracle.spectral import superellipse_K, wavenumbers_half
    for k0 in (0.0, 0.25):
        filt = FilterParams(p=3, semi=(2, 1, 1), rot=0.0, alpha=0.0, k0=k0, width=0.1)
        H = amplitude_half((32, 48), filt)
        K, _, _ = superellipse_K(wavenumbers_half((32, 48)), filt)
        off_dc = K > 0
        ref = np.exp(-(K - k0) ** 2 / (4 * 0.1 ** 2))        # sqrt of exp(-(K - k0)^2 / (2 w^2)), peak 1
        np.testing.assert_allclose(H[off_dc], ref[off_dc], rtol=1e-13)
        assert H.flat[0] == 0.0 and np.all(np.isfinite(H))


def test_offset_adds_to_chi():
    from oracle.spectral import superellipse_K, wavenumbers_half, ln_chi_rel
    base = FilterParams(p=4, semi=(1, 2, 1), rot=0.3, alpha=2.0, k0=0.2, width=0.05)
    eps = 1e-3
    H0 = amplitude_half((64, 64), base)
    H1 = amplitude_half((64, 64), base.replace(offset=eps))
    K, _, _ = superellipse_K(wavenumbers_half((64, 64)), base)
    off_dc = K > 0
    np.testing.assert_allclose(H1[off_dc] ** 2, H0[off_dc] ** 2 + eps, rtol=1e-13)
    assert H1.flat[0] == 0.0
    # a band far off the lattice is degenerate without the offset and not with it
    far = FilterParams(p=2, alpha=2.0, k0=5.0, width=0.01)
    with pytest.raises(DegenerateFilter):
        amplitude_half((16, 16), far)
    H = amplitude_half((16, 16), far.replace(offset=1e-6))
    np.testing.assert_allclose(H.ravel()[1:] ** 2, 1e-6, rtol=1e-9)


def test_negative_alpha_normalisation_bounds_chi_on_the_lattice():
    from oracle.spectral import superellipse_K, wavenumbers_half, ln_chi_rel
    for filt in (FilterParams(p=3, semi=(2, 1, 1), rot=0.4, alpha=-1.0, k0=0.0, width=0.3),
                 FilterParams(p=2, semi=(1, 1, 1), rot=0.0, alpha=-0.5, k0=0.5, width=0.01),   # band far above k_low
                 FilterParams(p=6, semi=(1, 3, 1), rot=1.0, alpha=-1.5, k0=0.2, width=0.05)):
        ks = wavenumbers_half((64, 96))
        K, _, _ = superellipse_K(ks, filt)
        lc = ln_chi_rel(K[K > 0], filt, ks)
        assert np.max(lc) <= 1e-12                       # chi_rel <= 1 on the lattice
        assert np.max(lc) > -20.0                        # and the bound is not far above the maximum
        H = amplitude_half((64, 96), filt)
        assert H.flat[0] == 0.0 and np.all(np.isfinite(H))


# ---------------------------------------------------------------------------------------------
# tabulated radial form: ln chi at K = i dK, linearly interpolated, held at the last sample
# ---------------------------------------------------------------------------------------------
def test_tabulated_form_reproduces_a_smooth_closed_form():
    # samples of the alpha = 0 Gaussian band (smooth in K): the interpolated amplitude matches the
    # closed form within the linear-interpolation bound |ln chi''| dK^2 / 8 = dK^2 / (8 w^2)
    from oracle.spectral import superellipse_K, wavenumbers_half
    band = FilterParams(p=3, semi=(2, 1, 1), rot=0.4, alpha=0.0, k0=0.2, width=0.05)
    dk = 2e-4
    Kg = dk * np.arange(int(3.0 / dk) + 1)
    prof = tuple(-(Kg - band.k0) ** 2 / (2 * band.width ** 2))
    tab = band.replace(prof=prof, prof_dk=dk)
    dims = (48, 64)
    K, _, _ = superellipse_K(wavenumbers_half(dims), band)
    assert K.max() < Kg[-1]
    H0, H1 = amplitude_half(dims, band), amplitude_half(dims, tab)
    bound = dk ** 2 / (8 * band.width ** 2)          # in ln chi, i.e. 2x in ln H
    np.testing.assert_allclose(H1, H0, rtol=bound, atol=0.0)
    assert H1.flat[0] == 0.0


def test_tabulated_form_constant_and_held_last_sample():
    from oracle.spectral import superellipse_K, wavenumbers_half
    # a constant profile: every mode but the DC gets amplitude exp(c / 2)
    tab = FilterParams(p=2, prof=(-1.0, -1.0), prof_dk=10.0)
    H = amplitude_half((16, 16), tab)
    np.testing.assert_allclose(H.ravel()[1:], np.exp(-0.5), rtol=1e-15)
    assert H.flat[0] == 0.0
    # a short ramp: modes past its end take its last sample, modes inside the linear value
    dims = (32, 32)
    tab = FilterParams(p=2, prof=(0.0, -2.0, -4.0), prof_dk=0.25)
    K, _, _ = superellipse_K(wavenumbers_half(dims), tab)
    H = amplitude_half(dims, tab)
    inside, past = (K > 0) & (K <= 0.5), K > 0.5
    assert np.any(inside) and np.any(past)
    np.testing.assert_allclose(np.log(H[inside]) * 2, -8.0 * K[inside], rtol=1e-12)
    np.testing.assert_allclose(H[past], np.exp(-2.0), rtol=1e-15)

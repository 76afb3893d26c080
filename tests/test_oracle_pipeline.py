"""Pins for the oracle's field pipeline (Eqs. (8), (9), (15) and the sign map).

* the half-spectrum route with H_sym equals the plain definition Re(ifftn(H fftn(w))) on the
  full canonical lattice (Eqs. (8)-(9)), with rotation so that the Nyquist planes matter;
* the normalised field has mean 0 and population variance sigma_f^2 (Eq. (15));
* the result does not depend on the constant C of Eq. (13) nor on the FFT scale;
* the raw field has zero mean because chi(0) = 0 (the sum rule, Eq. (5));
* the threshold is a sign map with sgn(0) = +1.
"""

import numpy as np
import pytest

import oracle as O

CASES = [
    ((16, 16), dict(p=4.0, semi=(3.0, 1.0, 1.0), rot=np.pi / 6, alpha=4, k0=0.2, width=0.04)),
    ((12, 20), dict(p=1.5, semi=(1.0, 2.0, 1.0), rot=1.1, alpha=2, k0=0.3, width=0.1)),
    ((8, 6, 10), dict(p=6.0, semi=(1.0, 2.0, 3.0), rot=0.4, alpha=2, k0=0.15, width=0.2)),
    ((6, 12, 8), dict(p=2.0, semi=(1.0, 1.0, 1.0), rot=0.0, alpha=6, k0=0.25, width=0.15)),
]


@pytest.mark.parametrize("dims,kw", CASES)
def test_half_spectrum_route_equals_plain_complex_route(dims, kw):
    f = O.FilterParams(**kw)
    out = O.gen_field(dims, f, seed=5)
    Hfull = O.amplitude_full(dims, f)
    plain = np.real(np.fft.ifftn(Hfull * np.fft.fftn(out["w"])))
    np.testing.assert_allclose(out["f_raw"], plain, atol=1e-13 * np.abs(plain).max())
    # and the plain complex route's imaginary part only comes from the unsymmetrised Nyquist planes
    if kw["rot"] == 0.0:
        assert np.max(np.abs(np.fft.ifftn(Hfull * np.fft.fftn(out["w"])).imag)) < 1e-13 * np.abs(plain).max()


@pytest.mark.parametrize("sigma_f", [1.0, 2.5])
def test_normalised_moments(sigma_f):
    f = O.FilterParams(p=2.0, semi=(1, 1, 1), alpha=2, k0=0.25, width=0.05, sigma_f=sigma_f)
    out = O.gen_field((64, 48), f, seed=0)
    assert abs(out["f"].mean()) < 1e-14 * sigma_f
    assert abs(np.mean(out["f"] ** 2) - sigma_f ** 2) < 1e-12 * sigma_f ** 2
    # sum rule: F(0) = 0 so the raw field's mean vanishes up to rounding
    assert abs(out["mu"]) < 1e-14 * np.sqrt(out["var"])


def test_invariant_to_C_and_fft_scale():
    dims = (16, 24)
    f = O.FilterParams(p=3.0, semi=(2, 1, 1), rot=0.3, alpha=4, k0=0.3, width=0.1)
    out = O.gen_field(dims, f, seed=3)
    F2 = 37.5 * out["F"]                       # any constant C, any forward scale
    g = np.fft.irfftn(F2, s=dims, axes=(0, 1)) * 1e-3     # any inverse scale
    g = (g - g.mean()) / g.std()
    np.testing.assert_allclose(g, out["f"], atol=1e-12)


def test_threshold_sign_map():
    f = np.array([-1.0, -0.0, 0.0, 1e-30, -1e-30, 2.0, 5e-6, -5e-6])
    t, n_pos, n_near = O.threshold(f)
    np.testing.assert_array_equal(t, [-1, 1, 1, 1, -1, 1, 1, -1])
    assert t.dtype == np.int8 and n_pos == 5 and n_near == 6


def test_pipeline_matches_paper_preset_scale():
    # the paper's 2D setting, scaled to a small grid: sigma = 2.0, L = 100 over 1024 points
    from paper_2509_08675_amd.workloads import paper_preset
    fp = paper_preset(1024, 100.0, sigma=2.0, alpha=20.0, p=1.0)
    assert abs(fp["width"] - 2.0 * (100 / 1024) / np.pi) < 1e-15
    out = O.pipeline((128, 128), O.FilterParams(**fp), seed=1, nr=32)
    assert out["t"].shape == (128, 128)
    # +-1 spectrum: Parseval, every mode counted once with its multiplicity
    assert abs(out["pm1_sum"].sum() - 128 * 128) < 1e-8
    assert int(out["pm1_cnt"].sum()) == 128 * 128

"""Pins for the oracle's binned spectra.

* Parseval: the binned sums over every slot (with the excluded corner slot) equal sum g^2, and
  the counts add up to N (every lattice mode counted once through the multiplicities);
* the half-spectrum binning with multiplicities equals a brute-force pass over the full lattice,
  each mode binned by floor(R |kappa|) and by its folded angle from atan2;
* the fused continuous spectrum (from F, via Parseval) equals the plain spectrum of f.
"""

import math

import numpy as np
import pytest

import oracle as O
from oracle.spectrum import bin_table


def brute_bins(g, nr, na):
    """Full-lattice loop: each mode m maps to its half-spectrum representative (m_x <= n_x/2,
    else the conjugate partner -m), is binned by floor(R |kappa|) and, in 2D, by the angle of
    the representative folded into [0, pi)."""
    dims = g.shape
    G = np.fft.fftn(g)
    P = np.abs(G) ** 2 / g.size
    ssum = np.zeros(nr * na + 1)
    cnt = np.zeros(nr * na + 1, dtype=np.int64)
    for m in np.ndindex(*dims):
        rep = list(m)
        if rep[-1] > dims[-1] // 2:
            rep = [(-v) % n for v, n in zip(rep, dims)]
        kap = []
        for i, (v, n) in enumerate(zip(rep, dims)):
            if i == len(dims) - 1:
                kap.append(2.0 * v / n)
            else:
                kap.append(2.0 * (v if v < n // 2 else v - n) / n)
        kk = math.sqrt(sum(k * k for k in kap))
        r = int(math.floor(nr * kk + 1e-12))
        if r >= nr:
            b = nr * na
        else:
            a = 0
            if na > 1 and kk > 0:
                ang = math.atan2(kap[0], kap[1])
                if ang < 0:
                    ang += math.pi
                a = min(int(math.floor(ang / (math.pi / na) + 1e-12)), na - 1)
            b = r * na + a
        ssum[b] += P[m]
        cnt[b] += 1
    return ssum, cnt


@pytest.mark.parametrize("dims,nr,na", [((16, 16), 8, 6), ((12, 20), 10, 4), ((16, 12), 16, 36),
                                        ((6, 8, 10), 8, 1), ((8, 8, 8), 12, 1)])
def test_binning_matches_full_lattice_brute_force(dims, nr, na):
    rng = np.random.default_rng(7)
    g = rng.standard_normal(dims)
    s_half, c_half = O.power_spectrum(g, nr, na)
    s_b, c_b = brute_bins(g, nr, na)
    np.testing.assert_array_equal(c_half.astype(np.int64), c_b)
    np.testing.assert_allclose(s_half, s_b, rtol=1e-12, atol=1e-12)


def test_parseval_totals_pm1():
    rng = np.random.default_rng(8)
    for dims, nr, na in [((32, 48), 16, 36), ((16, 16, 24), 32, 1)]:
        t = np.where(rng.standard_normal(dims) >= 0, 1.0, -1.0)
        s, c = O.power_spectrum(t, nr, na)
        N = t.size
        assert abs(s.sum() - N) < 1e-9 * N
        assert int(c.sum()) == N


def test_bin_edges_go_up_and_dc_is_bin_zero():
    # on a 16^2 grid with R = 8, |kappa| = 2|m|/16 = |m|/8: m = (0, 4) sits exactly on the edge r = 4
    idx, w = bin_table((16, 16), 8, 1)
    assert idx[0, 4] == 4 and idx[4, 0] == 4 and idx[0, 3] == 3
    assert idx[0, 0] == 0
    # (3,4): |kappa| = 5/8 exactly -> r = 5 ; corner modes |kappa| >= 1 are excluded
    assert idx[3, 4] == 5 and idx[8, 8] == 8 and idx[0, 8] == 8
    # angular: exactly 45 degrees goes to the upper bin
    idxa, _ = bin_table((16, 16), 8, 4)
    assert idxa[2, 2] % 4 == 1 and idxa[0, 2] % 4 == 0 and idxa[2, 0] % 4 == 2
    assert idxa[16 - 2, 2] % 4 == 3                                   # (kx, ky) = (+, -) folds to 135 degrees


def test_fused_continuous_spectrum_equals_plain():
    for dims, nr, na, kw in [((32, 32), 16, 36, dict(p=4.0, semi=(3, 1, 1), rot=0.52, alpha=4, k0=0.2, width=0.04)),
                             ((16, 12, 20), 24, 1, dict(p=6.0, semi=(1, 2, 3), alpha=2, k0=0.15, width=0.1))]:
        f = O.FilterParams(**kw)
        out = O.gen_field(dims, f, seed=2)
        s_plain, c_plain = O.power_spectrum(out["f"], nr, na)
        s_fused, c_fused = O.continuous_spectrum_fused(out["F"], dims, nr, na, f.sigma_f)
        np.testing.assert_array_equal(c_plain, c_fused)
        np.testing.assert_allclose(s_fused, s_plain, rtol=1e-9, atol=1e-12 * s_plain.max())
        assert s_fused[0] < 1e-20 or c_fused[0] > 1

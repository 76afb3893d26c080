"""Statistical pins: the ensemble spectrum converges to H_sym^2 (Eqs. (8), (10)-(11)).

Over 1000 seeds on small grids, the mean of |F(k)|^2 / N for the raw (pre-normalisation)
filtered spectrum must approach H_sym(k)^2 mode by mode, within 5 standard errors
(relative standard error 1/sqrt(1000) for complex modes, sqrt(2/1000) for self-conjugate
ones), and a global chi-square over the modes must be consistent with that spread.
The autocovariance of the raw field must match the inverse transform of H_sym^2
(the Wiener-Khinchin pair of Eqs. (10)-(11), on the lattice).
"""

import numpy as np
import pytest
from scipy import stats

import oracle as O

NSEED = 1000


@pytest.mark.parametrize("dims,kw", [
    ((8, 8), dict(p=2.0, semi=(1, 1, 1), rot=0.3, alpha=2, k0=0.4, width=0.3)),
    ((8, 12), dict(p=4.0, semi=(3, 1, 1), rot=0.5, alpha=4, k0=0.3, width=0.3)),
    ((4, 6, 8), dict(p=6.0, semi=(1, 2, 3), rot=0.0, alpha=2, k0=0.3, width=0.4)),
])
def test_ensemble_spectrum_converges_to_H2(dims, kw):
    f = O.FilterParams(**kw)
    N = int(np.prod(dims))
    Hs = O.amplitude_sym(dims, f)
    acc = np.zeros(Hs.shape)
    acov = np.zeros(dims)
    for s in range(NSEED):
        out = O.gen_field(dims, f, s)
        acc += np.abs(out["F"]) ** 2 / N
        fr = out["f_raw"]
        acov += np.real(np.fft.ifftn(np.abs(np.fft.fftn(fr)) ** 2)) / N
    mean = acc / NSEED
    H2 = Hs ** 2
    # self-conjugate modes: every index equals its own negative (0 or n/2 on each axis)
    selfc = np.ones(Hs.shape, dtype=bool)
    for i, n in enumerate(dims):
        m = np.arange(Hs.shape[i])
        sh = [1] * len(dims)
        sh[i] = Hs.shape[i]
        selfc = selfc & ((m == 0) | (2 * m == n)).reshape(sh)
    rel_se = np.where(selfc, np.sqrt(2.0 / NSEED), np.sqrt(1.0 / NSEED))
    live = H2 > 1e-6
    z = (mean[live] - H2[live]) / (H2[live] * rel_se[live])
    assert np.max(np.abs(z)) < 5.0
    chi2 = float(np.sum(z ** 2))
    dof = int(live.sum())
    assert stats.chi2.sf(chi2, dof) > 1e-4 and stats.chi2.cdf(chi2, dof) > 1e-4
    assert np.all(mean[~live] < 1e-4)
    # Wiener-Khinchin on the lattice: E[C(r)] = ifftn(|H|^2 on the full lattice) (unnormalised field)
    Hfull2 = np.abs(np.fft.fftn(np.fft.irfftn(Hs, s=dims, axes=tuple(range(len(dims)))))) ** 2
    C_theory = np.real(np.fft.ifftn(Hfull2))
    C_emp = acov / NSEED
    assert np.max(np.abs(C_emp - C_theory)) < 6 * C_theory.flat[0] / np.sqrt(NSEED)

"""General level cut and two-point statistics of a two-phase map (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

* Level cut (Sec. II.B, last paragraphs: any functional map of the field may define the two
  phases): g = +1 where f >= t_phi, else -1, with t_phi = sigma_f Phi^-1(1 - phi) so that a
  Gaussian field of standard deviation sigma_f has expected volume fraction phi in the +1 phase
  (phi = 1/2 gives the sign map).
* Two-point probability function of the +1 phase, S_2(r) = P(x and x + r both in phase +1),
  on the periodic lattice: S_2(r) = (1/N) sum_x I(x) I(x + r) with I = (1 + g) / 2.  By the
  Wiener-Khinchin relation (the autocovariance and the spectral density are a Fourier pair,
  Eqs. (10)-(11)) it is ifftn(|fftn(I)|^2) / N.
"""

import math

import numpy as np
import scipy.special


def level_threshold(phi, sigma_f=1.0):
    """t_phi = sigma_f Phi^-1(1 - phi), 0 < phi < 1, evaluated as -sigma_f Phi^-1(phi) (the normal
    quantile is odd about 1/2): forming 1 - phi first would drop the relative precision of a small
    tail probability."""
    if not (0.0 < phi < 1.0):
        raise ValueError("phi must lie in (0, 1)")
    return -sigma_f * float(scipy.special.ndtri(phi))


def level_cut(f, t):
    """+1 where f >= t, else -1 (int8)."""
    return np.where(np.asarray(f) >= t, 1, -1).astype(np.int8)


def s2_map(g):
    """S_2(r) of the +1 phase of the +-1 map g, for every lattice displacement r (array of g's shape,
    index = r mod n per axis)."""
    I = (1.0 + np.asarray(g, dtype=np.float64)) / 2.0
    X = np.fft.fftn(I)
    return np.real(np.fft.ifftn(np.abs(X) ** 2)) / I.size


def s2_brute(g):
    """The same by its definition (small maps only): average over x of I(x) I(x + r)."""
    I = (1.0 + np.asarray(g, dtype=np.float64)) / 2.0
    out = np.empty_like(I)
    for r in np.ndindex(*I.shape):
        out[r] = float(np.mean(I * np.roll(I, shift=tuple(-k for k in r), axis=tuple(range(I.ndim)))))
    return out

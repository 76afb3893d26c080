"""Hyperuniformity diagnostics of a field (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

* Local variance over a spherical window, Sec. II.A Eq. (1): sigma_F^2(R) is the variance of the
  field averaged over a ball (disk in 2D) of radius R.  On the periodic lattice the field is the
  trigonometric polynomial of its DFT, and averaging one Fourier mode of wavevector k over a ball
  multiplies it by the window's normalised form factor
      W_2(u) = 2 J_1(u) / u,                       W_3(u) = 3 (sin u - u cos u) / u^3,   u = |k| R,
  so over all window positions (which is the same as over the lattice positions, by orthogonality)
      sigma_F^2(R) = sum_{m != 0} |X(m)|^2 / N^2 * W_d(|k_m| R)^2,
  with X the unnormalised DFT, k_m = 2 pi m~ / n per axis (m~ the signed index, lattice spacing 1)
  and the mean mode excluded.  This is the Fourier form of Eq. (1) (the windowed integral of the
  autocovariance equals the spectral density weighted by the squared form factor).
* Small-k exponent of a binned spectrum, Sec. II.A (spectral density ~ |k|^alpha at small k):
  least-squares slope of ln P against ln k over radial bins 1..nfit (bin 0 holds the DC mode),
  P the bin mean and k the bin centre (r + 1/2) / R in Nyquist units.
* Class of Eqs. (6)-(7) from an exponent alpha.
"""

import math

import numpy as np
import scipy.special


def _signed_index(n):
    m = np.arange(n)
    return np.where(m < n // 2, m, m - n)


def form_factor(u, d):
    """W_d(u): the average of exp(i k.y) over a ball of radius R, u = |k| R (d = 2 or 3)."""
    u = np.asarray(u, dtype=np.float64)
    out = np.ones_like(u)
    nz = u != 0.0
    if d == 2:
        out[nz] = 2.0 * scipy.special.j1(u[nz]) / u[nz]
    elif d == 3:
        v = u[nz]
        out[nz] = 3.0 * (np.sin(v) - v * np.cos(v)) / v ** 3
    else:
        raise ValueError("d must be 2 or 3")
    return out


def window_variance(x, radii):
    """sigma_F^2(R) of the real periodic field x (shape = dims) for each R in radii (lattice units)."""
    x = np.asarray(x, dtype=np.float64)
    d = x.ndim
    N = x.size
    X = np.fft.fftn(x)
    P = np.abs(X) ** 2 / float(N) ** 2
    grids = np.meshgrid(*[2.0 * math.pi * _signed_index(n) / n for n in x.shape], indexing="ij")
    k = np.sqrt(sum(g * g for g in grids))
    P.flat[0] = 0.0                                   # the mean mode
    return np.array([float(np.sum(P * form_factor(k * R, d) ** 2)) for R in radii])


def small_k_exponent(bin_sum, bin_cnt, n_radial, nfit, n_angular=1):
    """Slope of ln P(k) over radial bins 1..nfit of a binned spectrum (flattened r * A + a)."""
    s = np.asarray(bin_sum, dtype=np.float64)[: n_radial * n_angular].reshape(n_radial, n_angular).sum(axis=1)
    c = np.asarray(bin_cnt, dtype=np.float64)[: n_radial * n_angular].reshape(n_radial, n_angular).sum(axis=1)
    r = np.arange(1, nfit + 1)
    ok = (c[r] > 0) & (s[r] > 0)
    if np.count_nonzero(ok) < 2:
        raise ValueError("fewer than two usable bins")
    lk = np.log((r[ok] + 0.5) / n_radial)
    lp = np.log(s[r[ok]] / c[r[ok]])
    A = np.stack([lk, np.ones_like(lk)], axis=1)
    slope, _ = np.linalg.lstsq(A, lp, rcond=None)[0]
    return float(slope)


CLASSES = ("hyperuniform class I", "hyperuniform class II", "hyperuniform class III",
           "nonhyperuniform (standard)", "antihyperuniform", "outside the classified range")


def hyperuniformity_class(alpha, d, tol=1e-6):
    """Index into CLASSES for a small-k exponent alpha in dimension d, Eqs. (6)-(7)."""
    if abs(alpha - 1.0) <= tol:
        return 1
    if alpha > 1.0:
        return 0
    if abs(alpha) <= tol:
        return 3
    if alpha > 0.0:
        return 2
    if alpha > -d:
        return 4
    return 5

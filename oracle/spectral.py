"""Generalized-superellipse spectral density and filter amplitude (FP64).

Definitions followed:
* superellipse norm K_{p,a,b}, Eq. (12): [(|k_x|/a)^p + (|k_y|/b)^p]^(1/p), with a third term
  (|k_z|/c)^p in 3D (the sentence after Eq. (12));
* target spectral density, Eq. (13): chi = C exp[alpha ln K - K^2/(2 sigma^2)], C fixing max chi = 1;
* filter amplitude, Eq. (8): A = sqrt(chi).

Mask variants beyond the paper's alpha > 0 (it states it omits any offset regularisation): alpha = 0
(the standard nonhyperuniform class of Eq. (7), chi(0) > 0), -d < alpha < 0 (antihyperuniform,
chi diverging as k -> 0; the continuum then has no maximum, so C is fixed by the bound of
``ln_chi_ref`` on the lattice), and an offset regularisation chi_rel + offset (offset >= 0,
relative to the continuum peak; alpha >= 0 only), which makes chi(k -> 0) = offset.  The DC mode
gets amplitude 0 for every alpha and offset: Eq. (15) removes the mean anyway.

A tabulated radial form (a radial profile beyond Eq. (13); Sec. IV names more elaborate radial
forms as the natural generalisation): ``prof`` holds ln chi at K = i * prof_dk, i = 0 .. n - 1,
and ln chi(K) is its linear interpolation, held at the last sample for K beyond the table; the
samples are used as given (no normalisation constant; the field is normalised by Eq. (15)).

Readings where the paper is silent or ambiguous (each is listed in the design notes):
* wavenumbers are in units of the Nyquist wavenumber: kappa_i = 2 m~_i / n_i with m~ the
  signed index (m for m < n/2, else m - n), except along the halved last axis of the
  real-to-complex half spectrum, where kappa_x = 2 m_x / n_x >= 0;
* a band centre k0 generalises Eq. (13): ln chi = alpha ln K - (K - k0)^2 / (2 w^2) - ln chi_max,
  which is exactly Eq. (13) at k0 = 0 with w = sigma;
* C is the continuum maximum, reached at K* = (k0 + sqrt(k0^2 + 4 alpha w^2)) / 2;
* the mask is rotated counter-clockwise by ``rot`` in the (kappa_x, kappa_y) plane (about z in 3D):
  kappa'_x = cos(rot) kx + sin(rot) ky, kappa'_y = -sin(rot) kx + cos(rot) ky;
* semi-axis a goes with x (last array axis), b with y, c with z;
* on Nyquist planes the amplitude is symmetrised, H_sym(m) = (H(kappa(m)) + H(kappa(-m))) / 2 with
  kappa the canonical full-lattice wavenumber (-1 at every Nyquist index), so that H_sym * W stays
  Hermitian and the real field equals Re(ifftn(H * fftn(w))) with H on the canonical full lattice.
"""

from dataclasses import dataclass
import numpy as np


class DegenerateFilter(ValueError):
    """The lattice maximum of ln chi (relative to its continuum peak) is below -80."""


DEGENERATE_LN_CHI = -80.0


@dataclass(frozen=True)
class FilterParams:
    """Parameters of Eqs. (12)-(13) plus the readings above.

    p      superellipse exponent (Eq. (12))
    semi   (a, b, c): semi-axes for x, y, z (c unused in 2D)
    rot    mask rotation in radians, counter-clockwise in (kappa_x, kappa_y)
    alpha  small-k exponent (Eqs. (13)-(14)), > -d (0: standard nonhyperuniform, < 0 antihyperuniform)
    k0     band centre in Nyquist units (0 reproduces Eq. (13))
    width  Gaussian band width w (sigma of Eq. (13)) in Nyquist units
    sigma_f target standard deviation of the field (Eq. (15))
    offset regularisation added to chi_rel (>= 0; 0 is the paper's mask)
    prof   tabulated radial form: ln chi at K = i * prof_dk (replaces alpha, k0, width), or None
    """
    p: float
    semi: tuple = (1.0, 1.0, 1.0)
    rot: float = 0.0
    alpha: float = 2.0
    k0: float = 0.0
    width: float = 0.1
    sigma_f: float = 1.0
    offset: float = 0.0
    prof: tuple = None      # tabulated ln chi at K = i * prof_dk, or None for Eq. (13)
    prof_dk: float = 0.0

    def replace(self, **kw):
        d = dict(p=self.p, semi=tuple(self.semi), rot=self.rot, alpha=self.alpha,
                 k0=self.k0, width=self.width, sigma_f=self.sigma_f, offset=self.offset,
                 prof=self.prof, prof_dk=self.prof_dk)
        d.update(kw)
        d["semi"] = tuple(float(s) for s in d["semi"]) + (1.0,) * (3 - len(d["semi"]))
        return FilterParams(**d)


def _signed_index(n):
    m = np.arange(n)
    return np.where(m < n // 2, m, m - n)


def wavenumbers_half(dims):
    """kappa arrays (one per axis, broadcastable) on the rfftn half spectrum of ``dims``."""
    d = len(dims)
    out = []
    for i, n in enumerate(dims):
        shape = [1] * d
        if i == d - 1:
            k = 2.0 * np.arange(n // 2 + 1) / n
            shape[i] = n // 2 + 1
        else:
            k = 2.0 * _signed_index(n) / n
            shape[i] = n
        out.append(k.reshape(shape))
    return out


def wavenumbers_full(dims):
    """kappa arrays on the full fftn lattice (canonical signed index on every axis)."""
    d = len(dims)
    out = []
    for i, n in enumerate(dims):
        shape = [1] * d
        shape[i] = n
        out.append((2.0 * _signed_index(n) / n).reshape(shape))
    return out


def _xyz(kappas):
    """Return (kx, ky, kz) from axis-ordered kappas (x = last axis); kz is None in 2D."""
    if len(kappas) == 2:
        return kappas[1], kappas[0], None
    return kappas[2], kappas[1], kappas[0]


def superellipse_K(kappas, filt):
    """K of Eq. (12) on the rotated wavenumbers; returns (K, u-list, kappa'-list).

    Evaluated as K = u_max (sum_i (u_i / u_max)^p)^(1/p), the same function written so that
    u^p neither underflows nor overflows for large p (the paper uses p up to 100)."""
    kx, ky, kz = _xyz(kappas)
    c, s = np.cos(filt.rot), np.sin(filt.rot)
    kxr = c * kx + s * ky
    kyr = -s * kx + c * ky
    comps = [kxr, kyr] + ([kz] if kz is not None else [])
    us = [np.abs(k) / filt.semi[i] for i, k in enumerate(comps)]
    us = np.broadcast_arrays(*us)
    umax = np.maximum.reduce(us)
    safe = np.where(umax > 0, umax, 1.0)
    S = sum((u / safe) ** filt.p for u in us)
    K = np.where(umax > 0, umax * S ** (1.0 / filt.p), 0.0)
    return K, list(us), comps


def k_star(filt):
    """Continuum peak of alpha ln K - (K - k0)^2/(2 w^2): root of K^2 - k0 K - alpha w^2 = 0 (for
    alpha < 0 the band's local maximum, when k0^2 + 4 alpha w^2 >= 0)."""
    return 0.5 * (filt.k0 + np.sqrt(filt.k0 ** 2 + 4.0 * filt.alpha * filt.width ** 2))


def k_low(kappas, filt):
    """For alpha < 0: a lower bound of K over every nonzero lattice wavenumber,
    min_i (smallest nonzero |kappa_i|) / (sqrt(d) max_i semi_i), since K >= max_i u_i >= |kappa'| /
    (sqrt(d) max semi)."""
    d = len(kappas)
    kmin = min(float(np.min(np.abs(k[k != 0]))) for k in kappas)
    return kmin / (np.sqrt(d) * max(filt.semi[:d]))


def ln_chi_ref(filt, kappas=None):
    """The normalisation of Eq. (13) (ln C = -ln chi_ref): the continuum peak for alpha >= 0; for
    alpha < 0, where the continuum has no maximum as K -> 0, the larger of chi at k_low and at the
    band's local maximum, which bounds chi on the lattice."""
    if filt.alpha >= 0.0:
        return float(ln_chi_unnorm(np.float64(k_star(filt)), filt))
    if kappas is None:
        raise ValueError("alpha < 0 needs the lattice for its normalisation")
    ref = float(ln_chi_unnorm(np.float64(k_low(kappas, filt)), filt))
    disc = filt.k0 ** 2 + 4.0 * filt.alpha * filt.width ** 2
    if disc >= 0.0:
        ref = max(ref, float(ln_chi_unnorm(np.float64(k_star(filt)), filt)))
    return ref


def ln_chi_unnorm(K, filt):
    """alpha ln K - (K - k0)^2/(2 w^2); -inf at K = 0 for alpha > 0 (chi(0) = 0, Eq. (4)); the
    alpha ln K term is 0 for alpha = 0."""
    with np.errstate(divide="ignore", invalid="ignore"):
        lnK = np.log(K)
        a = np.where(filt.alpha == 0.0, 0.0, filt.alpha * lnK)
    return a - (K - filt.k0) ** 2 / (2.0 * filt.width ** 2)


def ln_chi_rel(K, filt, kappas=None):
    """ln chi - ln chi_ref, i.e. ln chi of Eq. (13) with C = 1/chi_ref (max chi = 1 for alpha >= 0);
    for a tabulated radial form, the interpolated samples as given."""
    if filt.prof is not None:
        prof = np.asarray(filt.prof, dtype=np.float64)
        return np.interp(K, filt.prof_dk * np.arange(prof.size), prof)
    return ln_chi_unnorm(K, filt) - ln_chi_ref(filt, kappas)


def _amplitude(kappas, filt):
    """H = sqrt(chi_rel + offset) off the DC mode, 0 at the DC mode; also returns ln(chi_rel + offset)."""
    K, _, _ = superellipse_K(kappas, filt)
    lc = ln_chi_rel(K, filt, kappas)
    if filt.offset > 0.0:
        lc = np.logaddexp(lc, np.log(filt.offset))
    lc = np.where(K > 0, lc, -np.inf)
    return np.exp(0.5 * lc), lc


def _check_degenerate(lc):
    m = np.max(lc)
    if not np.isfinite(m) or m < DEGENERATE_LN_CHI:
        raise DegenerateFilter("max ln chi over the lattice is %r < %g" % (m, DEGENERATE_LN_CHI))


def amplitude_half(dims, filt, check=True):
    """H = sqrt(chi) (Eq. (8)) on the half-spectrum wavenumbers, unsymmetrised."""
    H, lc = _amplitude(wavenumbers_half(dims), filt)
    if check:
        _check_degenerate(lc)
    return H


def _canonical_half(dims):
    """kappa on the half spectrum with the canonical (full-lattice) sign at the x Nyquist index,
    kappa_x = -1 at m_x = n_x/2, as in the full lattice's signed index."""
    ks = wavenumbers_half(dims)
    n = dims[-1]
    m = np.arange(ks[-1].size).reshape(ks[-1].shape)
    ks[-1] = np.where(2 * m == n, -1.0, ks[-1])
    return ks


def _nyquist_flipped(dims):
    """Canonical half-spectrum kappa with every Nyquist component negated: by evenness of H
    this is the wavenumber of the conjugate partner -m."""
    out = []
    for i, k in enumerate(_canonical_half(dims)):
        n = dims[i]
        m = np.arange(k.size).reshape(k.shape)
        out.append(np.where(2 * m == n, -k, k))
    return out


def amplitude_sym(dims, filt, check=True):
    """H_sym(m) = (H(kappa(m)) + H(kappa(-m))) / 2 with kappa the canonical full-lattice
    wavenumber: the Hermitian part of H, so that irfftn(H_sym rfftn(w)) equals
    Re(ifftn(H fftn(w))).  It equals H off the Nyquist planes, and differs there only when the
    mask is rotated."""
    H, lc = _amplitude(_canonical_half(dims), filt)
    if check:
        _check_degenerate(lc)
    HN, _ = _amplitude(_nyquist_flipped(dims), filt)
    return 0.5 * (H + HN)


def amplitude_full(dims, filt, check=True):
    """H on the full canonical lattice (for the plain complex route Re(ifftn(H fftn(w))))."""
    H, lc = _amplitude(wavenumbers_full(dims), filt)
    if check:
        _check_degenerate(lc)
    return H

"""Field generation, normalisation and the sign threshold (FP64).

Pipeline (Sec. II.B): white noise -> forward FFT -> multiply by A = sqrt(chi) (Eq. (8)) ->
inverse FFT to a real field (Eq. (9)) -> demean and rescale to sigma_f (Eq. (15)) ->
optional sign map to a +-1 medium.

Readings:
* forward transform with kernel exp(-i k.x), unnormalised; inverse exp(+i k.x) with 1/N
  (numpy's rfftn/irfftn); the scale cancels in Eq. (15) but the sign does not;
* the noise is real white noise, so its transform is Hermitian and the field is real;
* Var[f] in Eq. (15) is the population variance (ddof = 0);
* sgn(0) is taken as +1 (f >= 0 -> +1, including -0.0), so no third phase appears.
"""

import numpy as np

from .philox import white_noise
from .spectral import amplitude_sym


def gen_field(dims, filt, seed):
    """Normalised field f and its intermediates for one seed.

    Returns a dict with
      w      real white noise,
      W      rfftn(w),
      Hs     symmetrised amplitude on the half spectrum,
      F      Hs * W (the filtered half spectrum, Eq. (8)),
      f_raw  irfftn(F) (Eq. (9)),
      mu, var  mean and population variance of f_raw,
      f      sigma_f (f_raw - mu) / sqrt(var) (Eq. (15)).
    """
    dims = tuple(int(n) for n in dims)
    w = white_noise(dims, seed)
    W = np.fft.rfftn(w)
    Hs = amplitude_sym(dims, filt)
    F = Hs * W
    f_raw = np.fft.irfftn(F, s=dims, axes=tuple(range(len(dims))))
    mu = float(f_raw.mean())
    var = float(((f_raw - mu) ** 2).mean())
    f = filt.sigma_f * (f_raw - mu) / np.sqrt(var)
    return dict(w=w, W=W, Hs=Hs, F=F, f_raw=f_raw, mu=mu, var=var, f=f)


def threshold(f, sigma_f=1.0, near_tol=1e-5):
    """Sign map t = +1 where f >= 0 else -1 (int8), with n_pos = #(t = +1) and
    n_near = #(|f| < near_tol * sigma_f), the sites whose sign is fragile under rounding."""
    f = np.asarray(f)
    t = np.where(f >= 0, 1, -1).astype(np.int8)
    n_pos = int(np.count_nonzero(t == 1))
    n_near = int(np.count_nonzero(np.abs(f) < near_tol * sigma_f))
    return t, n_pos, n_near


def pipeline(dims, filt, seed, nr, na=1):
    """Whole hot path for one field: field, threshold, continuous and +-1 binned spectra."""
    from .spectrum import power_spectrum
    out = gen_field(dims, filt, seed)
    t, n_pos, n_near = threshold(out["f"], filt.sigma_f)
    out.update(t=t, n_pos=n_pos, n_near=n_near)
    out["cont_sum"], out["cont_cnt"] = power_spectrum(out["f"], nr, na)
    out["pm1_sum"], out["pm1_cnt"] = power_spectrum(t.astype(np.float64), nr, na)
    return out

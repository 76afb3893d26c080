"""Binned power spectra of real fields (FP64, exact integer bin rules).

The paper shows the log spectral density of the continuous and the +-1 fields in every
figure row (Sec. III) but defines no estimator or binning.  Reading adopted:
* periodogram P(k) = |DFT(g)(k)|^2 / N on the lattice (unnormalised forward DFT);
* the real-to-complex half spectrum stands for the full lattice with multiplicity
  w = 1 where m_x is 0 or n_x/2 and w = 2 elsewhere;
* radial bin r = floor(R |kappa|), |kappa| in Nyquist units, computed exactly in integers:
  with D = lcm(n_i) and q_i = m~_i D / n_i, r is the largest integer with
  r^2 D^2 <= 4 R^2 sum q_i^2 (a mode on a bin edge goes to the upper bin);
  modes with r >= R (the corners, |kappa| >= 1) go to one extra "excluded" slot;
* angular bin (2D, A bins over [0, pi)): fold q -> -q when q_y < 0 (q_x >= 0 on the half
  spectrum); bin = #{j = 1..A-1 : e_jx q_y - e_jy q_x >= 0} in FP64 with separately rounded
  products, e_j = (cos j pi/A, sin j pi/A), the 45, 90 and 135 degree edges set exactly to
  (c, c), (0, 1), (-c, c); the DC mode goes to angular bin 0;
* outputs: per-bin sum of w P (FP64) and sum of w (integer), flattened r * A + a, with the
  excluded slot last (index R * A).
"""

import math
import numpy as np


def _lcm(values):
    out = 1
    for v in values:
        out = out * v // math.gcd(out, v)
    return out


def _signed_index(n):
    m = np.arange(n)
    return np.where(m < n // 2, m, m - n)


def angular_edges(na):
    """Unit vectors e_j, j = 1..na-1, at angles j pi / na, with the exact-tangent edges exact."""
    ex = np.empty(max(na - 1, 0))
    ey = np.empty(max(na - 1, 0))
    c = math.cos(math.pi / 4)
    for j in range(1, na):
        if 4 * j == na:
            ex[j - 1], ey[j - 1] = c, c
        elif 2 * j == na:
            ex[j - 1], ey[j - 1] = 0.0, 1.0
        elif 4 * j == 3 * na:
            ex[j - 1], ey[j - 1] = -c, c
        else:
            ex[j - 1], ey[j - 1] = math.cos(j * math.pi / na), math.sin(j * math.pi / na)
    return ex, ey


def bin_table(dims, nr, na=1):
    """Flat bin index (shape of the half spectrum, int64) and multiplicity weight w."""
    dims = tuple(int(n) for n in dims)
    d = len(dims)
    if na > 1 and d != 2:
        raise ValueError("angular bins are defined for 2D grids only")
    D = _lcm(dims)
    qs = []
    for i, n in enumerate(dims):
        shape = [1] * d
        if i == d - 1:
            m = np.arange(n // 2 + 1, dtype=np.int64)
            shape[i] = n // 2 + 1
        else:
            m = _signed_index(n).astype(np.int64)
            shape[i] = n
        qs.append((m * (D // n)).reshape(shape))
    s = sum(q * q for q in qs)                       # integer sum of q_i^2
    rhs = 4 * nr * nr * s                            # compare r^2 D^2 <= rhs
    r = np.floor(np.sqrt(rhs.astype(np.float64) / float(D * D))).astype(np.int64)
    # exact integer correction of the float estimate
    D2 = D * D
    r = np.where(r * r * D2 > rhs, r - 1, r)
    r = np.where((r + 1) * (r + 1) * D2 <= rhs, r + 1, r)
    if na > 1:
        qy = np.broadcast_to(qs[0], s.shape).astype(np.int64)
        qx = np.broadcast_to(qs[1], s.shape).astype(np.int64)
        flip = qy < 0
        qy = np.where(flip, -qy, qy).astype(np.float64)
        qx = np.where(flip, -qx, qx).astype(np.float64)
        ex, ey = angular_edges(na)
        a = np.zeros(s.shape, dtype=np.int64)
        for j in range(na - 1):
            t1 = ex[j] * qy                          # separately rounded FP64 products
            t2 = ey[j] * qx
            a += (t1 - t2 >= 0.0)
        a = np.where(s == 0, 0, a)
    else:
        a = np.zeros(s.shape, dtype=np.int64)
    idx = np.where(r >= nr, nr * na, r * na + a)
    mx = np.arange(dims[-1] // 2 + 1).reshape([1] * (d - 1) + [-1])
    w = np.where((mx == 0) | (2 * mx == dims[-1]), 1, 2)
    return np.broadcast_to(idx, s.shape), np.broadcast_to(w, s.shape)


def bin_power(P, dims, nr, na=1):
    """Sum of w * P and of w per bin (excluded slot last) for a half-spectrum array P."""
    idx, w = bin_table(dims, nr, na)
    nb = nr * na + 1
    ssum = np.bincount(idx.ravel(), weights=(w * P).ravel(), minlength=nb)
    cnt = np.bincount(idx.ravel(), weights=w.ravel().astype(np.float64), minlength=nb)
    return ssum, np.rint(cnt).astype(np.uint64)


def power_spectrum(g, nr, na=1):
    """Binned periodogram of a real field g: P = |rfftn(g)|^2 / N."""
    g = np.asarray(g, dtype=np.float64)
    G = np.fft.rfftn(g)
    P = (G.real ** 2 + G.imag ** 2) / g.size
    return bin_power(P, g.shape, nr, na)


def continuous_spectrum_fused(F, dims, nr, na=1, sigma_f=1.0):
    """Binned spectrum of the normalised field taken from the filtered half spectrum F:
    P(k) = sigma_f^2 |F(k)|^2 / (N v) for k != 0 and 0 at k = 0, with v = sum_half w |F|^2 / N^2 - mu^2
    and mu = Re F(0) / N (Parseval), i.e. Eq. (15) applied in Fourier space."""
    dims = tuple(dims)
    N = int(np.prod(dims))
    _, w = bin_table(dims, nr, na)
    A = F.real ** 2 + F.imag ** 2
    mu = F.flat[0].real / N
    v = float(np.sum(w * A)) / N ** 2 - mu ** 2
    P = sigma_f ** 2 * A / (N * v)
    P.flat[0] = 0.0
    return bin_power(P, dims, nr, na)

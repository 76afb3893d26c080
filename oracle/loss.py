"""Spectrum-matching loss and its analytic gradient with respect to the filter parameters (FP64).

The paper lists optimisation loops over the spectral parameters as future work (Sec. IV).
The loss adopted: the mean squared log-difference between the field's radial continuous
spectrum (bins 1..R-1 with modes) and the expected spectrum of a target parameter set,

    L = (1/|B|) sum_b (ln(P_b + eps) - ln(T_b + eps))^2 ,  eps = 1e-12 sigma_f^2,

with P_b = sigma_f^2 N G_b / (c_b G_tot), G_b = sum_{k in b} w H^2 |W|^2, G_tot = the same sum over
every mode, c_b the mode count of bin b, and T_b the bin mean of sigma_f^2 N H_t^2 / sum_k H_t^2.
The noise W is a pure function of the seed, so the gradient recomputes it instead of storing it.

Gradient (chain rule through G_b and G_tot; the constant C of Eq. (13) cancels):
    lambda_b = (2/|B|) (ln(P_b+eps) - ln(T_b+eps)) P_b / (P_b + eps),  Lambda = sum_b lambda_b,
    omega(k) = lambda_{b(k)} / G_{b(k)} [b(k) in B] - Lambda / G_tot,
    dL/dtheta_j = sum_k w omega(k) 2 H_sym dH_sym/dtheta_j |W|^2 .
"""

import numpy as np

from .philox import white_noise
from .spectral import superellipse_K, ln_chi_rel, amplitude_sym, _canonical_half, _nyquist_flipped
from .spectrum import bin_table

PARAM_NAMES = ("a", "b", "c", "p", "rot", "k0", "width")


def _theta(filt):
    return np.array([filt.semi[0], filt.semi[1], filt.semi[2], filt.p, filt.rot, filt.k0, filt.width])


def _with_theta(filt, th):
    return filt.replace(semi=(th[0], th[1], th[2]), p=th[3], rot=th[4], k0=th[5], width=th[6])


def _bins_radial(dims, nr):
    idx, w = bin_table(dims, nr, 1)
    return np.ascontiguousarray(idx), np.ascontiguousarray(w).astype(np.float64)


def target_bins(dims, filt_t, nr):
    """T_b: bin means of sigma_f^2 N H_t^2 / sum_full H_t^2 (expected normalised spectrum)."""
    dims = tuple(dims)
    N = int(np.prod(dims))
    idx, w = _bins_radial(dims, nr)
    H2 = amplitude_sym(dims, filt_t) ** 2
    T = filt_t.sigma_f ** 2 * N * H2 / np.sum(w * H2)
    s = np.bincount(idx.ravel(), weights=(w * T).ravel(), minlength=nr + 1)[:nr]
    c = np.bincount(idx.ravel(), weights=w.ravel(), minlength=nr + 1)[:nr]
    with np.errstate(invalid="ignore", divide="ignore"):
        return np.where(c > 0, s / np.maximum(c, 1), 0.0), c


def _loss_from_W(W2, dims, filt, T_b, nr, eps_rel):
    dims = tuple(dims)
    N = int(np.prod(dims))
    idx, w = _bins_radial(dims, nr)
    H2 = amplitude_sym(dims, filt) ** 2
    A = w * H2 * W2
    G_tot = float(A.sum())
    G_b = np.bincount(idx.ravel(), weights=A.ravel(), minlength=nr + 1)[:nr]
    c_b = np.bincount(idx.ravel(), weights=w.ravel(), minlength=nr + 1)[:nr]
    sf2 = filt.sigma_f ** 2
    eps = eps_rel * sf2
    B = np.zeros(nr, dtype=bool)
    B[1:] = c_b[1:] > 0
    P_b = np.zeros(nr)
    P_b[B] = sf2 * N * G_b[B] / (c_b[B] * G_tot)
    diff = np.log(P_b + eps) - np.log(T_b + eps)
    L = float(np.sum(diff[B] ** 2) / B.sum())
    return L, dict(G_tot=G_tot, G_b=G_b, c_b=c_b, P_b=P_b, B=B, diff=diff, eps=eps)


def spectrum_loss(dims, filt, seed, filt_t, nr, eps_rel=1e-12):
    """Loss L and the forward quantities (G_tot, G_b, c_b, P_b, T_b, ...)."""
    W = np.fft.rfftn(white_noise(dims, seed))
    T_b, _ = target_bins(dims, filt_t, nr)
    L, aux = _loss_from_W(W.real ** 2 + W.imag ** 2, dims, filt, T_b, nr, eps_rel)
    aux["T_b"] = T_b
    return L, aux


def _dlnH(kappas, filt):
    """H and d ln H / d theta (theta = a, b, c, p, rot, k0, w) at the wavenumbers ``kappas``,
    up to theta-dependent constants (from C), which cancel in the loss.  Partials from
    Eqs. (12)-(13): K = S^(1/p), S = sum u_i^p, u_i = |kappa'_i| / a_i."""
    K, us, comps = superellipse_K(kappas, filt)
    H = np.exp(0.5 * ln_chi_rel(K, filt, kappas))
    p, al, k0, w = filt.p, filt.alpha, filt.k0, filt.width
    pos = K > 0
    Ks = np.where(pos, K, 1.0)
    # r_i = u_i / K, so u_i^p / S = r_i^p and sum_i r_i^p = 1 (no u^p that could under/overflow)
    rs = [u / Ks for u in us]
    dK = 0.5 * (al / Ks - (Ks - k0) / w ** 2)            # d lnH / dK
    out = []
    for i in range(3):                                   # a, b, c: dK/da_i = -K r_i^p / a_i
        if i < len(us):
            out.append(dK * (-Ks * rs[i] ** p / filt.semi[i]))
        else:
            out.append(np.zeros_like(Ks))
    acc = 0.0                                            # dK/dp = (K/p) sum_i r_i^p ln r_i
    for r in rs:
        acc = acc + np.where(r > 0, r ** p * np.log(np.where(r > 0, r, 1.0)), 0.0)
    out.append(dK * (Ks / p) * acc)                      # p
    # dK/drot = sum_i r_i^(p-1) sgn(kappa'_i) (d kappa'_i / d rot) / a_i,
    # with d kappa'_x / d rot = kappa'_y and d kappa'_y / d rot = -kappa'_x
    rpm1 = [np.where(r > 0, np.where(r > 0, r, 1.0) ** (p - 1), 0.0) for r in rs[:2]]
    drot = (rpm1[0] * np.sign(comps[0]) * comps[1] / filt.semi[0]
            - rpm1[1] * np.sign(comps[1]) * comps[0] / filt.semi[1])
    out.append(dK * drot)                                # rot
    out.append(0.5 * (Ks - k0) / w ** 2)                 # k0
    out.append(0.5 * (Ks - k0) ** 2 / w ** 3)            # width
    shape = np.broadcast(*kappas).shape
    out = [np.where(pos, np.broadcast_to(o, shape), 0.0) for o in out]
    return np.broadcast_to(H, shape), out


def dlnH_half(dims, filt):
    """H_sym and d H_sym / d theta on the half spectrum (Nyquist planes differentiated term by term)."""
    H, d = _dlnH(_canonical_half(dims), filt)
    HN, dN = _dlnH(_nyquist_flipped(dims), filt)
    Hs = 0.5 * (H + HN)
    dHs = [0.5 * (H * a + HN * b) for a, b in zip(d, dN)]
    return Hs, dHs


def spectrum_loss_grad(dims, filt, seed, filt_t, nr, eps_rel=1e-12):
    """Analytic dL/dtheta (7 values, order PARAM_NAMES) with the noise recomputed from ``seed``."""
    dims = tuple(dims)
    W = np.fft.rfftn(white_noise(dims, seed))
    W2 = W.real ** 2 + W.imag ** 2
    T_b, _ = target_bins(dims, filt_t, nr)
    L, aux = _loss_from_W(W2, dims, filt, T_b, nr, eps_rel)
    B, P_b, G_b, G_tot, diff = aux["B"], aux["P_b"], aux["G_b"], aux["G_tot"], aux["diff"]
    lam = np.zeros(nr)
    lam[B] = (2.0 / B.sum()) * diff[B] * P_b[B] / (P_b[B] + aux["eps"])
    Lam = lam.sum()
    idx, w = _bins_radial(dims, nr)
    per_bin = np.zeros(nr + 1)
    per_bin[:nr][B] = lam[B] / G_b[B]
    omega = per_bin[idx] - Lam / G_tot
    Hs, dHs = dlnH_half(dims, filt)
    base = w * omega * 2.0 * Hs * W2
    grad = np.array([float(np.sum(base * d)) for d in dHs])
    return grad, L, aux


def spectrum_loss_fd(dims, filt, seed, filt_t, nr, rel_step=1e-6, eps_rel=1e-12):
    """FP64 central finite differences of L in each parameter (the independent check)."""
    W = np.fft.rfftn(white_noise(dims, seed))
    W2 = W.real ** 2 + W.imag ** 2
    T_b, _ = target_bins(dims, filt_t, nr)
    th0 = _theta(filt)
    g = np.zeros(7)
    for j in range(7):
        h = rel_step * max(abs(th0[j]), 1.0)
        tp, tm = th0.copy(), th0.copy()
        tp[j] += h
        tm[j] -= h
        Lp, _ = _loss_from_W(W2, dims, _with_theta(filt, tp), T_b, nr, eps_rel)
        Lm, _ = _loss_from_W(W2, dims, _with_theta(filt, tm), T_b, nr, eps_rel)
        g[j] = (Lp - Lm) / (2 * h)
    return g

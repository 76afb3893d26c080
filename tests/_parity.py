"""Shared GPU-vs-oracle comparisons for the parity tests, with the measured errors recorded.

Tolerances (the precision policy: FP32 transforms with FP64-generated twiddles, FP64 statistics
and bin sums; the filter's ln chi in FP32, or in FP64 where its FP32 rounding would not keep the
field within tolerance):
* field: max |f_gpu - f_oracle| <= 1e-5 * RMS;
* sign map: bit-exact except at sites with |f_oracle| < 1e-5 * RMS (counted);
* raw mean: |mu_gpu - mu| <= 1e-6 sqrt(var); raw variance: rtol 1e-6;
* bin counts exact; continuous bins against the oracle's fused form (the same spectrum taken from
  the filtered half spectrum F in FP64, which the oracle pins to the plain periodogram of f; the
  plain route's FP64 round trip through the field leaves an absolute error of about 1e-12 on each
  |F(k)|, i.e. relative errors up to 1e-2 in bins below 1e-20 of the largest): rtol 1e-5 for bins
  at >= 1e-3 of the largest bin (the band); further out, where chi falls to e^-10 .. e^-70 of its
  peak, the FP32 filter's own error grows: its superellipse norm K carries a relative rounding of
  ~1e-7 through the log2 / exp2 chain, which moves ln chi by |d ln chi / d ln K| dK/K (the slope
  grows like K (K - k0) / w^2 in the band's tails), and the terms of ln chi, whose FP32 rounding
  adds to it, grow with |ln chi| there; so each e-fold of the bin below 1e-3 of the largest adds
  1e-6 to its tolerance (measured: 1.2e-5 at 1e-9 of the largest bin for w = 0.04, 1.1e-5 at 1.5e-7
  for w = 0.02, 2.3e-5 at 1e-28); bins below 1e-30 of the largest only have an absolute floor;
* +-1 bins rtol 1e-5 when no site flips; with m flipped sites each mode's |T(k)|^2 / N moves by
  at most (4 m |T(k)| + 4 m^2) / N, so a bin may move by its multiplicity-weighted sum of that.

Every comparison appends one JSON line with the measured errors to the file that the environment
variable HU_PARITY_REPORT names, when it is set (a relative path is taken from the repository
root): field err/RMS, flips,
near-zero sites, mean and variance errors, and for each spectrum the largest relative bin error
in three bands of bin magnitude (>= 1e-3 of the largest bin, 1e-9 .. 1e-3, below 1e-9).
"""

import json
import math
import os

import numpy as np

import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
REPORT = os.path.join(ROOT, os.environ["HU_PARITY_REPORT"]) if os.environ.get("HU_PARITY_REPORT") else None

FIELD_TOL = 1e-5
NEAR_TOL = 1e-5
STAT_TOL = 1e-6
BIN_RTOL = 1e-5
UNDERFLOW_FLOOR = 1e-30


def record(kind, name, **kw):
    """Append one line of measured errors to the parity report (when one is named)."""
    if REPORT is None:
        return
    try:
        os.makedirs(os.path.dirname(REPORT), exist_ok=True)
        with open(REPORT, "a") as fh:
            fh.write(json.dumps(dict(kind=kind, name=name, **kw), default=float) + "\n")
    except OSError:
        pass


def band_errors(got, ref):
    """Largest relative error of the bins in three bands of magnitude relative to the largest bin,
    with the worst bin's index and magnitude."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    top = float(np.max(np.abs(ref))) if ref.size else 0.0
    out = {}
    if top == 0.0:
        return dict(hi=0.0, mid=0.0, lo=0.0)
    rel = np.abs(got - ref) / np.maximum(np.abs(ref), 1e-300)
    mag = np.abs(ref) / top
    for key, sel in (("hi", mag >= 1e-3), ("mid", (mag < 1e-3) & (mag >= 1e-9)),
                     ("lo", (mag < 1e-9) & (mag >= UNDERFLOW_FLOOR))):
        out[key] = float(np.max(rel[sel])) if np.any(sel) else 0.0
        if np.any(sel):
            i = int(np.flatnonzero(sel)[np.argmax(rel[sel])])
            out[key + "_worst"] = [i, float(mag[i])]
    return out


BAND_EDGE = 1e-3          # bins at >= BAND_EDGE of the largest: BIN_RTOL
TAIL_RTOL_PER_EFOLD = 1e-6


def bin_rtol(ref, log_scaled):
    """Per-bin relative tolerance: BIN_RTOL, plus TAIL_RTOL_PER_EFOLD per e-fold of the bin below
    BAND_EDGE of the largest bin when log_scaled (the FP32 filter's error model, see the module
    notes)."""
    ref = np.abs(np.asarray(ref, dtype=np.float64))
    if not log_scaled:
        return np.full(ref.shape, BIN_RTOL)
    mag = ref / max(float(np.max(ref)), 1e-300)
    efolds = np.maximum(0.0, np.log(BAND_EDGE) - np.log(np.clip(mag, 1e-300, 1.0)))
    return BIN_RTOL + TAIL_RTOL_PER_EFOLD * efolds


# +-1 spectrum: the FP32 transforms perturb a mode's X by about c eps32 sqrt(N) (the transform of
# N values of magnitude 1), so its power P = w |X|^2 / N moves by about 2 c eps32 sqrt(P), and a
# bin of many modes with random rounding signs by about 2 c eps32 sqrt(bin sum).  With c ~ 3 and
# a margin of 5 this is PM1_ABS sqrt(bin); it matters only for bins of a few weak modes (many
# bins on a small grid), where the relative tolerance alone asks for more than FP32 gives.
PM1_ABS = 2e-6


def check_bins(got, ref, what, log_scaled=False, sqrt_abs=0.0):
    """Per-bin tolerance bin_rtol, plus sqrt_abs sqrt(|ref|) (the +-1 spectrum's FP32 transform
    error), with an absolute floor at UNDERFLOW_FLOOR of the largest bin."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    floor = UNDERFLOW_FLOOR * float(np.max(np.abs(ref)))
    tol = bin_rtol(ref, log_scaled) * np.abs(ref) + sqrt_abs * np.sqrt(np.abs(ref)) + floor
    bad = np.abs(got - ref) > tol
    assert not np.any(bad), (what, np.nonzero(bad)[0][:8], got[bad][:4], ref[bad][:4])


def pm1_flip_bound(t_ref, m, dims, nr, na):
    """Per-bin bound on the change of the +-1 bin sums when m sites of t flip."""
    N = int(np.prod(dims))
    T = np.abs(np.fft.rfftn(t_ref.astype(np.float64)))
    idx, w = O.bin_table(dims, nr, na)
    per = w * (4.0 * m * T + 4.0 * m * m) / N
    return np.bincount(idx.ravel(), weights=per.ravel(), minlength=nr * na + 1)


def compare_field(name, dims, filt, seed, bins, got, ref=None):
    """Compare one field's GPU outputs with the oracle and record the errors.

    got: dict of host arrays: field (f32 or f64), pm1 (int8), stats [4] or None, counts [2] or
    None, cont_sum/cont_cnt, pm1_sum/pm1_cnt (each may be None).  ref: the oracle's pipeline
    output, or its gen_field output when no sign map or +-1 spectrum is compared.  Returns the
    record."""
    nr, na = bins
    fp = filt if isinstance(filt, O.FilterParams) else O.FilterParams(**filt)
    if ref is None:
        ref = O.pipeline(dims, fp, seed, nr, na)
    N = int(np.prod(dims))
    rec = dict(dims=list(dims), seed=int(seed), bins=[nr, na])
    f = np.asarray(got["field"], dtype=np.float64)
    rms = math.sqrt(float(np.mean(ref["f"] ** 2)))
    err = float(np.max(np.abs(f - ref["f"]))) / rms
    rec["field_err_rms"] = err
    near = np.abs(ref["f"]) < NEAR_TOL * rms
    rec["n_near"] = int(near.sum())
    flips = 0
    if got.get("pm1") is not None:
        t = np.asarray(got["pm1"])
        diff = t != ref["t"]
        flips = int(diff.sum())
        rec["flips"] = flips
        rec["flips_outside_near"] = int(np.sum(diff & ~near))
    if got.get("stats") is not None:
        st = np.asarray(got["stats"], dtype=np.float64)
        rec["mu_err_sd"] = abs(st[0] - ref["mu"]) / math.sqrt(ref["var"])
        rec["var_err_rel"] = abs(st[1] - ref["var"]) / ref["var"]
        rec["degenerate_flag"] = float(st[3])
    cont_ref = None
    if got.get("cont_sum") is not None:
        cont_ref, cont_cnt = O.continuous_spectrum_fused(ref["F"], dims, nr, na, fp.sigma_f)
        rec["cont_bins"] = band_errors(got["cont_sum"], cont_ref)
        if "cont_sum" in ref:
            rec["cont_bins_vs_plain"] = band_errors(got["cont_sum"], ref["cont_sum"])
    if got.get("pm1_sum") is not None:
        rec["pm1_bins"] = band_errors(got["pm1_sum"], ref["pm1_sum"])
    record("field", name, **rec)

    assert err <= FIELD_TOL, (name, seed, err)
    if "flips_outside_near" in rec:
        assert rec["flips_outside_near"] == 0, (name, seed, rec["flips_outside_near"])
    if "mu_err_sd" in rec:
        assert rec["mu_err_sd"] <= STAT_TOL, (name, seed, rec["mu_err_sd"])
        assert rec["var_err_rel"] <= STAT_TOL, (name, seed, rec["var_err_rel"])
        assert rec["degenerate_flag"] == 0.0
    if got.get("counts") is not None:
        cnt = got["counts"]
        assert abs(int(cnt[0]) - ref["n_pos"]) <= flips
        # n_near (|f| < 1e-5 sigma_f): exact up to the sites within the field tolerance of the edge
        edge = int(np.sum(np.abs(np.abs(ref["f"]) - NEAR_TOL * fp.sigma_f) <= 2 * FIELD_TOL * rms))
        assert abs(int(cnt[1]) - ref["n_near"]) <= edge, (int(cnt[1]), ref["n_near"], edge)
    if got.get("cont_sum") is not None:
        if got.get("cont_cnt") is not None:
            np.testing.assert_array_equal(got["cont_cnt"], cont_cnt)
        check_bins(got["cont_sum"], cont_ref, (name, seed, "cont"), log_scaled=True)
    if got.get("pm1_sum") is not None:
        if got.get("pm1_cnt") is not None:
            np.testing.assert_array_equal(got["pm1_cnt"], ref["pm1_cnt"])
        ps = np.asarray(got["pm1_sum"], dtype=np.float64)
        if flips == 0:
            check_bins(ps, ref["pm1_sum"], (name, seed, "pm1"), sqrt_abs=PM1_ABS)
        else:
            bound = pm1_flip_bound(ref["t"], flips, dims, nr, na)
            assert np.all(np.abs(ps - ref["pm1_sum"]) <= BIN_RTOL * ref["pm1_sum"] + bound), (name, seed)
        assert abs(ps.sum() - N) < 1e-4 * N
    return rec

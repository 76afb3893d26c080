"""Host-built bin tables behind the deterministic spectrum binning (no GPU needed).

* the bin of every half-spectrum mode equals the oracle's bin rule (exact integer radius, FP64
  angular edges), up to the full 2048^2 / 128 x 36 layout;
* each tile's partials are its distinct bins in ascending order, every mode points at its bin's
  slot, and the per-bin lists (CSR) hold every partial once, in tile order;
* the integer combination of a tile's runs (the kernels' scheme, emulated here with Python
  integers) gives the same bits for any order of the runs, and the spectrum assembled from the
  partials in CSR order equals the direct FP64 sum to rounding.
"""

import math
import os

import numpy as np
import pytest

from oracle.spectrum import bin_table

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2509_08675_amd", "libhufield.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libhufield.so not built")

# elements per thread of the axis-0 transform of each length (the run segments of the binning)
EPT = {4: 4, 6: 6, 8: 8, 12: 12, 16: 16, 24: 24, 32: 16, 48: 12, 64: 16, 96: 24, 128: 16, 192: 24, 256: 16,
       384: 24, 512: 16, 768: 24, 1024: 16, 2048: 16}

CASES = [((64, 48), (8, 6)), ((48, 64), (12, 1)), ((96, 32), (16, 4)), ((16, 12, 24), (6, 1)),
         ((24, 16, 8), (9, 1)), ((8, 8), (3, 2))]


@pytest.fixture(scope="module")
def hf():
    from paper_2509_08675_amd import hufield
    return hufield


def oracle_columns(dims, nr, na):
    idx, _ = bin_table(dims, nr, na)
    return np.ascontiguousarray(idx).reshape(dims[0], -1).T


def check_structure(t, ref, nb):
    assert np.array_equal(t["table"].astype(np.int64), ref)
    ncol, n0, w = t["ncol"], t["n0"], t["width"]
    assert t["ntiles"] == (ncol + w - 1) // w and t["toff"][0] == 0 and t["toff"][-1] == t["M"]
    nloc = 0
    for k in range(t["ntiles"]):
        cols = ref[k * w:(k + 1) * w]
        distinct = np.unique(cols)
        j0, j1 = int(t["toff"][k]), int(t["toff"][k + 1])
        assert j1 - j0 == len(distinct)
        assert np.array_equal(distinct[t["ltab"][k * w:(k + 1) * w].astype(np.int64)], cols)
        nloc = max(nloc, len(distinct))
    assert nloc == t["nloc_max"]
    # CSR: every partial once, grouped by bin, tile order inside a bin
    owner = np.concatenate([np.unique(ref[k * w:(k + 1) * w]) for k in range(t["ntiles"])])
    assert len(owner) == t["M"] and t["coff"][-1] == t["M"] and len(t["coff"]) == nb + 1
    assert np.array_equal(np.sort(t["cpos"]), np.arange(t["M"]))
    for b in range(nb):
        pos = t["cpos"][t["coff"][b]:t["coff"][b + 1]]
        assert np.all(owner[pos] == b) and np.all(np.diff(pos.astype(np.int64)) > 0)
    assert np.array_equal(np.diff(t["coff"].astype(np.int64)), np.bincount(owner, minlength=nb))


@pytest.mark.parametrize("dims,bins", CASES)
@pytest.mark.parametrize("variant", [0, 1])
def test_tables_match_oracle_bins(hf, dims, bins, variant):
    t = hf.debug_bin_tables(dims, bins, variant)
    nb = bins[0] * bins[1] + 1
    check_structure(t, oracle_columns(dims, *bins), nb)
    if bins[1] == 1:
        # radial bins: the modes e and n0 - e of a column share their bin (the binning passes pair them)
        n0 = t["n0"]
        assert np.array_equal(t["ltab"][:, 1:], t["ltab"][:, :0:-1])


def test_full_size_2d_table(hf):
    t = hf.debug_bin_tables((2048, 2048), (128, 36), 0)
    ref = oracle_columns((2048, 2048), 128, 36)
    assert np.array_equal(t["table"].astype(np.int64), ref)
    assert t["width"] == 4 and t["nloc_max"] < 1024
    # every mode's local slot points at its bin
    for k in (0, 1, 100, t["ntiles"] - 1):
        cols = ref[4 * k:4 * k + 4]
        distinct = np.unique(cols)
        assert np.array_equal(distinct[t["ltab"][4 * k:4 * k + 4].astype(np.int64)], cols)


# ---- the integer scheme of the kernels
SHIFT = 48


def tile_partials(P, t, E, rng=None):
    """Per-tile partials as the kernels form them: runs of equal local bin over E consecutive modes
    of a column, summed in FP64 in mode order; per bin the largest exponent, then each run rounded
    to 2^(e - 48) units and added as an integer; the partial is the integer sum times 2^(e - 48).
    rng: shuffle the runs of each tile first (the schedule must not matter)."""
    w, n0 = t["width"], t["n0"]
    out = np.zeros(t["M"])
    for k in range(t["ntiles"]):
        runs = []
        for g in range(k * w, min((k + 1) * w, t["ncol"])):
            for e0 in range(0, n0, E):
                loc = t["ltab"][g, e0:e0 + E]
                v = P[g, e0:e0 + E]
                cur, acc = int(loc[0]), float(v[0])
                for i in range(1, len(loc)):
                    if loc[i] != cur:
                        runs.append((cur, acc))
                        cur, acc = int(loc[i]), 0.0
                    acc += float(v[i])
                runs.append((cur, acc))
        if rng is not None:
            rng.shuffle(runs)
        ex, q = {}, {}
        for j, s in runs:
            if s > 0.0:
                ex[j] = max(ex.get(j, -10 ** 9), math.frexp(s)[1])
        for j, s in runs:
            if s > 0.0:
                x = math.ldexp(s, SHIFT - ex[j])
                assert 0.0 <= x < 2.0 ** SHIFT
                q[j] = q.get(j, 0) + (int(x + 4503599627370496.0) - (1 << 52))
        j0 = int(t["toff"][k])
        for j in q:
            assert q[j] < 1 << 63
            out[j0 + j] = math.ldexp(float(q[j]), ex[j] - SHIFT)
    return out


@pytest.mark.parametrize("dims,bins", [((64, 48), (8, 6)), ((16, 12, 24), (6, 1)), ((96, 32), (16, 4))])
def test_integer_combination(hf, dims, bins):
    t = hf.debug_bin_tables(dims, bins, 0)
    nb = bins[0] * bins[1] + 1
    rng = np.random.default_rng(5)
    # FP32 power values over many decades, some exact zeros
    P = np.exp(rng.normal(0.0, 8.0, size=t["table"].shape)).astype(np.float32)
    P[rng.random(P.shape) < 0.05] = 0.0
    E = EPT[t["n0"]]
    a = tile_partials(P, t, E)
    b = tile_partials(P, t, E, rng=np.random.default_rng(11))
    assert np.array_equal(a.view(np.int64), b.view(np.int64))
    spec = np.zeros(nb)
    for k in range(nb):
        s = 0.0
        for pos in t["cpos"][t["coff"][k]:t["coff"][k + 1]]:
            s += a[pos]
        spec[k] = s
    direct = np.bincount(t["table"].ravel().astype(np.int64), weights=P.ravel().astype(np.float64), minlength=nb)
    np.testing.assert_allclose(spec, direct, rtol=1e-13, atol=0.0)

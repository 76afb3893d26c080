"""GPU tests of the mask variants beyond the paper's alpha > 0 (alpha = 0, -d < alpha < 0 and the
offset regularisation); the whole-pipeline parity cases for them are in test_gpu_parity.py.

* the expected spectrum of a filter with an offset against the oracle (rtol 1e-5);
* the adjoint refuses a filter with an offset (HU_ERR_UNSUPPORTED), and negative alpha or offset
  are argument errors;
* the small-k exponents of generated alpha = 0 and alpha = -1 fields are near 0 and -1 (standard
  nonhyperuniform and antihyperuniform; properties of the method, statistical tolerance 0.15);
* a tabulated radial form (two bands, FP32 samples shared by both sides): its expected spectrum
  against the oracle (rtol 1e-5), a batch mixing it with Eq. (13) fields, and the whole
  pipeline against the oracle: field max-abs <= 1e-5 RMS, continuous bins rtol 1e-4.
"""

import numpy as np
import pytest
import torch

import oracle as O
from paper_2509_08675_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_08675_amd import hufield
    return hufield


def test_filter_spectrum_with_offset_matches_oracle(hf):
    dims, nr = (96, 64), 24
    filt = W.filt(p=4, semi=(2, 1, 1), rot=0.4, alpha=2, k0=0.2, width=0.05, offset=5e-3)
    s, c = hf.filter_spectrum(dims, filt, (nr, 1))
    torch.cuda.synchronize()
    T_ref, c_ref = O.target_bins(dims, O.FilterParams(**filt), nr)
    cnt = hf.u64_view(c)
    np.testing.assert_array_equal(cnt[:nr], c_ref.astype(np.uint64))
    got = s.cpu().numpy()[:nr] / np.maximum(cnt[:nr], 1)
    np.testing.assert_allclose(got[c_ref > 0], T_ref[c_ref > 0], rtol=1e-5)


def test_variant_argument_errors(hf):
    dims, bins = (32, 32), (8, 1)
    d = torch.zeros(9, dtype=torch.float64, device="cuda")
    c = torch.zeros(9, dtype=torch.int64, device="cuda")
    st = torch.zeros(4, dtype=torch.float64, device="cuda")
    with pytest.raises(hf.HuError) as e:
        hf.spectrum_grad(dims, W.filt(p=2, alpha=2, k0=0.2, width=0.05, offset=1e-3), 1, bins, d, d, c, st)
    assert e.value.code == hf.HU_ERR_UNSUPPORTED
    for bad in (dict(alpha=-2.0), dict(offset=-1e-3), dict(offset=float("inf"))):
        f = {**W.filt(p=2, alpha=2, k0=0.2, width=0.05), **bad}
        with pytest.raises(hf.HuError) as e:
            hf.gen_field(dims, f, [1])
        assert e.value.code == hf.HU_ERR_ARG
    with pytest.raises(hf.HuError) as e:                    # the offset is relative to a continuum peak
        hf.gen_field(dims, W.filt(p=2, alpha=-1.0, k0=0.2, width=0.05, offset=1e-3), [1])
    assert e.value.code == hf.HU_ERR_UNSUPPORTED


def test_negative_alpha_field_is_antihyperuniform(hf):
    dims, bins = (2048, 2048), (64, 1)
    filt = W.filt(p=2, alpha=-1.0, k0=0.0, width=2.0)
    out = hf.gen_field(dims, filt, [6], cont_bins=bins)
    a = hf.small_k_exponent(out["cont_sum"][0], hf.u64_view(out["cont_cnt"][0]), bins, 12)
    print("exponent", a, flush=True)
    assert abs(a + 1.0) < 0.15
    assert hf.hyperuniformity_class(a, 2) == "antihyperuniform"


def test_alpha_zero_field_is_standard_nonhyperuniform(hf):
    dims, bins = (2048, 2048), (64, 1)
    filt = W.filt(p=2, alpha=0.0, k0=0.0, width=2.0)
    out = hf.gen_field(dims, filt, [5], cont_bins=bins)
    a = hf.small_k_exponent(out["cont_sum"][0], hf.u64_view(out["cont_cnt"][0]), bins, 12)
    print("exponent", a, flush=True)
    assert abs(a) < 0.15
    assert hf.hyperuniformity_class(a, 2, tol=0.15) == "nonhyperuniform (standard)"


# ---------------------------------------------------------------------------------------------
# tabulated radial form (two bands), through the whole pipeline against the oracle
# ---------------------------------------------------------------------------------------------
def _two_band_profile(dk=0.005, kmax=2.0):
    K = dk * np.arange(int(kmax / dk) + 1)
    chi = np.exp(-(K - 0.15) ** 2 / (2 * 0.03 ** 2)) + 0.5 * np.exp(-(K - 0.45) ** 2 / (2 * 0.05 ** 2))
    return np.log(np.maximum(chi, 1e-30)).astype(np.float32), dk


@pytest.mark.parametrize("dims,rot,bins", [((96, 128), 0.5, (32, 6)), ((32, 24, 16), 0.3, (16, 1))])
def test_tabulated_radial_form_pipeline_matches_oracle(hf, dims, rot, bins):
    prof, dk = _two_band_profile()
    print("tabulated form", dims, flush=True)
    prof_dev = torch.from_numpy(prof).cuda()
    base = dict(p=3.0, semi=(1.0, 2.0, 1.5), rot=rot, sigma_f=1.0)
    gpu_filt = dict(base, prof=prof_dev, prof_dk=dk)
    ref_filt = O.FilterParams(p=3.0, semi=(1.0, 2.0, 1.5), rot=rot, prof=tuple(float(x) for x in prof), prof_dk=dk)
    seeds = [21, 22]
    bufs = hf.PipelineBuffers(dims, len(seeds), bins)
    hf.pipeline(bufs, gpu_filt, seeds)
    torch.cuda.synchronize()
    hf.check_degenerate(bufs.stats)
    for i, s in enumerate(seeds):
        ref = O.pipeline(dims, ref_filt, s, bins[0], bins[1])
        f = bufs.field[i].double().cpu().numpy()
        rms = float(np.sqrt(np.mean(ref["f"] ** 2)))
        err = float(np.max(np.abs(f - ref["f"]))) / rms
        assert err <= 1e-5, (dims, s, err)
        cs = bufs.cont_sum[i].cpu().numpy()
        np.testing.assert_allclose(cs, ref["cont_sum"], rtol=1e-4, atol=1e-7 * ref["cont_sum"].max())


def test_tabulated_radial_form_in_a_batch_equals_single_calls(hf):
    # a shape class mixing a tabulated form and Eq. (13): each field equals its own pipeline call
    prof, dk = _two_band_profile()
    prof_dev = torch.from_numpy(prof).cuda()
    tab = dict(p=3.0, semi=(1.0, 2.0, 1.0), rot=0.5, sigma_f=1.0, prof=prof_dev, prof_dk=dk)
    eq13 = W.filt(p=4, semi=(2, 1, 1), rot=0.2, alpha=4, k0=0.2, width=0.05)
    jobs = [dict(dims=(64, 96), filt=tab, seed=31, bins=(24, 6)), dict(dims=(64, 96), filt=eq13, seed=32, bins=(24, 6)),
            dict(dims=(16, 24, 32), filt=tab, seed=33, bins=(16, 1))]
    bb = hf.BatchBuffers(jobs)
    st = hf.pipeline_batch(bb)
    torch.cuda.synchronize()
    assert st == [0] * len(jobs)
    for i, j in enumerate(jobs):
        b = hf.PipelineBuffers(j["dims"], 1, j["bins"])
        hf.pipeline(b, j["filt"], [j["seed"]])
        torch.cuda.synchronize()
        assert torch.equal(bb.out[i]["field"], b.field[0]), i
        assert torch.equal(bb.out[i]["pm1"], b.pm1[0]), i


def test_filter_spectrum_with_tabulated_form_matches_oracle(hf):
    prof, dk = _two_band_profile()
    prof_dev = torch.from_numpy(prof).cuda()
    dims, nr = (128, 96), 32
    s, c = hf.filter_spectrum(dims, dict(p=2.5, semi=(1.0, 1.5, 1.0), rot=0.3, sigma_f=1.0, prof=prof_dev, prof_dk=dk),
                              (nr, 1))
    torch.cuda.synchronize()
    ref = O.FilterParams(p=2.5, semi=(1.0, 1.5, 1.0), rot=0.3, prof=tuple(float(x) for x in prof), prof_dk=dk)
    T_ref, c_ref = O.target_bins(dims, ref, nr)
    cnt = hf.u64_view(c)
    np.testing.assert_array_equal(cnt[:nr], c_ref.astype(np.uint64))
    got = s.cpu().numpy()[:nr] / np.maximum(cnt[:nr], 1)
    np.testing.assert_allclose(got[c_ref > 0], T_ref[c_ref > 0], rtol=1e-5)

"""GPU tests of the differentiation path: the expected (target) spectrum of a filter, the adjoint
of the binned continuous spectrum with respect to theta = (a, b, c, p, rot, k0, w), and the
spectrum-matching loss behind torch.autograd.

* hu_filter_spectrum against the oracle's target spectrum (bin means, counts exact);
* the loss and its gradient against the oracle's analytic gradient (noise recomputed from the
  seed on both sides), 2D and 3D, rotated and not; tolerance rtol 1e-4, norm-relative for
  components near zero;
* the gradient against the oracle's FP64 central differences (the independent check);
* the 512-point transform lengths of the 512^3 workload against the oracle's gradient: 512 on the
  axis-0 and y passes ((512, 512, 16)) and on the rows ((16, 32, 512)), with its filters;
* bit-reproducibility of the gradient;
* the full 512^3 case: directional derivatives of the GPU loss along three directions against
  the adjoint (a property that holds at any size).
"""

import math

import numpy as np
import pytest
import torch

import oracle as O
from oracle.loss import spectrum_loss_fd
from paper_2509_08675_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_08675_amd import hufield
    return hufield


def _say(*a):
    print(*a, flush=True)


def _theta(f):
    s = tuple(f["semi"]) + (1.0,) * 3
    return [s[0], s[1], s[2], f["p"], f["rot"], f["k0"], f["width"]]


def _grad_close(g, ref, rtol=1e-4):
    g, ref = np.asarray(g, float), np.asarray(ref, float)
    scale = np.linalg.norm(ref)
    err = np.abs(g - ref)
    assert np.all(err <= rtol * np.abs(ref) + rtol * scale), (g, ref, err / max(scale, 1e-300))


CASES = [
    # dims, field filter, target filter, radial bins
    ((24, 24, 24), W.filt(p=6, semi=(1, 2, 3), alpha=2, k0=0.15, width=0.03 * 4),
     W.filt(p=4, semi=(1, 1.5, 2), alpha=4, k0=0.15, width=0.03 * 4), 12),
    ((64, 96), W.filt(p=3, semi=(2, 1, 1), rot=0.4, alpha=2, k0=0.2, width=0.06),
     W.filt(p=2, semi=(1, 1, 1), rot=0.0, alpha=2, k0=0.25, width=0.05), 32),
    ((48, 32, 24), W.filt(p=2.5, semi=(1.5, 1, 2), rot=0.7, alpha=4, k0=0.1, width=0.08),
     W.filt(p=4, semi=(1, 1.5, 2), alpha=4, k0=0.15, width=0.06), 16),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_filter_spectrum_matches_oracle(hf, case):
    dims, _, target, nr = CASES[case]
    _say("filter_spectrum", dims)
    s, c = hf.filter_spectrum(dims, target, (nr, 1))
    torch.cuda.synchronize()
    T_ref, c_ref = O.target_bins(dims, O.FilterParams(**target), nr)
    cnt = hf.u64_view(c)
    np.testing.assert_array_equal(cnt[:nr], c_ref.astype(np.uint64))
    got = s.cpu().numpy()[:nr] / np.maximum(cnt[:nr], 1)
    np.testing.assert_allclose(got[c_ref > 0], T_ref[c_ref > 0], rtol=1e-5, atol=1e-9 * T_ref.max())


def test_filter_spectrum_angular_matches_oracle(hf):
    dims, filt, bins = (96, 64), W.filt(p=4, semi=(3, 1, 1), rot=0.5, alpha=4, k0=0.2, width=0.05), (16, 6)
    s, c = hf.filter_spectrum(dims, filt, bins)
    torch.cuda.synchronize()
    idx, w = O.bin_table(dims, *bins)
    H2 = O.amplitude_sym(dims, O.FilterParams(**filt)) ** 2
    N = math.prod(dims)
    E = N * H2 / np.sum(w * H2)
    nb = bins[0] * bins[1] + 1
    ref = np.bincount(idx.ravel(), weights=(w * E).ravel(), minlength=nb)
    cref = np.bincount(idx.ravel(), weights=w.ravel(), minlength=nb)
    np.testing.assert_array_equal(hf.u64_view(c), cref.astype(np.uint64))
    np.testing.assert_allclose(s.cpu().numpy(), ref, rtol=1e-5, atol=1e-9 * ref.max())


@pytest.mark.parametrize("dims,bins", [((96, 64), (16, 6)), ((512, 512), (128, 36)), ((128, 128, 128), (64, 1))])
def test_filter_spectrum_is_bit_reproducible(hf, dims, bins):
    """No floating-point atomics in the expected spectrum: repeated calls give the same bits (the
    2D 512^2 case spans many chunks per workgroup, the 128^3 one many workgroups per bin)."""
    filt = W.filt(p=3, semi=(2, 1, 1.5), rot=0.4, alpha=4, k0=0.2, width=0.05)
    runs = []
    for _ in range(3):
        s, c = hf.filter_spectrum(dims, filt, bins)
        torch.cuda.synchronize()
        runs.append((s.cpu().numpy().copy(), hf.u64_view(c).copy()))
    for s, c in runs[1:]:
        assert np.array_equal(s.view(np.uint64), runs[0][0].view(np.uint64))
        assert np.array_equal(c, runs[0][1])
    assert np.all(np.isfinite(runs[0][0])) and runs[0][0].sum() > 0


def _gpu_loss_grad(hf, dims, filt, seed, target, nr):
    theta = torch.tensor(_theta(filt), dtype=torch.float64, requires_grad=True)
    L = hf.spectrum_loss(theta, dims, seed, nr, target, filt["alpha"], filt.get("sigma_f", 1.0))
    L.backward()
    torch.cuda.synchronize()
    return float(L.detach().cpu()), theta.grad.numpy().copy()


@pytest.mark.parametrize("case", range(len(CASES)))
def test_loss_and_gradient_match_oracle(hf, case):
    dims, filt, target, nr = CASES[case]
    seed = 42 + case
    _say("adjoint", dims, "rot", filt["rot"])
    L, g = _gpu_loss_grad(hf, dims, filt, seed, target, nr)
    g_ref, L_ref, _ = O.spectrum_loss_grad(dims, O.FilterParams(**filt), seed, O.FilterParams(**target), nr)
    assert abs(L - L_ref) <= 1e-5 * abs(L_ref)
    if len(dims) == 2:
        assert g[2] == 0.0
    _grad_close(g, g_ref)


@pytest.mark.parametrize("rot", [0.0, 0.3])
def test_gradient_64cube_matches_oracle_and_fd(hf, rot):
    c5 = W.C5
    dims = c5["fd_dims"]
    filt = dict(c5["filt"], rot=rot)
    seed, target, nr = c5["seed"], c5["target"], c5["nr"] // 4
    _say("adjoint 64^3 rot", rot)
    L, g = _gpu_loss_grad(hf, dims, filt, seed, target, nr)
    fp, tp = O.FilterParams(**filt), O.FilterParams(**target)
    g_ref, L_ref, _ = O.spectrum_loss_grad(dims, fp, seed, tp, nr)
    assert abs(L - L_ref) <= 1e-5 * abs(L_ref)
    _grad_close(g, g_ref)
    g_fd = spectrum_loss_fd(dims, fp, seed, tp, nr)
    _grad_close(g, g_fd, rtol=2e-4)


@pytest.mark.parametrize("dims", [(512, 512, 16), (16, 32, 512)])
def test_gradient_512_point_axes_match_oracle(hf, dims):
    c5 = W.C5
    filt, seed, target, nr = c5["filt"], c5["seed"], c5["target"], 32
    _say("adjoint", dims)
    L, g = _gpu_loss_grad(hf, dims, filt, seed, target, nr)
    g_ref, L_ref, _ = O.spectrum_loss_grad(dims, O.FilterParams(**filt), seed, O.FilterParams(**target), nr)
    assert abs(L - L_ref) <= 1e-5 * abs(L_ref)
    _grad_close(g, g_ref)


def test_gradient_is_bit_reproducible(hf):
    dims, filt, target, nr = CASES[1]
    _, g1 = _gpu_loss_grad(hf, dims, filt, 7, target, nr)
    _, g2 = _gpu_loss_grad(hf, dims, filt, 7, target, nr)
    assert np.array_equal(g1, g2)


def test_spectrum_grad_argument_errors(hf):
    dims, bins = (32, 32), (8, 1)
    d = torch.zeros(9, dtype=torch.float64, device="cuda")
    c = torch.zeros(9, dtype=torch.int64, device="cuda")
    st = torch.zeros(4, dtype=torch.float64, device="cuda")
    with pytest.raises(hf.HuError) as e:
        hf.spectrum_grad(dims, W.filt(p=0.0, alpha=2, k0=0.2, width=0.05), 1, bins, d, d, c, st)
    assert e.value.code == hf.HU_ERR_ARG
    with pytest.raises(hf.HuError) as e:
        hf.spectrum_grad(dims, W.filt(p=2, alpha=2, k0=0.2, width=0.05), 1, bins, d, d, c, st,
                         work=torch.empty(256, dtype=torch.uint8, device="cuda"))
    assert e.value.code == hf.HU_ERR_WORKSPACE


@pytest.mark.slow
def test_full_size_512cube_directional_derivatives(hf):
    c5 = W.C5
    dims, filt, seed, target, nr = c5["dims"], c5["filt"], c5["seed"], c5["target"], c5["nr"]
    _say("adjoint 512^3")
    L0, g = _gpu_loss_grad(hf, dims, filt, seed, target, nr)
    assert np.all(np.isfinite(g)) and np.linalg.norm(g) > 0
    th0 = np.array(_theta(filt))
    rng = np.random.default_rng(5)
    dirs = [g / np.linalg.norm(g)] + [v / np.linalg.norm(v) for v in rng.standard_normal((2, 7))]
    h = 2e-3
    for u in dirs:
        vals = []
        for sgn in (1.0, -1.0):
            th = torch.tensor(th0 + sgn * h * u, dtype=torch.float64)
            with torch.no_grad():
                vals.append(float(hf.spectrum_loss(th, dims, seed, nr, target, filt["alpha"]).cpu()))
        fd = (vals[0] - vals[1]) / (2 * h)
        _say("  directional", fd, float(g @ u))
        assert abs(fd - g @ u) <= 2e-2 * np.linalg.norm(g)

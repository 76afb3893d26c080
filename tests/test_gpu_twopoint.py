"""GPU tests of the general level cut and the two-point probability function (through the C-ABI).

* hu_level_cut against the oracle's cut, bit-exact: both sides compare the FP32 field with the
  level rounded to FP32 (the decision is taken in the kernel's precision); counts exact;
* hu_two_point against the oracle's S_2 (Wiener-Khinchin in FP64) element by element on random and
  level-cut maps, 2D and 3D, power-of-two and 3 * 2^k sizes, several tiles with a ragged tail;
  tolerance 2e-6 absolute (S_2 lies in [0, 1]; FP32 transforms of |G|^2, whose DC term is up to N^2);
* identities on the GPU output: S_2(0) = phi, the mean over r is phi^2;
* a batch equals its maps one by one; full-size 2048^2 and 256^3 maps (sampled displacements).
"""

import numpy as np
import pytest
import torch

from oracle import twopoint as TP
import oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_08675_amd import hufield
    return hufield


def _say(*a):
    print(*a, flush=True)


def _random_map(dims, p, seed):
    rng = np.random.default_rng(seed)
    return np.where(rng.random(dims) < p, 1, -1).astype(np.int8)


@pytest.mark.parametrize("dims,phi", [((64, 64), 0.5), ((96, 48), 0.3), ((16, 16, 16), 0.7), ((24, 48, 32), 0.05)])
def test_level_cut_matches_oracle(hf, dims, phi):
    _say("level cut", dims, phi)
    filt = O.FilterParams(p=3, semi=(2, 1, 1), rot=0.2, alpha=2, k0=0.2, width=0.05)
    f = np.stack([O.gen_field(dims, filt, s)["f"] for s in (1, 2)]).astype(np.float32)
    g, c = hf.level_cut(torch.from_numpy(f).cuda(), phi, sigma_f=1.0, near_tol=1e-3)
    torch.cuda.synchronize()
    t32 = np.float32(TP.level_threshold(phi, 1.0))
    ref = TP.level_cut(f, t32)
    np.testing.assert_array_equal(g.cpu().numpy(), ref)
    cnt = hf.u64_view(c)
    for b in range(2):
        assert int(cnt[b, 0]) == int(np.count_nonzero(ref[b] == 1))
        assert int(cnt[b, 1]) == int(np.count_nonzero(np.abs(f[b] - t32) < np.float32(1e-3)))


@pytest.mark.parametrize("dims", [(8, 8), (64, 64), (96, 48), (48, 96), (256, 128), (16, 16, 16), (24, 16, 32),
                                  (12, 24, 48)])
def test_two_point_matches_oracle(hf, dims):
    _say("two point", dims)
    g = np.stack([_random_map(dims, p, 3 + i) for i, p in enumerate((0.5, 0.2))])
    s2 = hf.two_point(torch.from_numpy(g).cuda()).cpu().numpy()
    for b in range(2):
        ref = TP.s2_map(g[b])
        np.testing.assert_allclose(s2[b], ref, rtol=0, atol=2e-6)
        phi = float(np.mean(g[b] == 1))
        assert abs(float(s2[b].flat[0]) - phi) < 2e-6
        assert abs(float(s2[b].astype(np.float64).mean()) - phi * phi) < 2e-6


def test_two_point_of_a_level_cut_field(hf):
    dims = (128, 96)
    filt = O.FilterParams(p=4, semi=(3, 1, 1), rot=0.5, alpha=4, k0=0.2, width=0.04)
    f = O.gen_field(dims, filt, 7)["f"].astype(np.float32)[None]
    g, _ = hf.level_cut(torch.from_numpy(f).cuda(), 0.35, counts=False)
    s2 = hf.two_point(g).cpu().numpy()[0]
    np.testing.assert_allclose(s2, TP.s2_map(g.cpu().numpy()[0]), rtol=0, atol=2e-6)


def test_two_point_batch_equals_singles(hf):
    dims = (32, 64, 16)
    g = torch.from_numpy(np.stack([_random_map(dims, 0.4, 20 + i) for i in range(3)])).cuda()
    all3 = hf.two_point(g)
    for b in range(3):
        assert torch.equal(hf.two_point(g[b:b + 1].contiguous())[0], all3[b])


@pytest.mark.parametrize("dims", [(2048, 2048), (256, 256, 256)])
def test_two_point_full_size_sampled(hf, dims):
    _say("two point full size", dims)
    g = _random_map(dims, 0.45, 31)[None]
    s2 = hf.two_point(torch.from_numpy(g).cuda()).cpu().numpy()[0]
    I = (1.0 + g[0].astype(np.float64)) / 2.0
    rng = np.random.default_rng(1)
    for _ in range(6):
        r = tuple(int(rng.integers(0, n)) for n in dims)
        ref = float(np.mean(I * np.roll(I, shift=tuple(-k for k in r), axis=tuple(range(len(dims))))))
        assert abs(float(s2[r]) - ref) < 2e-6, (r, float(s2[r]), ref)
    phi = float(I.mean())
    assert abs(float(s2.flat[0]) - phi) < 2e-6


def test_two_point_batch_beyond_one_chunk(hf):
    # 70 maps: two chunks of the 64-field launch limit
    dims = (8, 16, 12)
    g = np.stack([_random_map(dims, 0.3 + 0.005 * i, 100 + i) for i in range(70)])
    s2 = hf.two_point(torch.from_numpy(g).cuda()).cpu().numpy()
    for b in (0, 63, 64, 69):
        np.testing.assert_allclose(s2[b], TP.s2_map(g[b]), rtol=0, atol=2e-6)

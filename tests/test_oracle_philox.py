"""Pins for the oracle's noise generator (Philox4x32-10, uniforms, Box-Muller).

* Philox words are compared with rocRAND's header-only Philox4x32-10 engine, an implementation
  written independently of this repository, built here as a host program;
* the uniforms are odd multiples of 2^-24, exactly representable in FP32;
* Box-Muller output is checked for N(0,1) moments and with a Kolmogorov-Smirnov test;
* the voxel layout (voxel i <- z_{i mod 4} of block i // 4) is checked voxel by voxel.
"""

import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND reference")
    exe = str(tmp_path_factory.mktemp("philox") / "philox_ref")
    src = os.path.join(HERE, "golden", "philox_rocrand_ref.cpp")
    # a host-only program: built as HIP so that the ROCm headers resolve, no kernels inside
    subprocess.run([hipcc, "-O1", "-x", "hip", "--offload-arch=gfx950", src, "-o", exe],
                   check=True, capture_output=True)
    return exe


def _ref_words(exe, seed, first, n):
    out = subprocess.run([exe, str(seed), str(first), str(n)], check=True, capture_output=True, text=True)
    return np.array([int(x, 16) for x in out.stdout.split()], dtype=np.uint32).reshape(n, 4).T


@pytest.mark.parametrize("seed,first,n", [
    (0, 0, 512), (1, 0, 256), (42, 1000, 256), (7, 0, 64),
    ((1 << 32) + 5, 12345, 128),                      # high key word in use
    (0xDEADBEEFCAFEF00D, (1 << 32) - 3, 16),           # counter crosses into its high word
])
def test_philox_matches_rocrand(rocrand_ref, seed, first, n):
    ref = _ref_words(rocrand_ref, seed, first, n)
    got = O.philox4x32_10(np.arange(first, first + n, dtype=np.uint64), seed)
    np.testing.assert_array_equal(got, ref)


def test_uniforms_exact_and_open_interval():
    words = np.array([0, 1, 511, 512, 0xFFFFFFFF, 0x80000000, 0x7FFFFE00], dtype=np.uint32)
    u = O.uniforms_from_words(words)
    assert np.all(u > 0) and np.all(u < 1)
    np.testing.assert_array_equal(u.astype(np.float32).astype(np.float64), u)
    assert u[0] == 2.0 ** -24 and u[4] == 1 - 2.0 ** -24
    k = u * 2 ** 24
    np.testing.assert_array_equal(k % 2, 1)


def test_box_muller_is_standard_normal():
    z = O.white_noise((1024, 1024), 3).ravel()
    n = z.size
    assert abs(z.mean()) < 5 / np.sqrt(n)
    assert abs(z.var() - 1) < 5 * np.sqrt(2 / n)
    assert abs(stats.kurtosis(z, fisher=False) - 3) < 5 * np.sqrt(24 / n)
    assert stats.kstest(z[:200000], "norm").pvalue > 1e-3
    # the four lanes of a block are mutually uncorrelated
    zz = z[: (n // 4) * 4].reshape(-1, 4)
    c = np.corrcoef(zz.T)
    assert np.max(np.abs(c - np.eye(4))) < 5 / np.sqrt(zz.shape[0])


def test_noise_voxel_layout():
    dims = (3, 5, 6)              # 90 voxels: last block is partial
    w = O.white_noise(dims, 11).ravel()
    for i in range(w.size):
        x = O.philox4x32_10(np.array([i // 4], dtype=np.uint64), 11)[:, 0]
        u = O.uniforms_from_words(x)
        pair = (u[0], u[1]) if (i % 4) < 2 else (u[2], u[3])
        r = np.sqrt(-2 * np.log(pair[0]))
        ang = 2 * np.pi * pair[1]
        want = r * np.cos(ang) if i % 2 == 0 else r * np.sin(ang)
        assert w[i] == want


def test_seeds_give_independent_streams():
    a = O.white_noise((64, 64), 1).ravel()
    b = O.white_noise((64, 64), 2).ravel()
    assert abs(np.corrcoef(a, b)[0, 1]) < 5 / 64

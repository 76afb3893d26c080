"""Seeded white noise: Philox4x32-10 counter RNG, 23-bit uniforms, Box-Muller.

The paper draws i.i.d. Gaussian white noise and takes its forward FFT
(Sec. II.B, Eq. (8) and the pipeline summary after Eq. (15)); it names no
generator.  The generator adopted here is Philox4x32 with 10 rounds from
J. K. Salmon, M. A. Moraes, R. O. Dror and D. E. Shaw, "Parallel random numbers:
as easy as 1, 2, 3", SC'11 (Sec. 4 there: the Philox S-box, multipliers and
Weyl key schedule).

Stream layout (a reading, the paper being silent):
* key = (seed mod 2^32, seed >> 32); block j uses counter (j mod 2^32, j >> 32, 0, 0);
* each block gives four words x0..x3; word x gives the uniform
  u = (2*(x >> 9) + 1) * 2^-24, an odd multiple of 2^-24 in (0, 1) that is exact
  in both FP32 and FP64;
* Box-Muller on (u0, u1) and on (u2, u3) gives four N(0,1) values z0..z3;
* voxel i (row-major linear index, last axis fastest) takes z_{i mod 4} of block i // 4.
"""

import numpy as np

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = 0x9E3779B9
_W1 = 0xBB67AE85
_LO = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def philox4x32_10(block_index, seed):
    """Philox4x32-10 words for the blocks ``block_index`` under ``seed``.

    Returns a (4, n) uint32 array (x0, x1, x2, x3 per block).  Each of the ten
    rounds multiplies words 0 and 2 by the two Philox multipliers, swaps the
    high/low halves into the four lanes and XORs the high halves with the
    other two words and the round key; the key is bumped by the two Weyl
    constants between rounds (Salmon et al. SC'11, Sec. 4).
    """
    j = np.asarray(block_index, dtype=np.uint64).ravel()
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    c0 = j & _LO
    c1 = j >> _S32
    c2 = np.zeros_like(j)
    c3 = np.zeros_like(j)
    k0 = seed & 0xFFFFFFFF
    k1 = seed >> 32
    for _ in range(10):
        p0 = _M0 * c0          # < 2^64: exact in uint64
        p1 = _M1 * c2
        c0, c1, c2, c3 = ((p1 >> _S32) ^ c1 ^ np.uint64(k0), p1 & _LO,
                          (p0 >> _S32) ^ c3 ^ np.uint64(k1), p0 & _LO)
        k0 = (k0 + _W0) & 0xFFFFFFFF
        k1 = (k1 + _W1) & 0xFFFFFFFF
    return np.stack([c0, c1, c2, c3]).astype(np.uint32)


def uniforms_from_words(words):
    """u = (2*(x >> 9) + 1) / 2^24 in FP64 (exactly representable in FP32 too)."""
    x = np.asarray(words, dtype=np.uint64)
    return ((x >> np.uint64(9)) * np.uint64(2) + np.uint64(1)).astype(np.float64) * 2.0 ** -24


def box_muller(u0, u1):
    """Box-Muller pair: sqrt(-2 ln u0) * (cos 2 pi u1, sin 2 pi u1), in FP64."""
    r = np.sqrt(-2.0 * np.log(u0))
    a = 2.0 * np.pi * u1
    return r * np.cos(a), r * np.sin(a)


def white_noise(dims, seed):
    """i.i.d. N(0,1) real white noise on the grid ``dims`` (row-major, last axis fastest)."""
    dims = tuple(int(n) for n in dims)
    n = int(np.prod(dims))
    nblk = (n + 3) // 4
    u = uniforms_from_words(philox4x32_10(np.arange(nblk, dtype=np.uint64), seed))
    z0, z1 = box_muller(u[0], u[1])
    z2, z3 = box_muller(u[2], u[3])
    z = np.stack([z0, z1, z2, z3], axis=1).reshape(-1)[:n]
    return z.reshape(dims)

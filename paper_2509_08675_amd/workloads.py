"""Seeded synthetic workloads: grid shapes, filter parameters, seeds and bin layouts.

This module holds no arithmetic of the method.  It only names the workloads and draws
their parameters, and it serves both the GPU path and the CPU oracle in tests and in the
benchmark.  Filter parameters are plain dicts with the keys
p, semi (a, b, c), rot, alpha, k0, width, sigma_f.

The paper runs 1024^2 grids (L = 100) and 256^3 grids (L = 25) with sigma = 2.0 in
physical units (Sec. III.A, Sec. III.B).  The workloads below are stated directly in
Nyquist units; ``paper_preset`` converts the paper's physical parameters.
"""

import math

import numpy as np


def filt(p, semi=(1.0, 1.0, 1.0), rot=0.0, alpha=2.0, k0=0.0, width=0.1, sigma_f=1.0, offset=0.0):
    semi = tuple(float(s) for s in semi) + (1.0,) * (3 - len(semi))
    return dict(p=float(p), semi=semi, rot=float(rot), alpha=float(alpha), k0=float(k0),
                width=float(width), sigma_f=float(sigma_f), offset=float(offset))


# 2D 128^2, one field, isotropic circle, alpha = 2, band at 0.25 k_Nyq, width 0.05; 64 radial bins.
C1 = dict(name="2d_128x128_x1", dims=(128, 128), seeds=[0],
          filt=filt(p=2, semi=(1, 1), rot=0.0, alpha=2, k0=0.25, width=0.05), bins=(64, 1))

# 2D 2048^2, 16 fields, p = 4, semi-axes 3:1, rotated 30 degrees, alpha = 4; 128 x 36 bins.
C2 = dict(name="2d_2048x2048_x16", dims=(2048, 2048), seeds=list(range(1, 17)),
          filt=filt(p=4, semi=(3, 1), rot=math.pi / 6, alpha=4, k0=0.2, width=0.04), bins=(128, 36))

# 3D 256^3, 4 fields, superellipsoid p = 6, semi-axes 1:2:3, alpha = 2; 128 radial bins.
C3 = dict(name="3d_256x256x256_x4", dims=(256, 256, 256), seeds=[1, 2, 3, 4],
          filt=filt(p=6, semi=(1, 2, 3), rot=0.0, alpha=2, k0=0.15, width=0.03), bins=(128, 1))

# 3D 512^3 field plus its spectrum-matching adjoint; the target uses perturbed parameters.
C5 = dict(name="3d_512x512x512_adjoint", dims=(512, 512, 512), seed=42,
          filt=filt(p=6, semi=(1, 2, 3), rot=0.0, alpha=2, k0=0.15, width=0.03),
          target=filt(p=4, semi=(1, 1.5, 2), rot=0.0, alpha=4, k0=0.15, width=0.03),
          nr=128, fd_dims=(64, 64, 64))


def c4_jobs(seed=7, n2d=448, n3d=64):
    """Uneven batch: 448 2D fields with sides from {64..1024} and 64 3D fields from {64, 96, 128},
    parameters drawn per field from numpy's PCG64 stream seeded with ``seed``:
    p in [1.5, 8], axis ratio r in [1, 4] (semi = (r, 1, 1)), rot in [0, pi), alpha in {2, 4, 6},
    band centre k0 in [0.1, 0.3], width 0.2 k0; noise seed 1000 + i; 64 radial bins."""
    rng = np.random.default_rng(seed)
    jobs = []
    for i in range(n2d + n3d):
        if i < n2d:
            side = int(rng.choice([64, 128, 256, 512, 1024]))
            dims = (side, side)
        else:
            side = int(rng.choice([64, 96, 128]))
            dims = (side, side, side)
        p = float(rng.uniform(1.5, 8.0))
        r = float(rng.uniform(1.0, 4.0))
        rot = float(rng.uniform(0.0, math.pi))
        alpha = float(rng.choice([2.0, 4.0, 6.0]))
        k0 = float(rng.uniform(0.1, 0.3))
        jobs.append(dict(dims=dims, seed=1000 + i, bins=(64, 1),
                         filt=filt(p=p, semi=(r, 1.0, 1.0), rot=rot, alpha=alpha, k0=k0, width=0.2 * k0)))
    return jobs


def paper_preset(n, L, sigma=2.0, alpha=20.0, p=1.0, semi=(1.0, 1.0, 1.0)):
    """The paper's physical parameters in Nyquist units: dx = L / n, k_Nyq = pi / dx, so the band
    width sigma (physical wavenumber) becomes sigma dx / pi and the band centre is 0."""
    dx = L / n
    return filt(p=p, semi=semi, rot=0.0, alpha=alpha, k0=0.0, width=sigma * dx / math.pi)


def random_field(dims, seed, dtype=np.float32):
    """N(0,1) test input for the standalone threshold and spectrum calls."""
    return np.random.default_rng(seed).standard_normal(size=tuple(dims)).astype(dtype)


def random_pm1(dims, seed):
    """+-1 int8 test input for the standalone spectrum call."""
    g = np.random.default_rng(seed).integers(0, 2, size=tuple(dims), dtype=np.int8)
    return (2 * g - 1).astype(np.int8)

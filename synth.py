"""Seeded synthetic inputs for the five workloads of this project.

This module holds no part of the persistence computation: it only draws
float32 images and volumes from NumPy's PCG64 generator.  Both the GPU path and
the CPU oracle consume its arrays.

Recipes (all arithmetic in float64, cast to float32 at the end, -0.0 -> +0.0):

* ``uniform2d(shape, seed)``: i.i.d. U[0,1) pixels (``rng.random`` in float32).
* ``grf(shape, sigma, rng)``: a Gaussian random field.  i.i.d. N(0,1) noise is
  drawn on the grid padded by r = ceil(4 sigma) on every side, filtered along
  each axis by the normalised 1D Gaussian kernel (taps -r..r, 'valid' part, no
  periodic wrap), and divided by ||k||_2^ndim so every pixel is N(0,1).
* ``blobs3d(n, seed)``: the sum of 200 Gaussian blobs in an n^3 box (centres
  U[0,n)^3, sigma U[3,12] voxels, amplitude U[-1,1]) plus U[-0.05,0.05) noise,
  drawn in that order from one generator.
* ``batch2d(n_images, seed)``: side lengths (H_i, W_i) drawn with
  ``rng.integers(28, 513)``; image i uses its own stream from
  ``SeedSequence(seed).spawn(n_images)``; even i: U[0,1) noise, odd i: GRF with
  sigma = 2.
* ``batch3d_grf(n_volumes, side, sigma, seed)``: GRF volumes, one spawned stream
  per volume.
* ``random_walk(n, seed)``: a 1D time series, the running sum of n i.i.d.
  N(0,1) steps.
* ``ball_mask(shape, hole)``: True inside the ball inscribed in the grid and
  outside the concentric ball of radius ``hole`` times the first; a masked
  input takes +inf where it is False (pixels outside the domain).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.ndimage import correlate1d


def _finish(a: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float32)
    a[a == 0] = 0.0  # -0.0 -> +0.0
    return a


def uniform2d(shape, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return _finish(rng.random(tuple(shape), dtype=np.float32))


def grf(shape, sigma: float, rng: np.random.Generator) -> np.ndarray:
    shape = tuple(int(s) for s in shape)
    r = int(math.ceil(4.0 * sigma))
    t = np.arange(-r, r + 1, dtype=np.float64)
    k = np.exp(-0.5 * (t / sigma) ** 2)
    k /= k.sum()
    a = rng.standard_normal(tuple(s + 2 * r for s in shape))
    for ax in range(len(shape)):
        a = correlate1d(a, k, axis=ax, mode="constant")
        sl = [slice(None)] * len(shape)
        sl[ax] = slice(r, r + shape[ax])
        a = a[tuple(sl)]
    a = a / (np.sqrt((k * k).sum()) ** len(shape))
    return _finish(a)


def grf_seeded(shape, sigma: float, seed: int) -> np.ndarray:
    return grf(shape, sigma, np.random.default_rng(seed))


def blobs3d(n: int = 256, seed: int = 2, n_blobs: int = 200, noise: float = 0.05) -> np.ndarray:
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.0, n, size=(n_blobs, 3))
    sigmas = rng.uniform(3.0, 12.0, size=n_blobs)
    amps = rng.uniform(-1.0, 1.0, size=n_blobs)
    t = np.arange(n, dtype=np.float64)
    g = [np.exp(-0.5 * ((t[None, :] - centres[:, a][:, None]) / sigmas[:, None]) ** 2)
         for a in range(3)]  # each (n_blobs, n)
    # sum_b amp_b * gz_b (x) gy_b (x) gx_b as one matrix product
    yx = (g[1][:, :, None] * g[2][:, None, :]).reshape(n_blobs, n * n)
    vol = ((g[0] * amps[:, None]).T @ yx).reshape(n, n, n)
    vol += rng.uniform(-noise, noise, size=(n, n, n))
    return _finish(vol)


def batch2d(n_images: int = 512, seed: int = 3, lo: int = 28, hi: int = 512):
    rng = np.random.default_rng(seed)
    sides = rng.integers(lo, hi + 1, size=(n_images, 2))
    streams = np.random.SeedSequence(seed).spawn(n_images)
    out = []
    for i in range(n_images):
        r = np.random.default_rng(streams[i])
        shp = (int(sides[i, 0]), int(sides[i, 1]))
        if i % 2 == 0:
            out.append(_finish(r.random(shp, dtype=np.float32)))
        else:
            out.append(grf(shp, 2.0, r))
    return out


def batch3d_grf(n_volumes: int = 32, side: int = 128, sigma: float = 3.0, seed: int = 4):
    streams = np.random.SeedSequence(seed).spawn(n_volumes)
    return [grf((side,) * 3, sigma, np.random.default_rng(s)) for s in streams]


def random_walk(n: int, seed: int = 7) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return _finish(np.cumsum(rng.standard_normal(n)))


def ball_mask(shape, hole: float = 0.0) -> np.ndarray:
    grids = np.indices(tuple(shape), dtype=np.float64)
    c = [(s - 1) / 2 for s in shape]
    r2 = sum((g - ci) ** 2 for g, ci in zip(grids, c))
    rmax = (min(shape) - 1) / 2
    return (r2 <= rmax ** 2) & (r2 >= (hole * rmax) ** 2)


def config(name: str, small: bool = False):
    """The named workload.  ``small`` shrinks it for quick checks (same recipe)."""
    if name == "C1":
        return uniform2d((64, 64), 0)
    if name == "C2":
        return grf_seeded((256, 256) if small else (1024, 1024), 4.0, 1)
    if name == "C3":
        return blobs3d(48 if small else 256, 2)
    if name == "C4":
        return batch2d(16 if small else 512, 3, 28, 96 if small else 512)
    if name == "C5":
        return batch3d_grf(4 if small else 32, 24 if small else 128, 3.0, 4)
    raise KeyError(name)

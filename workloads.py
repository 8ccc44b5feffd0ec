"""Seeded synthetic inputs for the FCC cosine transform workloads.

This module holds random-number recipes only: no arithmetic of the transform.
It serves both the tests (oracle side) and the benchmark (GPU side).  Every
generator is numpy PCG64 (``default_rng(seed)``), drawn in the order written.
Input index k = (a,b,c) in [0,n)^3 is flattened lexicographically and sits at
the unit-cube position p = k/n (k*15/(n-1) for the upsampled field).
"""
import numpy as np

SIZES_RAGGED = (8, 16, 32, 64, 128)


def uniform_fp64(n=4, seed=0):
    """n^3 i.i.d. uniform[-1,1] values in FP64 (the n=4 round-trip case)."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, n ** 3)


def gaussian_field(n=64, seed=1, count=16):
    """Sum of `count` unit-amplitude 3-D Gaussians plus N(0, 0.01) noise (FP32).

    Centres uniform in [0,1)^3, widths uniform[0.05, 0.2] of the domain; the
    noise variance is 0.01 (standard deviation 0.1)."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.0, 1.0, (count, 3))
    widths = rng.uniform(0.05, 0.2, count)
    noise = rng.normal(0.0, 0.1, n ** 3)
    ax = np.arange(n) / n
    p = np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), -1).reshape(-1, 3)
    field = np.zeros(n ** 3)
    for c, w in zip(centres, widths):
        field += np.exp(-np.sum((p - c) ** 2, axis=1) / (2.0 * w * w))
    return (field + noise).astype(np.float32)


def quantised_blocks(count=4096, n=8, seed=2):
    """`count` independent n^3 blocks of 8-bit levels / 255 (FP32), shape (count, n^3)."""
    rng = np.random.default_rng(seed)
    return (rng.integers(0, 256, (count, n ** 3)) / 255.0).astype(np.float32)


def upsampled_field(n=256, seed=3, coarse=16):
    """Trilinear (align-corners) upsampling of a coarse^3 uniform[-1,1] grid to n^3 (FP32)."""
    g = np.random.default_rng(seed).uniform(-1.0, 1.0, (coarse, coarse, coarse))
    t = np.arange(n) * (coarse - 1) / max(n - 1, 1)
    i0 = np.minimum(np.floor(t).astype(np.int64), coarse - 2)
    f = t - i0
    # separable linear interpolation, axis by axis
    a = g[i0] * (1 - f)[:, None, None] + g[i0 + 1] * f[:, None, None]
    a = a[:, i0] * (1 - f)[None, :, None] + a[:, i0 + 1] * f[None, :, None]
    a = a[:, :, i0] * (1 - f)[None, None, :] + a[:, :, i0 + 1] * f[None, None, :]
    return a.astype(np.float32).reshape(-1)


def ragged_sizes(count=512, seed=4, sizes=SIZES_RAGGED):
    """The size list of the ragged batch: n_b drawn uniformly from `sizes`."""
    return [int(v) for v in np.random.default_rng(seed).choice(np.array(sizes), count)]


def ragged_batch(count=512, seed=4, sizes=SIZES_RAGGED, limit=None):
    """Ragged batch: sizes as in `ragged_sizes`, then each volume i.i.d. N(0,1) FP32,
    drawn in order from the same generator.  `limit` truncates the list (tests)."""
    rng = np.random.default_rng(seed)
    ns = [int(v) for v in rng.choice(np.array(sizes), count)]
    if limit is not None:
        ns = ns[:limit]
    return ns, [rng.standard_normal(m ** 3).astype(np.float32) for m in ns]

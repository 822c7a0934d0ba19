"""Seeded synthetic inputs: smoothed Gaussian random fields and the workload mixes.

This module holds no part of the EC computation: it only draws the fields that
both the HIP path and the test oracle are given.  The paper's own benchmark
inputs are white-noise fields translated to integers 0..255 (Computational
Results section); its real data sets are not available, so smoothed Gaussian
random fields of the sizes below stand in for them.

Recipe (every field):
  1. z = standard normal, float64, numpy PCG64 seeded per field;
  2. periodic Gaussian smoothing in Fourier space: multiply the real FFT by
     exp(-2 pi^2 sigma^2 |k|^2), k in cycles per cell;
  3. standardise to zero mean and unit variance;
  4. integer fields: q = min(floor((z - zmin) / (zmax - zmin) * Q), Q - 1),
     Q = 256 for uint8 and 4096 for uint16 (the paper translates every input
     to 0..255 levels).
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass, field as dc_field

import numpy as np

_WORKERS = max(1, min(16, os.cpu_count() or 1))

try:  # scipy's FFT can use several threads
    import scipy.fft as _fft

    def _rfftn(a):
        return _fft.rfftn(a, workers=_WORKERS)

    def _irfftn(a, s):
        return _fft.irfftn(a, s=s, workers=_WORKERS)
except ImportError:  # pragma: no cover
    def _rfftn(a):
        return np.fft.rfftn(a)

    def _irfftn(a, s):
        return np.fft.irfftn(a, s=s)


def grf(shape, sigma: float, seed, out_dtype=np.float32) -> np.ndarray:
    """Standardised, periodically smoothed Gaussian random field."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal(tuple(int(s) for s in shape))
    spec = _rfftn(z)
    del z
    gain = None
    for ax, n in enumerate(shape):
        k = np.fft.rfftfreq(n) if ax == len(shape) - 1 else np.fft.fftfreq(n)
        g = np.exp(-2.0 * math.pi ** 2 * sigma ** 2 * k ** 2)
        sh = [1] * len(shape)
        sh[ax] = g.size
        g = g.reshape(sh)
        gain = g if gain is None else gain * g
    spec *= gain
    z = _irfftn(spec, s=tuple(int(s) for s in shape))
    del spec
    z -= z.mean()
    sd = z.std()
    if sd > 0:
        z /= sd
    return z.astype(out_dtype, copy=False)


def quantise(z: np.ndarray, q_levels: int) -> np.ndarray:
    zmin, zmax = float(z.min()), float(z.max())
    span = zmax - zmin if zmax > zmin else 1.0
    q = np.floor((z.astype(np.float64) - zmin) / span * q_levels)
    q = np.minimum(q, q_levels - 1)
    return q.astype(np.uint8 if q_levels <= 256 else np.uint16)


def white_noise(shape, seed, q_levels=256, kind="uniform") -> np.ndarray:
    """The paper's own synthetic inputs: i.i.d. uniform or normal noise on 0..Q-1."""
    rng = np.random.default_rng(seed)
    if kind == "uniform":
        return rng.integers(0, q_levels, size=shape).astype(np.uint8 if q_levels <= 256 else np.uint16)
    return quantise(rng.standard_normal(shape), q_levels)


# The paper's own benchmark inputs (Computational Results, Tables 3 and 4):
# white noise translated to 0..255 at these shapes, all 256 levels, 8-C in 2D
# and 26-C in 3D.  (name, shape, noise, the paper's 24-core CPU figure in
# Mcells/s, its table); field k is white_noise(shape, 500 + k, 256, noise).
PAPER_WORKLOADS = [
    ("2d_1280x720_u8_uniform", (720, 1280), "uniform", 97.7, "Table 3"),
    ("2d_1280x720_u8_normal", (720, 1280), "normal", 99.3, "Table 3"),
    ("2d_1920x1080_u8_uniform", (1080, 1920), "uniform", 107.4, "Table 3"),
    ("2d_1920x1080_u8_normal", (1080, 1920), "normal", 110.8, "Table 3"),
    ("2d_2048x2048_u8_uniform", (2048, 2048), "uniform", 96.5, "Table 3"),
    ("2d_2048x2048_u8_normal", (2048, 2048), "normal", 110.4, "Table 3"),
    ("2d_4096x4096_u8_uniform", (4096, 4096), "uniform", 82.2, "Table 3"),
    ("2d_4096x4096_u8_normal", (4096, 4096), "normal", 81.95, "Table 3"),
    ("3d_128^3_u8_uniform", (128, 128, 128), "uniform", 26.67, "Table 4"),
    ("3d_128^3_u8_normal", (128, 128, 128), "normal", 27.47, "Table 4"),
    ("3d_256^3_u8_uniform", (256, 256, 256), "uniform", 27.90, "Table 4"),
    ("3d_256^3_u8_normal", (256, 256, 256), "normal", 28.38, "Table 4"),
]


def paper_workload(k: int) -> np.ndarray:
    """Field k of PAPER_WORKLOADS."""
    _, shape, kind, _, _ = PAPER_WORKLOADS[k]
    return white_noise(shape, 500 + k, 256, kind)


# ----------------------------------------------------------------------------
# the five workloads
# ----------------------------------------------------------------------------
def linspace_thresholds(lo: float, hi: float, n: int) -> np.ndarray:
    """n uniformly spaced thresholds, computed in float64 and rounded to float32."""
    return np.linspace(lo, hi, n).astype(np.float32)


@dataclass
class FieldSpec:
    """One field of a workload: the array plus its filtration."""
    data: np.ndarray
    n_levels: int
    thresholds: np.ndarray | None = None
    connectivity: int | None = None
    meta: dict = dc_field(default_factory=dict)


def small_2d_u8() -> FieldSpec:
    """256 x 256 uint8, sigma 4 px, all 256 levels (seed 1)."""
    return FieldSpec(quantise(grf((256, 256), 4.0, 1), 256), 256, None, 8,
                     dict(name="2d_256x256_u8_sigma4"))


def large_2d_f32(side: int = 8192) -> FieldSpec:
    """8192 x 8192 float32, sigma 16 px, 1024 thresholds on [-4, 4] (seed 2)."""
    return FieldSpec(grf((side, side), 16.0, 2), 1024, linspace_thresholds(-4.0, 4.0, 1024), 8,
                     dict(name=f"2d_{side}x{side}_f32_sigma16_L1024"))


def large_3d_u16(side: int = 512) -> FieldSpec:
    """512^3 uint16 (4096 levels), sigma 6 voxels, all 4096 levels (seed 3)."""
    return FieldSpec(quantise(grf((side, side, side), 6.0, 3), 4096), 4096, None, 26,
                     dict(name=f"3d_{side}^3_u16_sigma6_L4096"))


def batch_shapes(n: int = 4096, seed: int = 4, lo: int = 64, hi: int = 2048, max_aspect: float = 4.0):
    """Side lengths log-uniform in [lo, hi], aspect ratio at most max_aspect."""
    rng = np.random.default_rng(seed)
    shapes = []
    while len(shapes) < n:
        h, w = np.exp(rng.uniform(math.log(lo), math.log(hi), size=2))
        h, w = int(round(h)), int(round(w))
        if max(h, w) > max_aspect * min(h, w):
            continue
        shapes.append((h, w))
    return shapes


def _quantised_grf(args):
    shape, sigma, seed, q = args
    return quantise(grf(shape, sigma, seed), q)


def _single_threaded_fft():
    """Worker initializer: the FFT runs in the calling thread (a forked child
    does not inherit the parent's FFT thread pool)."""
    global _WORKERS
    _WORKERS = 1


def _map(fn, args, workers: int):
    """fn over args, in `workers` forked processes when workers > 1 (the
    results do not depend on the worker count: every field has its own seed).
    Forked workers leave no helper process behind (the spawn start method
    keeps a resource tracker alive until the parent exits); callers draw their
    inputs before the process touches the GPU."""
    if workers <= 1 or len(args) < 2:
        return [fn(a) for a in args]
    import concurrent.futures as cf
    import multiprocessing as mp
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("fork"),
                                initializer=_single_threaded_fft) as ex:
        return list(ex.map(fn, args, chunksize=max(1, len(args) // (8 * workers))))


def batch_2d_u8(n: int = 4096, seed: int = 4, lo: int = 64, hi: int = 2048, workers: int = 1):
    """n uint8 smoothed GRFs of uneven shape, sigma ~ U[2, 16] px, 256 levels."""
    shapes = batch_shapes(n, seed, lo, hi)
    ss = np.random.SeedSequence(seed).spawn(n)
    rng = np.random.default_rng(seed + 1000)
    sigmas = rng.uniform(2.0, 16.0, size=n)
    data = _map(_quantised_grf, [(sh, float(s), ss[k], 256) for k, (sh, s) in enumerate(zip(shapes, sigmas))],
                workers)
    return [FieldSpec(a, 256, None, 8, dict(name=f"batch{k}", sigma=float(s)))
            for k, (a, s) in enumerate(zip(data, sigmas))]


def batch_3d_grids(n: int = 4096, side: int = 20, seed: int = 6, workers: int = 1):
    """n uint8 volumes of side^3 voxels (smoothed GRFs, sigma ~ U[1, 3] voxels,
    256 levels, 26-C): a stand-in for the paper's molecular-dynamics case, many
    20 x 20 x 20 density grids translated to 0..255."""
    ss = np.random.SeedSequence(seed).spawn(n)
    rng = np.random.default_rng(seed + 1000)
    sigmas = rng.uniform(1.0, 3.0, size=n)
    data = _map(_quantised_grf, [((side, side, side), float(s), ss[k], 256) for k, s in enumerate(sigmas)],
                workers)
    return [FieldSpec(a, 256, None, 26, dict(name=f"grid{k}", sigma=float(s)))
            for k, (a, s) in enumerate(zip(data, sigmas))]


def field_4d(shape=(32, 96, 96, 96), seed: int = 7) -> FieldSpec:
    """A 4D uint8 field (a smoothed GRF, sigma 3 cells, 256 levels, 80-C): a
    stand-in for 4D data such as a time series of volumes."""
    return FieldSpec(quantise(grf(shape, 3.0, seed), 256), 256, None, 80,
                     dict(name="4d_" + "x".join(str(s) for s in shape) + "_u8_sigma3_L256"))


def serving_pool(n2d: int = 64, n3d: int = 32, seed: int = 5, max2d: int = 4096, max3d: int = 384,
                 workers: int = 1):
    """Pool of request fields: 2D uint8 (side log-uniform in [128, max2d], 256
    levels) and 3D uint16 (side log-uniform in [64, max3d], 256/1024/4096
    levels); requests replay fields of this pool by id."""
    rng = np.random.default_rng(seed)
    ss = np.random.SeedSequence(seed).spawn(n2d + n3d)
    jobs, meta = [], []
    for k in range(n2d):
        h, w = (int(round(x)) for x in np.exp(rng.uniform(math.log(128), math.log(max2d), size=2)))
        s = float(rng.uniform(2.0, 16.0))
        jobs.append(((h, w), s, ss[k], 256))
        meta.append((256, 8, dict(name=f"pool2d{k}", sigma=s)))
    for k in range(n3d):
        d, h, w = (int(round(x)) for x in np.exp(rng.uniform(math.log(64), math.log(max3d), size=3)))
        s = float(rng.uniform(3.0, 8.0))
        L = int(rng.choice([256, 1024, 4096]))
        jobs.append(((d, h, w), s, ss[n2d + k], 4096))
        meta.append((L, 26, dict(name=f"pool3d{k}", sigma=s)))
    data = _map(_quantised_grf, jobs, workers)
    pool = []
    for q, (L, conn, m) in zip(data, meta):
        if q.ndim == 3 and L < 4096:  # rescale to L levels
            q = (q.astype(np.uint32) * L // 4096).astype(np.uint16)
        pool.append(FieldSpec(q, L, None, conn, m))
    return pool


def poisson_trace(n_requests: int, rate_hz: float, pool_size: int, frac_2d: float, n2d: int,
                  seed: int = 5):
    """Arrival times (s) and pool ids: 70 % 2D / 30 % 3D by default mix."""
    rng = np.random.default_rng(seed + 77)
    gaps = rng.exponential(1.0 / rate_hz, size=n_requests)
    t = np.cumsum(gaps)
    is2d = rng.random(n_requests) < frac_2d
    ids = np.where(is2d, rng.integers(0, n2d, size=n_requests),
                   n2d + rng.integers(0, pool_size - n2d, size=n_requests))
    return t, ids

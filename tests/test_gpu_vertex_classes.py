"""GPU parity of the vertex class counts (contribution map), through the C ABI.

* Counts equal the oracle's (oracle.vertex_classes_2d) bit for bit: the
  degenerate shapes, ragged tails over several strips, every level mode
  (identity integer levels, integer levels through thresholds, affine float
  thresholds, irregular thresholds with ties and NaN), level counts above the
  per-pass window, a field whose base address is not 16-byte aligned.
* On a large field the counts, weighted by Table 1, give the same EC (8-C and
  4-C), perimeter and area curves as ecc_curves_compute.
* 3D: the 21 octant classes equal the oracle's on degenerate shapes, ragged
  tiles, more levels than one pass holds, float thresholds with NaN, and a
  smooth volume.
"""
from __future__ import annotations

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2311_11740_amd import ecc
    c = ecc.Context(0)
    yield c
    c.close()


def compare(ctx, arr, L, thr=None, tag="", offset=0):
    import torch
    import oracle
    print(f"[case] classes {tag} shape={arr.shape} dtype={arr.dtype} L={L} "
          f"thr={'none' if thr is None else 'yes'} offset={offset}", flush=True)
    flat = torch.from_numpy(np.concatenate([np.zeros(offset, arr.dtype), np.ascontiguousarray(arr).ravel()])).cuda()
    dev = flat[offset:].view(*arr.shape)
    got = ctx.vertex_classes(dev, L, thresholds=thr)
    torch.cuda.synchronize()
    ref = oracle.class_counts(arr, L, thr)
    g = got.cpu().numpy()
    if not np.array_equal(g, ref):
        c, lvl = (int(x[0]) for x in np.nonzero(g != ref))
        raise AssertionError(f"{tag}: class {c} level {lvl}: gpu {g[c, lvl]} oracle {ref[c, lvl]}")


SHAPES = [(1, 1), (1, 300), (300, 1), (37, 513), (257, 1025), (1021, 769)]


@pytest.mark.parametrize("shape", SHAPES)
def test_classes_u8_identity(ctx, shape):
    rng = np.random.default_rng(hash(shape) % (1 << 30))
    compare(ctx, rng.integers(0, 256, size=shape).astype(np.uint8), 256, tag="u8")


@pytest.mark.parametrize("shape", [(1, 1), (37, 513), (301, 700)])
def test_classes_f32_affine(ctx, shape):
    from paper_2311_11740_amd import synth
    z = synth.grf(shape, 3.0, 11 + shape[0])
    compare(ctx, z, 300, synth.linspace_thresholds(-3, 3, 300), tag="f32 affine")


def test_classes_f32_irregular_nan(ctx):
    rng = np.random.default_rng(7)
    x = rng.normal(size=(211, 333)).astype(np.float32)
    x[rng.random(x.shape) < 0.05] = np.nan
    thr = np.sort(rng.normal(size=97)).astype(np.float32)
    thr[10:13] = thr[10]
    x.ravel()[:50] = thr[:50]
    compare(ctx, x, 97, thr, tag="f32 irregular")


def test_classes_u16_multipass(ctx):
    rng = np.random.default_rng(8)
    compare(ctx, rng.integers(0, 6000, size=(123, 457)).astype(np.uint16), 5000, tag="u16 5000 levels")


def test_classes_u16_thresholds(ctx):
    rng = np.random.default_rng(9)
    thr = np.sort(rng.uniform(0, 1000, size=64)).astype(np.float32)
    compare(ctx, rng.integers(0, 1100, size=(97, 301)).astype(np.uint16), 64, thr, tag="u16 thresholds")


def test_classes_unaligned_base(ctx):
    rng = np.random.default_rng(10)
    compare(ctx, rng.integers(0, 200, size=(77, 333)).astype(np.uint8), 200, tag="u8 unaligned", offset=3)


def test_classes_weightings_equal_curves_large(ctx):
    import torch
    from paper_2311_11740_amd import synth
    print("[case] classes vs curves 2048x3000 f32", flush=True)
    z = synth.grf((2048, 3000), 8.0, 12)
    thr = synth.linspace_thresholds(-4, 4, 1024)
    dev = torch.from_numpy(z).cuda()
    n = ctx.vertex_classes(dev, 1024, thresholds=thr).cpu().numpy()
    c8 = {k: v.cpu().numpy() for k, v in ctx.compute(dev, 1024, thresholds=thr, connectivity=8).items()}
    c4 = ctx.compute(dev, 1024, thresholds=thr, connectivity=4, channels=("ec",))["ec"].cpu().numpy()
    one, adj, diag, three, four = n
    assert np.array_equal(one - 2 * diag - three, 4 * c8["ec"])
    assert np.array_equal(one + 2 * diag - three, 4 * c4)
    assert np.array_equal(2 * one + 2 * adj + 4 * diag + 2 * three, 2 * c8["perimeter"])
    assert np.array_equal(one + 2 * adj + 2 * diag + 3 * three + 4 * four, 4 * c8["area"])


SHAPES_3D = [(1, 1, 1), (1, 1, 70), (70, 1, 1), (9, 13, 70), (20, 33, 65)]


@pytest.mark.parametrize("shape", SHAPES_3D)
def test_classes_3d_u8(ctx, shape):
    rng = np.random.default_rng(sum(shape))
    compare(ctx, rng.integers(0, 60, size=shape).astype(np.uint8), 50, tag="3D u8")


def test_classes_3d_u16_multipass(ctx):
    rng = np.random.default_rng(60)
    compare(ctx, rng.integers(0, 700, size=(11, 17, 40)).astype(np.uint16), 600, tag="3D u16 600 levels")


def test_classes_3d_f32_nan(ctx):
    rng = np.random.default_rng(61)
    x = rng.normal(size=(7, 30, 40)).astype(np.float32)
    x[rng.random(x.shape) < 0.05] = np.nan
    thr = np.sort(rng.normal(size=40)).astype(np.float32)
    compare(ctx, x, 40, thr, tag="3D f32")


def test_classes_3d_medium(ctx):
    from paper_2311_11740_amd import synth
    v = synth.quantise(synth.grf((64, 96, 128), 3.0, 62), 256)
    compare(ctx, v, 256, tag="3D GRF 64x96x128")


def test_classes_3d_integer_thresholds(ctx):
    rng = np.random.default_rng(63)
    thr = np.sort(rng.uniform(0, 1000, size=48)).astype(np.float32)
    compare(ctx, rng.integers(0, 1100, size=(8, 21, 67)).astype(np.uint16), 48, thr, tag="3D u16 thresholds")

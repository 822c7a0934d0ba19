"""GPU parity at the full workload sizes, in the launch configuration the
benchmark times.

* 2D 256 x 256 uint8 (256 levels), 8- and 4-connectivity: every level against
  the per-level counting oracle (O1) and the all-levels oracle (O2).
* 2D 8192 x 8192 float32 (1024 thresholds) and 3D 512^3 uint16 (4096 levels):
  whole curves against O2, and a few sampled levels against O1, which
  binarises and counts cells at one level at a time.
* A 3D volume whose z-marching launch is split along z (workgroup bins would
  otherwise see too many cells), against O2.
* The 8192 x 8192 float32 field over its superlevel filtration (falling
  thresholds), against O2 and sampled levels of O1.
"""
from __future__ import annotations

import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

NT = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2311_11740_amd import ecc
    c = ecc.Context(0)
    yield c
    c.close()


def gpu_curves(ctx, spec, channels):
    import torch
    dev = torch.from_numpy(spec.data).cuda()
    got = ctx.compute(dev, spec.n_levels, thresholds=spec.thresholds, connectivity=spec.connectivity,
                      channels=channels)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in got.items()}


def check_o2(spec, got, tag):
    import oracle
    ref = oracle.o2_curves(spec.data, spec.n_levels, thresholds=spec.thresholds,
                           connectivity=spec.connectivity, channels=tuple(got), n_threads=NT)
    for k in got:
        bad = np.nonzero(got[k] != ref[k])[0]
        assert bad.size == 0, f"{tag} {k}: {bad.size} levels differ, first {bad[:1]}"


def check_o1_levels(spec, got, levels, tag):
    import oracle
    ref = oracle.o1_curves(spec.data, spec.n_levels, thresholds=spec.thresholds,
                           connectivity=spec.connectivity, levels=levels, channels=tuple(got))
    for k in got:
        for i, lv in enumerate(levels):
            assert got[k][lv] == ref[k][i], f"{tag} {k} level {lv}: gpu {got[k][lv]} oracle {ref[k][i]}"


@pytest.mark.parametrize("conn", [8, 4])
def test_small_2d_all_levels(conn):
    """The 256 x 256 uint8 field at every level, with both readings of its
    pixels: closed faces (8-connectivity) and grid vertices (4-connectivity)."""
    from paper_2311_11740_amd import ecc, synth
    import oracle
    spec = synth.small_2d_u8()
    spec = synth.FieldSpec(spec.data, spec.n_levels, spec.thresholds, conn,
                           dict(spec.meta, name=f"{spec.meta['name']}_{conn}c"))
    print(f"[case] {spec.meta['name']}", flush=True)
    c = ecc.Context(0)
    try:
        got = gpu_curves(c, spec, None)
    finally:
        c.close()
    ref = oracle.o1_curves(spec.data, spec.n_levels, connectivity=conn)
    for k in got:
        assert np.array_equal(got[k], ref[k]), k
    check_o2(spec, got, spec.meta["name"])


def test_large_2d_f32(ctx):
    from paper_2311_11740_amd import synth
    spec = synth.large_2d_f32()
    print(f"[case] {spec.meta['name']}", flush=True)
    got = gpu_curves(ctx, spec, None)
    check_o2(spec, got, spec.meta["name"])
    check_o1_levels(spec, got, [0, 300, 511, 512, 700, 1023], spec.meta["name"])


def test_large_2d_f32_superlevel(ctx):
    """The same 8192 x 8192 float32 field over its superlevel filtration (the
    1024 thresholds in falling order, sets {value >= t_l}) against O2's
    superlevel route, and sampled levels against O1 binarising with >=."""
    import torch
    import oracle
    from paper_2311_11740_amd import synth
    spec = synth.large_2d_f32()
    t = spec.thresholds[::-1].copy()
    print(f"[case] {spec.meta['name']} superlevel", flush=True)
    dev = torch.from_numpy(spec.data).cuda()
    got = ctx.compute(dev, spec.n_levels, thresholds=t, superlevel=True)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in got.items()}
    ref = oracle.o2_curves(spec.data, spec.n_levels, thresholds=t, channels=tuple(got), n_threads=NT,
                           superlevel=True)
    for k in got:
        bad = np.nonzero(got[k] != ref[k])[0]
        assert bad.size == 0, f"superlevel {k}: {bad.size} levels differ, first {bad[:1]}"
    levels = [0, 400, 512, 1023]
    ref1 = oracle.o1_curves(spec.data, spec.n_levels, thresholds=t, levels=levels, channels=tuple(got),
                            superlevel=True)
    for k in got:
        for i, lv in enumerate(levels):
            assert got[k][lv] == ref1[k][i], (k, lv)


@pytest.mark.parametrize("channels", [("ec", "area", "volume"), None], ids=["no_crease", "all_channels"])
def test_large_3d_u16(ctx, channels):
    from paper_2311_11740_amd import synth
    spec = synth.large_3d_u16()
    print(f"[case] {spec.meta['name']} channels={channels}", flush=True)
    got = gpu_curves(ctx, spec, channels)
    check_o2(spec, got, spec.meta["name"])
    if channels is not None:
        check_o1_levels(spec, got, [1500, 2048, 2600], spec.meta["name"])


@pytest.mark.parametrize("conn,channels", [(26, ("ec", "area", "volume")), (6, ("ec", "area", "volume")),
                                           (26, None)], ids=["26c", "6c", "26c_all_channels"])
def test_3d_zmarch_split_along_z(ctx, conn, channels):
    """288 x 1024 x 1024 uint8: 1024 columns x 288 planes exceed what one
    launch may add to a workgroup's bins, so the launch is split along z
    (with the crease channel too, which shares the split)."""
    from paper_2311_11740_amd import synth
    rng = np.random.default_rng(77)
    a = rng.integers(0, 200, size=(288, 1024, 1024), dtype=np.uint8)
    a[rng.integers(0, 288, 64), rng.integers(0, 1024, 64), rng.integers(0, 1024, 64)] = 255  # never
    spec = synth.FieldSpec(a, 200, None, conn, dict(name=f"3d_288x1024x1024_u8_{conn}c"))
    print(f"[case] {spec.meta['name']}", flush=True)
    got = gpu_curves(ctx, spec, channels)
    check_o2(spec, got, spec.meta["name"])

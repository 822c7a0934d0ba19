"""GPU parity at the level boundaries of float thresholds (against the oracle).

Float fields with thresholds on a grid take their level from one fma in the
kernels, settled against the thresholds only within a margin of a level
boundary; the margin comes from evaluating the estimate at every threshold and
at the float above it.  These fields hold, for every threshold t_l, the value
t_l and the floats one to three steps below and above it, mixed into a smooth
field, so every boundary is probed from both sides in every kernel that uses
the estimate: the 2D kernel (both connectivities, one and two pass windows),
the z-marching and tile 3D kernels (with and without the crease), the batched
2D and 3D kernels, the vertex class counts (2D and 3D), the streamed and
allocation-free entry points, and the superlevel direction.
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


def edge_values(thr):
    """t_l and the floats 1..3 steps below and above each threshold."""
    t = np.asarray(thr, np.float32)
    vals = [t]
    up, dn = t.copy(), t.copy()
    for _ in range(3):
        up = np.nextafter(up, np.float32(np.inf)).astype(np.float32)
        dn = np.nextafter(dn, np.float32(-np.inf)).astype(np.float32)
        vals += [up, dn]
    return np.concatenate(vals)


def edge_field(shape, thr, seed):
    """A smooth field scaled to the thresholds' range with every edge value
    placed at random cells (the rest of the field keeps its smooth values)."""
    from paper_2311_11740_amd import synth
    rng = np.random.default_rng(seed)
    t = np.asarray(thr, np.float32)
    lo, hi = float(min(t[0], t[-1])), float(max(t[0], t[-1]))
    z = synth.grf(shape, 3.0, seed).astype(np.float64)
    z = (lo + (z - z.min()) / (z.max() - z.min() + 1e-30) * (hi - lo)).astype(np.float32)
    ev = edge_values(t)
    flat = z.reshape(-1)
    assert flat.size >= ev.size
    flat[rng.permutation(flat.size)[:ev.size]] = rng.permutation(ev)
    return z


def check(got, ref, tag):
    for k in got:
        g = got[k].cpu().numpy() if hasattr(got[k], "cpu") else got[k]
        bad = np.nonzero(g != ref[k])[0]
        assert bad.size == 0, f"{tag} {k}: {bad.size} levels differ, first {bad[:1]}: {g[bad[:1]]} vs {ref[k][bad[:1]]}"


def run(ctx, z, L, thr, conn=0, channels=None, superlevel=False, tag="", **kw):
    import torch
    import oracle
    print(f"[case] edges {tag} shape={z.shape} L={L} conn={conn} superlevel={superlevel} {kw}", flush=True)
    dev = torch.from_numpy(np.ascontiguousarray(z)).cuda()
    got = ctx.compute(dev, L, thresholds=thr, connectivity=conn, channels=channels, superlevel=superlevel, **kw)
    torch.cuda.synchronize()
    c = conn or (8 if z.ndim == 2 else 26)
    ref = oracle.o2_curves(z, L, thresholds=thr, connectivity=c, channels=tuple(got), n_threads=NT,
                           superlevel=superlevel)
    check(got, ref, tag)


GRIDS_2D = [(-4.0, 4.0, 1024), (0.0, 1.0, 4096), (-2.0, 2.0, 5000), (1000.0, 1001.0, 300)]


@pytest.mark.parametrize("grid", GRIDS_2D, ids=lambda g: f"{g[0]}_{g[1]}_{g[2]}")
@pytest.mark.parametrize("conn", [8, 4])
def test_2d(ctx, grid, conn):
    from paper_2311_11740_amd import synth
    thr = synth.linspace_thresholds(*grid)
    z = edge_field((257, 700), thr, 7 + grid[2])
    run(ctx, z, grid[2], thr, conn=conn, tag=f"2d {grid}")


@pytest.mark.parametrize("grid", [(-4.0, 4.0, 1024), (-2.0, 2.0, 5000)], ids=["1024", "5000"])
def test_2d_superlevel(ctx, grid):
    from paper_2311_11740_amd import synth
    thr = synth.linspace_thresholds(*grid)[::-1].copy()
    z = edge_field((257, 700), thr, 17 + grid[2])
    run(ctx, z, grid[2], thr, superlevel=True, tag=f"2d superlevel {grid}")


ALL_3D = ("ec", "perimeter", "area", "volume")
NO_CREASE = ("ec", "area", "volume")


@pytest.mark.parametrize("which,channels", [("zmarch", NO_CREASE), ("zmarch", ALL_3D), ("tile", ALL_3D),
                                            ("tile", NO_CREASE)], ids=["zmarch", "zmarch_crease", "tile",
                                                                      "tile_no_crease"])
@pytest.mark.parametrize("superlevel", [False, True], ids=["sub", "super"])
def test_3d(ctx, monkeypatch, which, channels, superlevel):
    from paper_2311_11740_amd import synth
    monkeypatch.setenv("ECC_3D_KERNEL", which)
    thr = synth.linspace_thresholds(-3.0, 3.0, 300)
    if superlevel:
        thr = thr[::-1].copy()
    z = edge_field((24, 40, 300), thr, 27)
    run(ctx, z, 300, thr, channels=channels, superlevel=superlevel, tag=f"3d {which} {channels}")


def test_3d_two_pass_windows(ctx, monkeypatch):
    from paper_2311_11740_amd import synth
    monkeypatch.setenv("ECC_3D_KERNEL", "zmarch")
    thr = synth.linspace_thresholds(-2.0, 2.0, 5000)
    z = edge_field((20, 48, 300), thr, 37)
    run(ctx, z, 5000, thr, channels=NO_CREASE, tag="3d zmarch 5000 levels")


def test_batched(ctx):
    import torch
    import oracle
    from paper_2311_11740_amd import synth
    t2 = synth.linspace_thresholds(-4.0, 4.0, 1024)
    t3 = synth.linspace_thresholds(-3.0, 3.0, 300)
    fields, L, thr, sup = [], [], [], []
    for k in range(8):
        t = t2 if k % 2 == 0 else t3
        tt = t[::-1].copy() if k % 4 == 3 else t
        shape = (97 + 13 * k, 120 + 29 * k) if k % 2 == 0 else (16 + k, 24, 40 + 5 * k)
        fields.append(edge_field(shape, tt, 47 + k))
        L.append(len(t)), thr.append(tt), sup.append(k % 4 == 3)
    print(f"[case] edges batched n={len(fields)}", flush=True)
    dev = [torch.from_numpy(f).cuda() for f in fields]
    out = ctx.compute_batch(dev, L, thresholds=thr, superlevel=sup)
    torch.cuda.synchronize()
    for i, f in enumerate(fields):
        ref = oracle.o2_curves(f, L[i], thresholds=thr[i], channels=tuple(out[i]), n_threads=NT,
                               superlevel=sup[i])
        check(out[i], ref, f"batched field {i} shape={f.shape} super={sup[i]}")


def test_vertex_classes(ctx):
    import torch
    import oracle
    from paper_2311_11740_amd import synth
    for shape, grid in (((257, 700), (-4.0, 4.0, 1024)), ((20, 40, 90), (-3.0, 3.0, 300))):
        thr = synth.linspace_thresholds(*grid)
        z = edge_field(shape, thr, 57 + len(shape))
        print(f"[case] edges vertex classes shape={shape} L={grid[2]}", flush=True)
        got = ctx.vertex_classes(torch.from_numpy(z).cuda(), grid[2], thresholds=thr)
        torch.cuda.synchronize()
        ref = oracle.class_counts(z, grid[2], thr)
        g = got.cpu().numpy()
        assert np.array_equal(g, ref), f"vertex classes {shape}: {np.argwhere(g != ref)[:1]}"


def test_streamed_and_noalloc(ctx):
    from paper_2311_11740_amd import synth
    thr = synth.linspace_thresholds(-4.0, 4.0, 1024)
    z = edge_field((1500, 700), thr, 67)
    print("[case] edges streamed 2D", flush=True)
    import oracle
    got = ctx.compute_streamed(z, 1024, thresholds=thr, slab_bytes=1 << 20)
    check(got, oracle.o2_curves(z, 1024, thresholds=thr, channels=tuple(got), n_threads=NT), "streamed")
    run(ctx, z, 1024, thr, tag="noalloc 2D", noalloc=True)

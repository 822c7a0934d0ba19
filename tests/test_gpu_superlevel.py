"""GPU parity of the superlevel filtration (ECC_SUPERLEVEL: a cell is active at
level l when value >= t_l, thresholds non-increasing; integer levels
t_l = L - 1 - l) through the C ABI, against the oracle's superlevel route.

* Single field: every level mode (integer levels through the implied
  thresholds, integer fields with thresholds, affine and irregular float
  thresholds), NaN / +-inf / -0.0 / values on thresholds, level counts above
  the per-pass window, both connectivities, the 3D z-marching and tile kernels
  with and without the crease.
* The library's superlevel curves of f equal its sublevel curves of -f at -t.
* Batched calls mixing both directions (also one threshold array used in both
  directions, whose level tables differ), the serving loop, host-resident
  fields, the allocation-free entry point and the vertex-class counts.
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


def oracle_sup(a, L, thr, conn, channels):
    import oracle
    return oracle.o2_curves(a, L, thresholds=thr, connectivity=conn, channels=channels, n_threads=NT,
                            superlevel=True)


def check(got, ref, tag):
    for k in got:
        g = got[k].cpu().numpy() if hasattr(got[k], "cpu") else got[k]
        bad = np.nonzero(g != ref[k])[0]
        assert bad.size == 0, f"{tag} {k}: {bad.size} levels differ, first {bad[:1]}: {g[bad[:1]]} vs {ref[k][bad[:1]]}"


def run_sup(ctx, a, L, thr=None, conn=0, channels=None, tag=""):
    import torch
    print(f"[case] superlevel {tag} shape={a.shape} dtype={a.dtype} L={L} conn={conn} "
          f"thr={'none' if thr is None else 'yes'} channels={channels}", flush=True)
    dev = torch.from_numpy(np.ascontiguousarray(a)).cuda()
    got = ctx.compute(dev, L, thresholds=thr, connectivity=conn, channels=channels, superlevel=True)
    torch.cuda.synchronize()
    c = conn or (8 if a.ndim == 2 else 26)
    check(got, oracle_sup(a, L, thr, c, tuple(got)), tag)
    return got


def with_specials(x, thr):
    x = x.copy()
    flat = x.reshape(-1)
    k = min(flat.size, 7)
    flat[:k] = np.array([np.nan, np.inf, -np.inf, -0.0, thr[0], thr[-1], thr[len(thr) // 2]],
                        np.float32)[:k]
    return x


@pytest.mark.parametrize("shape", [(1, 1), (1, 300), (300, 1), (37, 513), (1021, 769)])
@pytest.mark.parametrize("conn", [8, 4])
def test_2d_u8_integer_levels(ctx, shape, conn):
    rng = np.random.default_rng(hash((shape, conn, "sup")) % 2**32)
    a = rng.integers(0, 256, size=shape).astype(np.uint8)
    run_sup(ctx, a, 256, conn=conn, tag="2d_u8")


def test_2d_u8_fewer_and_more_levels(ctx):
    from paper_2311_11740_amd import synth
    a = synth.quantise(synth.grf((257, 1025), 3.0, 21), 256)
    run_sup(ctx, a, 100, tag="2d_u8_L100")  # values >= 99 at level 0
    run_sup(ctx, a, 300, tag="2d_u8_L300")  # levels 0..43 hold no cell
    run_sup(ctx, a, 1, tag="2d_u8_L1")


def test_2d_u16_multipass_and_thresholds(ctx):
    rng = np.random.default_rng(31)
    a = rng.integers(0, 12000, size=(70, 600)).astype(np.uint16)
    run_sup(ctx, a, 5000, tag="2d_u16_L5000")  # two passes of the level window
    thr = np.sort(rng.uniform(0, 12000, size=700)).astype(np.float32)[::-1].copy()
    thr[5] = thr[4]
    run_sup(ctx, a, 700, thr=thr, tag="2d_u16_thresholds")


@pytest.mark.parametrize("conn", [8, 4])
def test_2d_f32_affine_and_search(ctx, conn):
    from paper_2311_11740_amd import synth
    z = synth.grf((513, 1031), 6.0, 22)
    t_aff = synth.linspace_thresholds(-4.0, 4.0, 1024)[::-1].copy()
    run_sup(ctx, with_specials(z, t_aff), 1024, thr=t_aff, conn=conn, tag="2d_f32_affine")
    rng = np.random.default_rng(23)
    t_irr = np.sort(rng.normal(size=500)).astype(np.float32)[::-1].copy()
    t_irr[10:14] = t_irr[10]
    run_sup(ctx, with_specials(z, t_irr), 500, thr=t_irr, conn=conn, tag="2d_f32_search")


def test_2d_f32_multipass(ctx):
    from paper_2311_11740_amd import synth
    z = synth.grf((300, 700), 4.0, 24)
    t = synth.linspace_thresholds(-3.5, 3.5, 5000)[::-1].copy()
    run_sup(ctx, with_specials(z, t), 5000, thr=t, tag="2d_f32_L5000")


@pytest.mark.parametrize("kernel", ["zmarch", "tile"])
@pytest.mark.parametrize("conn", [26, 6])
def test_3d(ctx, monkeypatch, kernel, conn):
    from paper_2311_11740_amd import synth
    monkeypatch.setenv("ECC_3D_KERNEL", kernel)
    v = synth.quantise(synth.grf((21, 70, 300), 2.5, 25), 4096)
    run_sup(ctx, v, 4096, conn=conn, tag=f"3d_u16_{kernel}")
    z = synth.grf((13, 40, 270), 2.0, 26)
    t = synth.linspace_thresholds(-3.0, 3.0, 600)[::-1].copy()
    run_sup(ctx, with_specials(z, t), 600, thr=t, conn=conn, tag=f"3d_f32_{kernel}")
    u8 = np.random.default_rng(27).integers(0, 256, size=(9, 33, 65)).astype(np.uint8)
    run_sup(ctx, u8, 256, conn=conn, tag=f"3d_u8_{kernel}")


def test_3d_256_cubed(ctx):
    from paper_2311_11740_amd import synth
    v = synth.quantise(synth.grf((256, 256, 256), 4.0, 28), 4096)
    run_sup(ctx, v, 4096, tag="3d_256^3_u16")


def test_superlevel_equals_sublevel_of_negation(ctx):
    """f32: the library's superlevel curves of f at t equal its sublevel
    curves of -f at -t, bit for bit (2D and 3D)."""
    import torch
    from paper_2311_11740_amd import synth
    for shape, t in (((400, 900), synth.linspace_thresholds(-3, 3, 777)),
                     ((17, 60, 280), np.sort(np.random.default_rng(29).normal(size=300)).astype(np.float32))):
        z = with_specials(synth.grf(shape, 3.0, 30), t)
        print(f"[case] superlevel vs negation {shape}", flush=True)
        tdesc = t[::-1].copy()
        a = ctx.compute(torch.from_numpy(z).cuda(), len(t), thresholds=tdesc, superlevel=True)
        b = ctx.compute(torch.from_numpy(-z).cuda(), len(t), thresholds=-tdesc)
        torch.cuda.synchronize()
        for k in a:
            assert torch.equal(a[k], b[k]), k


def test_batch_mixed_directions(ctx):
    """One batched call with sublevel and superlevel fields: integer levels in
    both directions, float thresholds in both, and one constant threshold
    array (valid both ways) used by uint16 fields in both directions, whose
    value -> level tables differ."""
    import torch
    import oracle
    from paper_2311_11740_amd import synth
    rng = np.random.default_rng(40)
    fields, L, thr, sup = [], [], [], []
    t_up = synth.linspace_thresholds(-2.5, 2.5, 200)
    const = np.full(16, 300.0, np.float32)
    for k in range(48):
        kind = k % 6
        h, w = (int(x) for x in rng.integers(10, 400, size=2))
        if kind in (0, 1):
            fields.append(synth.quantise(synth.grf((h, w), 3.0, int(rng.integers(1 << 30))), 256))
            L.append(256), thr.append(None), sup.append(kind == 1)
        elif kind in (2, 3):
            z = synth.grf((h, w), 3.0, int(rng.integers(1 << 30)))
            L.append(200), sup.append(kind == 3)
            thr.append(t_up[::-1].copy() if kind == 3 else t_up)
            fields.append(with_specials(z, thr[-1]))
        else:
            fields.append(rng.integers(0, 600, size=(h, w)).astype(np.uint16))
            L.append(16), thr.append(const), sup.append(kind == 5)
    print(f"[case] batch mixed directions n={len(fields)}", flush=True)
    dev = [torch.from_numpy(f).cuda() for f in fields]
    out = ctx.compute_batch(dev, L, thresholds=thr, superlevel=sup)
    torch.cuda.synchronize()
    for i, f in enumerate(fields):
        ref = oracle.o2_curves(f, L[i], thresholds=thr[i], channels=tuple(out[i]), n_threads=NT,
                               superlevel=sup[i])
        check(out[i], ref, f"batch field {i} super={sup[i]}")


def test_serving_superlevel(ctx):
    from paper_2311_11740_amd import ecc, synth
    rng = np.random.default_rng(41)
    t = synth.linspace_thresholds(-3, 3, 150)[::-1].copy()
    reqs = []
    for k in range(30):
        kind = k % 3
        if kind == 0:
            h, w = (int(x) for x in rng.integers(20, 500, size=2))
            reqs.append((synth.quantise(synth.grf((h, w), 3.0, int(rng.integers(1 << 30))), 256), 256, None))
        elif kind == 1:
            h, w = (int(x) for x in rng.integers(20, 300, size=2))
            reqs.append((synth.grf((h, w), 3.0, int(rng.integers(1 << 30))), 150, t))
        else:
            d, h, w = (int(x) for x in rng.integers(4, 30, size=3))
            reqs.append((rng.integers(0, 1000, size=(d, h, w)).astype(np.uint16), 1000, None))
    print(f"[case] serving superlevel n={len(reqs)}", flush=True)
    srv = ecc.Server(ctx, 256 << 20, max_slots=64, max_batch=32)
    results = [None] * len(reqs)
    try:
        tickets = {}
        for i, (a, L, thr) in enumerate(reqs):
            while True:
                tk = srv.submit(a, L, thresholds=thr, superlevel=True)
                if tk is not None:
                    break
                for q in list(tickets):
                    r = srv.poll(q)
                    if r is not None:
                        results[tickets.pop(q)] = r
            tickets[tk] = i
        srv.drain()
        for q in list(tickets):
            results[tickets.pop(q)] = srv.poll(q)
    finally:
        srv.close()
    for i, ((a, L, thr), got) in enumerate(zip(reqs, results)):
        assert got is not None, i
        check(got, oracle_sup(a, L, thr, 8 if a.ndim == 2 else 26, tuple(got)), f"served {i}")


def test_streamed_superlevel(ctx):
    from paper_2311_11740_amd import synth
    z = synth.grf((3000, 700), 5.0, 42)
    t = synth.linspace_thresholds(-3, 3, 900)[::-1].copy()
    z = with_specials(z, t)
    print("[case] streamed superlevel 2D f32 and 3D u16", flush=True)
    got = ctx.compute_streamed(z, 900, thresholds=t, slab_bytes=1 << 20, superlevel=True)
    check(got, oracle_sup(z, 900, t, 8, tuple(got)), "streamed 2d")
    v = synth.quantise(synth.grf((60, 50, 300), 3.0, 43), 4096)
    got3 = ctx.compute_streamed(v, 4096, slab_bytes=1 << 20, superlevel=True)
    check(got3, oracle_sup(v, 4096, None, 26, tuple(got3)), "streamed 3d")


def test_noalloc_superlevel(ctx):
    import torch
    from paper_2311_11740_amd import synth
    z = synth.grf((600, 900), 4.0, 44)
    t = synth.linspace_thresholds(-3, 3, 512)[::-1].copy()
    z = with_specials(z, t)
    v = synth.quantise(synth.grf((30, 64, 280), 3.0, 45), 4096)
    u = np.random.default_rng(46).integers(0, 60000, size=(80, 333)).astype(np.uint16)
    for a, L, thr, tag in ((z, 512, t, "2d_f32"), (v, 4096, None, "3d_u16"), (u, 3000, None, "2d_u16")):
        print(f"[case] noalloc superlevel {tag}", flush=True)
        got = ctx.compute(torch.from_numpy(a).cuda(), L, thresholds=thr, noalloc=True, superlevel=True)
        torch.cuda.synchronize()
        check(got, oracle_sup(a, L, thr, 8 if a.ndim == 2 else 26, tuple(got)), f"noalloc {tag}")


def test_vertex_classes_superlevel(ctx):
    import torch
    import oracle
    from paper_2311_11740_amd import synth
    a = synth.quantise(synth.grf((300, 517), 3.0, 47), 256)
    z = synth.grf((200, 333), 3.0, 48)
    t = synth.linspace_thresholds(-3, 3, 300)[::-1].copy()
    z = with_specials(z, t)
    v = np.random.default_rng(49).integers(0, 40, size=(12, 30, 70)).astype(np.uint8)
    for arr, L, thr, tag in ((a, 256, None, "2d_u8"), (z, 300, t, "2d_f32"), (v, 40, None, "3d_u8")):
        print(f"[case] vertex classes superlevel {tag}", flush=True)
        got = ctx.vertex_classes(torch.from_numpy(arr).cuda(), L, thresholds=thr, superlevel=True)
        torch.cuda.synchronize()
        ref = oracle.class_counts(arr, L, thr, superlevel=True)
        assert np.array_equal(got.cpu().numpy(), ref), tag

"""Batched form for volumes: many small 3D fields in one persistent launch
(items of whole tiles, per-field histograms and tickets, the last workgroup of
a field scans it).

Each volume's curves from the batched call must equal the oracle's and the
single-field call's, bit for bit: for a workload shaped like the paper's
molecular-dynamics case (many 20 x 20 x 20 grids quantised to 0..255), for
a mix of dtypes, level modes, connectivities, channel sets (with and without
the crease) and filtration directions with degenerate shapes, together with
2D fields and with fields the batched kernels do not take (large volumes, more
than 4096 levels), on repeated calls of the captured graph, after autotuning,
and through the serving loop.
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


def check(outs, specs, tag):
    import torch
    import oracle
    torch.cuda.synchronize()
    for i, sp in enumerate(specs):
        a, L, thr, conn = sp[:4]
        sup = sp[4] if len(sp) > 4 else False
        got = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in outs[i].items()}
        ref = oracle.o2_curves(a, L, thresholds=thr, connectivity=conn, channels=tuple(got), n_threads=NT,
                               superlevel=sup)
        for k in got:
            if not np.array_equal(got[k], ref[k]):
                bad = np.nonzero(got[k] != ref[k])[0]
                raise AssertionError(f"{tag}: field {i} shape {a.shape} {a.dtype} L={L} conn={conn} sup={sup} "
                                     f"channel {k}: {bad.size} levels differ, first {bad[0]}: "
                                     f"{got[k][bad[0]]} vs {ref[k][bad[0]]}")


def md_grids(rng, n, side=20):
    from paper_2311_11740_amd import synth
    return [synth.quantise(synth.grf((side, side, side), float(rng.uniform(1.0, 3.0)), int(rng.integers(1 << 30))),
                           256) for _ in range(n)]


@pytest.mark.parametrize("conn", [26, 6])
def test_batch3d_md_grids(ctx, conn):
    import torch
    rng = np.random.default_rng(500 + conn)
    arrs = md_grids(rng, 300)
    print(f"[case] batch3d 300 x 20^3 u8 conn={conn}", flush=True)
    dev = [torch.from_numpy(a).cuda() for a in arrs]
    outs = ctx.compute_batch(dev, 256, connectivity=conn)
    check(outs, [(a, 256, None, conn) for a in arrs], f"md_{conn}")


def test_batch3d_mixed(ctx):
    import torch
    from paper_2311_11740_amd import synth
    rng = np.random.default_rng(510)
    thr_f = synth.linspace_thresholds(-3, 3, 300)
    thr_irr = np.sort(rng.normal(size=77)).astype(np.float32)
    thr_u16 = np.sort(rng.uniform(0, 3000, size=500)).astype(np.float32)
    specs, chans = [], []
    for k in range(72):
        kind = k % 8
        d, h, w = (int(x) for x in rng.integers(1, 45, size=3))
        conn = 26 if k % 3 else 6
        sup = k % 5 == 0
        ch = None if k % 4 else ("ec", "area", "volume")  # with and without the crease
        if kind == 0:
            a, L, thr = rng.integers(0, 256, size=(d, h, w)).astype(np.uint8), 256, None
        elif kind == 1:
            a, L, thr = rng.integers(0, 5000, size=(d, h, w)).astype(np.uint16), 4096, None
        elif kind == 2:
            a, L, thr = rng.integers(0, 3000, size=(d, h, w)).astype(np.uint16), 500, thr_u16
        elif kind == 3:
            z = synth.grf((d, h, w), 2.0, k)
            z.ravel()[::29] = thr_f[rng.integers(0, 300, size=z.ravel()[::29].size)]
            z.ravel()[0] = np.nan
            a, L, thr = z, 300, thr_f
        elif kind == 4:
            a, L, thr = rng.normal(size=(d, h, w)).astype(np.float32), 77, thr_irr
        elif kind == 5:
            a, L, thr = rng.integers(0, 30, size=(d, h, w)).astype(np.uint8), 17, None
        elif kind == 6:
            a, L, thr = rng.integers(0, 256, size=(int(rng.integers(2, 8)), 2 + k, 300)).astype(np.uint8), 256, None
        else:
            a, L, thr = synth.quantise(synth.grf((d, h, w), 2.0, k), 256), 256, None
        if sup and thr is not None:
            thr = thr[::-1].copy()
        specs.append((a, L, thr, conn, sup))
        chans.append(ch)
    # degenerate shapes, 2D fields and fields the batched kernels do not take
    extra = [
        (np.full((1, 1, 1), 3, np.uint8), 256, None, 26, False),
        (rng.integers(0, 256, size=(1, 1, 300)).astype(np.uint8), 256, None, 26, False),
        (rng.integers(0, 256, size=(300, 1, 1)).astype(np.uint8), 256, None, 6, True),
        (rng.integers(0, 256, size=(1, 300, 1)).astype(np.uint8), 256, None, 26, False),
        (rng.integers(0, 256, size=(70, 80)).astype(np.uint8), 256, None, 8, False),
        (rng.integers(0, 256, size=(30, 500)).astype(np.uint8), 256, None, 4, True),
        (rng.integers(0, 4096, size=(80, 200, 300)).astype(np.uint16), 4096, None, 26, False),  # large volume
        (rng.integers(0, 9000, size=(6, 20, 30)).astype(np.uint16), 9000, None, 26, False),  # > 4096 levels
    ]
    specs += extra
    chans += [None] * len(extra)
    order = rng.permutation(len(specs))
    specs = [specs[i] for i in order]
    chans = [chans[i] for i in order]
    print(f"[case] batch3d mixed n={len(specs)}", flush=True)
    dev = [torch.from_numpy(np.ascontiguousarray(s[0])).cuda() for s in specs]
    b = ctx.batch(dev, [s[1] for s in specs], [s[2] for s in specs], [s[3] for s in specs],
                  superlevel=[s[4] for s in specs])
    b.run()
    check(b.outputs, specs, "mixed")
    # a quarter of the volumes again, without the crease channel
    sub = [i for i, ch in enumerate(chans) if ch is not None]
    dev_sub = [dev[i] for i in sub]
    specs_sub = [specs[i] for i in sub]
    b2 = ctx.batch(dev_sub, [s[1] for s in specs_sub], [s[2] for s in specs_sub], [s[3] for s in specs_sub],
                   channels=("ec", "area", "volume"), superlevel=[s[4] for s in specs_sub])
    b2.run()
    check(b2.outputs, specs_sub, "mixed_no_crease")


def test_batch3d_replay_and_tune(ctx):
    import torch
    rng = np.random.default_rng(520)
    shapes = [tuple(int(x) for x in rng.integers(3, 40, size=3)) for _ in range(90)]
    for rep in range(3):
        arrs = [rng.integers(0, 256, size=s).astype(np.uint8) for s in shapes]
        dev = [torch.from_numpy(a).cuda() for a in arrs]
        print(f"[case] batch3d replay {rep}", flush=True)
        b = ctx.batch(dev, 256)
        b.run()
        junk = torch.randn(1 << 20, device="cuda").sum()  # unrelated work between replays
        torch.cuda.synchronize()
        del junk
        check(b.outputs, [(a, 256, None, 26) for a in arrs], f"replay{rep}")
    print("[case] batch3d tune", flush=True)
    b.tune()
    arrs = [rng.integers(0, 256, size=s).astype(np.uint8) for s in shapes]
    dev = [torch.from_numpy(a).cuda() for a in arrs]
    b = ctx.batch(dev, 256)
    b.run()
    check(b.outputs, [(a, 256, None, 26) for a in arrs], "tuned")


def test_batch3d_equals_single_field_calls(ctx):
    import torch
    rng = np.random.default_rng(530)
    arrs = md_grids(rng, 64, side=24) + [rng.integers(0, 256, size=(33, 40, 90)).astype(np.uint8)]
    print("[case] batch3d vs per-field calls", flush=True)
    dev = [torch.from_numpy(a).cuda() for a in arrs]
    b = ctx.batch(dev, 256)
    b.run()
    singles = [ctx.compute(d, 256) for d in dev]
    torch.cuda.synchronize()
    for i in range(len(arrs)):
        for k in singles[i]:
            assert torch.equal(b.outputs[i][k], singles[i][k]), (i, k)


def test_serving_small_volumes(ctx):
    """Small volumes now join the batched launch of the serving loop."""
    import time
    from paper_2311_11740_amd import ecc
    rng = np.random.default_rng(540)
    reqs = []
    for k in range(80):
        if k % 4 == 3:
            h, w = (int(x) for x in rng.integers(10, 300, size=2))
            reqs.append((rng.integers(0, 256, size=(h, w)).astype(np.uint8), 256, None, 8))
        else:
            reqs.append((md_grids(rng, 1)[0], 256, None, 26 if k % 2 else 6))
    print(f"[case] serving {len(reqs)} requests, mostly 20^3 grids", flush=True)
    srv = ecc.Server(ctx, 64 << 20, max_slots=128, max_batch=128)
    results = [None] * len(reqs)
    try:
        tickets = {}
        for i, (a, L, thr, conn) in enumerate(reqs):
            while True:
                t = srv.submit(a, L, thresholds=thr, connectivity=conn)
                if t is not None:
                    break
                time.sleep(0.0005)
                for q in list(tickets):
                    r = srv.poll(q)
                    if r is not None:
                        results[tickets.pop(q)] = r
            tickets[t] = i
        srv.drain()
        for q in list(tickets):
            results[tickets.pop(q)] = srv.poll(q)
    finally:
        srv.close()
    check(results, reqs, "serving_volumes")

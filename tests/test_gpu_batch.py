"""Batched form: one call over many fields of uneven shapes.

Each field's curves from the batched call must equal the oracle's and the
single-field call's, bit for bit: for a mix the batched kernels take (2D, any
dtype and level mode, both connectivities; small volumes) and one handed to
the single-field path (more than 4096 levels, fields smaller than one vector
load); on repeated calls (the captured graph replayed with new data, with
other work between the calls); and after autotuning.  Volumes in more depth:
test_gpu_batch3d.py.
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


def oracle_curves(a, L, thr, conn, channels):
    import oracle
    return oracle.o2_curves(a, L, thresholds=thr, connectivity=conn, channels=channels, n_threads=NT)


def check_batch(outs, specs, tag):
    import torch
    torch.cuda.synchronize()
    for i, (a, L, thr, conn) in enumerate(specs):
        got = {k: v.cpu().numpy() for k, v in outs[i].items()}
        ref = oracle_curves(a, L, thr, conn, tuple(got))
        for k in got:
            if not np.array_equal(got[k], ref[k]):
                bad = np.nonzero(got[k] != ref[k])[0]
                raise AssertionError(f"{tag}: field {i} shape {a.shape} {a.dtype} L={L} conn={conn} "
                                     f"channel {k}: {bad.size} levels differ, first {bad[0]}")


def u8_fields(rng, n, lo=3, hi=700):
    from paper_2311_11740_amd import synth
    out = []
    for k in range(n):
        h, w = (int(x) for x in np.exp(rng.uniform(np.log(lo), np.log(hi), size=2)))
        a = synth.quantise(synth.grf((h, w), float(rng.uniform(1.5, 8)), int(rng.integers(1 << 30))), 256)
        out.append(a)
    return out


def test_batch_u8_identity(ctx):
    import torch
    rng = np.random.default_rng(100)
    arrs = u8_fields(rng, 120)
    arrs += [np.zeros((1, 1), np.uint8), np.full((2, 5), 7, np.uint8), np.full((3, 900), 255, np.uint8)]
    print(f"[case] batch u8 identity n={len(arrs)}", flush=True)
    dev = [torch.from_numpy(a).cuda() for a in arrs]
    outs = ctx.compute_batch(dev, 256, connectivity=8)
    check_batch(outs, [(a, 256, None, 8) for a in arrs], "u8_identity")


def test_batch_mixed_kinds(ctx):
    """dtypes, level modes, level counts and connectivities mixed in one call,
    plus fields for the single-field path."""
    import torch
    from paper_2311_11740_amd import synth
    rng = np.random.default_rng(101)
    specs = []
    thr_u8 = np.array([3.5, 10, 10, 99.9, 100, 200, 254.5], np.float32)
    thr_f = synth.linspace_thresholds(-3, 3, 300)
    thr_irr = np.sort(rng.normal(size=77)).astype(np.float32)
    for k in range(60):
        kind = k % 6
        h, w = (int(x) for x in rng.integers(2, 400, size=2))
        conn = 8 if k % 2 == 0 else 4
        if kind == 0:
            specs.append((rng.integers(0, 256, size=(h, w)).astype(np.uint8), 256, None, conn))
        elif kind == 1:
            specs.append((rng.integers(0, 256, size=(h, w)).astype(np.uint8), len(thr_u8), thr_u8, conn))
        elif kind == 2:
            specs.append((rng.integers(0, 5000, size=(h, w)).astype(np.uint16), 4096, None, conn))
        elif kind == 3:
            z = synth.grf((h, w), 3.0, k)
            z.ravel()[::31] = thr_f[rng.integers(0, 300, size=z.ravel()[::31].size)]
            z.ravel()[0] = np.nan
            specs.append((z, 300, thr_f, conn))
        elif kind == 4:
            specs.append((rng.normal(size=(h, w)).astype(np.float32), 77, thr_irr, conn))
        else:
            specs.append((rng.integers(0, 30, size=(h, w)).astype(np.uint8), 17, None, conn))
    # small volumes (3D batched kernel), more than 4096 levels and smaller than
    # one vector load (single-field path)
    specs.append((rng.integers(0, 40, size=(9, 20, 33)).astype(np.uint8), 36, None, 26))
    specs.append((rng.integers(0, 40, size=(7, 5, 300)).astype(np.uint16), 36, None, 6))
    specs.append((rng.integers(0, 9000, size=(50, 70)).astype(np.uint16), 9000, None, 8))
    specs.append((rng.integers(0, 256, size=(1, 3)).astype(np.uint8), 256, None, 4))
    order = rng.permutation(len(specs))
    specs = [specs[i] for i in order]
    print(f"[case] batch mixed n={len(specs)}", flush=True)
    dev = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a, _, _, _ in specs]
    b = ctx.batch(dev, [s[1] for s in specs], [s[2] for s in specs], [s[3] for s in specs])
    b.run()
    check_batch(b.outputs, specs, "mixed")


def test_batch_replay_new_data_and_tune(ctx):
    """The same shapes again (the cached plan and its graph) with new data,
    other work on the stream between calls, then after autotuning."""
    import torch
    rng = np.random.default_rng(102)
    shapes = [a.shape for a in u8_fields(rng, 80, 3, 1500)]
    for rep in range(3):
        arrs = [rng.integers(0, 256, size=s).astype(np.uint8) for s in shapes]
        dev = [torch.from_numpy(a).cuda() for a in arrs]
        print(f"[case] batch replay {rep}", flush=True)
        b = ctx.batch(dev, 256, connectivity=8)
        b.run()
        junk = torch.randn(1 << 20, device="cuda").sum()  # unrelated work between replays
        torch.cuda.synchronize()
        del junk
        check_batch(b.outputs, [(a, 256, None, 8) for a in arrs], f"replay{rep}")
    print("[case] batch tune", flush=True)
    b.tune()
    arrs = [rng.integers(0, 256, size=s).astype(np.uint8) for s in shapes]
    dev = [torch.from_numpy(a).cuda() for a in arrs]
    b = ctx.batch(dev, 256, connectivity=8)
    b.run()
    check_batch(b.outputs, [(a, 256, None, 8) for a in arrs], "tuned")


def test_batch_equals_single_field_calls(ctx):
    """A slice of the 4096-field workload: batched == one call per field."""
    import torch
    from paper_2311_11740_amd import synth
    specs = synth.batch_2d_u8(n=192)
    print("[case] batch vs per-field, 192 fields of the batched workload", flush=True)
    dev = [torch.from_numpy(s.data).cuda() for s in specs]
    b = ctx.batch(dev, 256, connectivity=8)
    b.run()
    singles = [ctx.compute(d, 256, connectivity=8) for d in dev]
    torch.cuda.synchronize()
    for i in range(len(specs)):
        for k in singles[i]:
            assert torch.equal(b.outputs[i][k], singles[i][k]), (i, k)
    check_batch(b.outputs[:24], [(s.data, 256, None, 8) for s in specs[:24]], "c4_slice")


def test_batch_many_threshold_arrays(ctx):
    """40 float32 fields with 40 distinct threshold arrays and 60 with copies
    of one array (equal content, separate buffers) in one call; then more
    distinct arrays than the context caches at once is refused up front."""
    import torch
    from paper_2311_11740_amd import ecc, synth
    rng = np.random.default_rng(103)
    common = synth.linspace_thresholds(-3, 3, 128)
    specs = []
    for k in range(100):
        h, w = (int(x) for x in rng.integers(5, 120, size=2))
        a = rng.normal(size=(h, w)).astype(np.float32)
        if k < 40:
            thr = np.sort(rng.normal(size=int(rng.integers(3, 60)))).astype(np.float32)
        else:
            thr = common.copy()
        specs.append((a, len(thr), thr, 8))
    print(f"[case] batch with {len(specs)} thresholded fields, 41 distinct arrays", flush=True)
    dev = [torch.from_numpy(a).cuda() for a, _, _, _ in specs]
    b = ctx.batch(dev, [s[1] for s in specs], [s[2] for s in specs], [s[3] for s in specs])
    b.run()
    check_batch(b.outputs, specs, "many_thresholds")
    too_many = [np.sort(rng.normal(size=8)).astype(np.float32) for _ in range(257)]
    dev2 = [torch.from_numpy(rng.normal(size=(9, 9)).astype(np.float32)).cuda() for _ in too_many]
    with pytest.raises(ecc.EccError) as ei:
        ctx.compute_batch(dev2, 8, thresholds=too_many)
    assert ei.value.status == ecc.ECC_ERR_UNSUPPORTED


def test_batch_c4_full(ctx):
    """The whole batched workload: 4096 uint8 fields, sides log-uniform in
    [64, 2048], 256 levels, 8-C, as the benchmark runs it: the batched call
    equals one call per field on every field, and a sample equals the oracle."""
    import torch
    from paper_2311_11740_amd import synth
    specs = synth.batch_2d_u8(workers=min(16, os.cpu_count() or 1))
    print(f"[case] batch C4, {len(specs)} fields", flush=True)
    dev = [torch.from_numpy(s.data).cuda() for s in specs]
    b = ctx.batch(dev, 256, connectivity=8)
    b.run()
    singles = [ctx.compute(d, 256, connectivity=8) for d in dev]
    torch.cuda.synchronize()
    for i in range(len(specs)):
        for k in singles[i]:
            assert torch.equal(b.outputs[i][k], singles[i][k]), (i, k)
    sample = list(range(0, len(specs), len(specs) // 16))
    check_batch([b.outputs[i] for i in sample], [(specs[i].data, 256, None, 8) for i in sample], "c4_full")

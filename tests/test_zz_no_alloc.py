"""The allocation-free entry point (ecc_curves_compute_noalloc), called through
the C ABI, against ecc_curves_compute: bit-exact on every case, on two calls
in a row whose second input is smaller than the first (the shared scratch
array keeps the first call's contents), for each dtype and level mode and in
2D and 3D, up to the largest level count; a request whose buffers do not fit
the scratch array is refused before any work is queued.
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


def both(ctx, a, L, thr, conn):
    import torch
    dev = torch.from_numpy(np.ascontiguousarray(a)).cuda()
    ref = ctx.compute(dev, L, thresholds=thr, connectivity=conn)
    out = {k: torch.full_like(v, -7) for k, v in ref.items()}
    got = ctx.compute(dev, L, thresholds=thr, connectivity=conn, out=out, noalloc=True)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in ref.items()}, {k: v.cpu().numpy() for k, v in got.items()}


def check_pair(ctx, cases, tag):
    for i, (a, L, thr, conn) in enumerate(cases):
        print(f"[case] {tag} call {i}: {a.shape} {a.dtype} L={L} conn={conn}", flush=True)
        ref, got = both(ctx, a, L, thr, conn)
        for k in ref:
            assert np.array_equal(ref[k], got[k]), f"{tag} call {i} channel {k}"


def test_noalloc_2d_f32_then_smaller(ctx):
    from paper_2311_11740_amd import synth
    thr = synth.linspace_thresholds(-4, 4, 1024)
    big = synth.grf((2048, 3000), 16.0, 21).astype(np.float32)
    small = synth.grf((300, 517), 4.0, 22).astype(np.float32)
    check_pair(ctx, [(big, 1024, thr, 8), (small, 1024, thr, 8)], "2d_f32")


def test_noalloc_2d_integer_modes_then_smaller(ctx):
    rng = np.random.default_rng(31)
    thr8 = np.array([3.5, 10, 10, 99.9, 100, 200, 254.5], np.float32)
    cases = [(rng.integers(0, 256, size=(1500, 1200)).astype(np.uint8), 256, None, 4),
             (rng.integers(0, 256, size=(123, 77)).astype(np.uint8), len(thr8), thr8, 8),
             (rng.integers(0, 6000, size=(40, 333)).astype(np.uint16), 5000, None, 8),
             (rng.integers(0, 256, size=(1, 3)).astype(np.uint8), 256, None, 8)]
    check_pair(ctx, cases, "2d_int")


def test_noalloc_3d_then_smaller(ctx):
    from paper_2311_11740_amd import synth
    rng = np.random.default_rng(32)
    vol = synth.quantise(synth.grf((96, 200, 300), 4.0, 33), 4096)
    thr = np.linspace(100.5, 3900.5, 300).astype(np.float32)
    cases = [(vol, 4096, None, 26), (vol[:20, :50, :70].copy(), 300, thr, 6),
             (rng.normal(size=(9, 17, 31)).astype(np.float32), 50, np.sort(rng.normal(size=50)).astype(np.float32),
              26)]
    check_pair(ctx, cases, "3d")


def test_noalloc_most_levels_then_too_large(ctx):
    """65535 levels (the most a field may have) fit for a 2D field; a small
    volume on the tile kernel, whose per-workgroup partials take workgroups x
    4 x 65535 x 4 bytes, does not, and is refused."""
    import torch
    from paper_2311_11740_amd import ecc
    rng = np.random.default_rng(34)
    check_pair(ctx, [(rng.integers(0, 65535, size=(700, 900)).astype(np.uint16), 65535, None, 8)], "2d_65535")
    a = torch.zeros((64, 64, 64), dtype=torch.uint16, device="cuda")
    out = {k: torch.full((65535,), -7, dtype=torch.int64, device="cuda") for k in ("ec", "area", "volume")}
    with pytest.raises(ecc.EccError) as ei:
        ctx.compute(a, 65535, out=out, noalloc=True)
    assert ei.value.status == ecc.ECC_ERR_UNSUPPORTED
    torch.cuda.synchronize()
    assert all(bool((v == -7).all()) for v in out.values()), "a refused call wrote its outputs"

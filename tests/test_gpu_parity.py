"""GPU parity: libecc curves == the oracle's curves, bit for bit, through the C ABI.

Every case is printed (and flushed) before it runs so that a failing GPU step
names its case.  Sizes span several work units (2D: strips of 62 lanes x 16
bytes of a row, streamed down the rows; 3D: columns of 4 rows x 256 voxels
marched along z, or tiles of 16 x 4 x 64 voxels) with ragged tails, the degenerate shapes (1 x 1, 1 x N,
N x 1), every level mode (identity integer levels, integer levels through
thresholds, affine float thresholds, irregular float thresholds with ties),
NaN and never-active values, constant fields, one level, and level counts above
the per-pass window (several passes).
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


def run_and_compare(ctx, arr, L, thr=None, conn=0, channels=None, tag=""):
    import torch
    import oracle
    print(f"[case] {tag} shape={arr.shape} dtype={arr.dtype} L={L} conn={conn} "
          f"thr={'none' if thr is None else 'yes'} channels={channels}", flush=True)
    dev = torch.from_numpy(np.ascontiguousarray(arr)).cuda()
    got = ctx.compute(dev, L, thresholds=thr, connectivity=conn, channels=channels)
    torch.cuda.synchronize()
    nd = arr.ndim
    if conn == 0:
        conn = 8 if nd == 2 else 26
    want_ch = tuple(got.keys())
    ref = oracle.o2_curves(arr, L, thresholds=thr, connectivity=conn, channels=want_ch, n_threads=NT)
    for k in want_ch:
        g = got[k].cpu().numpy()
        r = ref[k]
        if not np.array_equal(g, r):
            bad = np.nonzero(g != r)[0]
            raise AssertionError(f"{tag} channel {k}: {bad.size} levels differ, first at {bad[0]}: "
                                 f"gpu {g[bad[0]]} oracle {r[bad[0]]}")
    return got


SHAPES_2D = [(1, 1), (1, 300), (300, 1), (37, 513), (64, 256), (257, 1025), (1021, 769)]


@pytest.mark.parametrize("shape", SHAPES_2D)
@pytest.mark.parametrize("conn", [8, 4])
def test_2d_u8_identity(ctx, shape, conn):
    rng = np.random.default_rng(hash((shape, conn)) % 2**32)
    a = rng.integers(0, 256, size=shape).astype(np.uint8)
    run_and_compare(ctx, a, 256, conn=conn, tag="2d_u8")


@pytest.mark.parametrize("shape", [(45, 300), (513, 257)])
def test_2d_u8_smooth_and_fewer_levels(ctx, shape):
    from paper_2311_11740_amd import synth
    a = synth.quantise(synth.grf(shape, 3.0, 11), 256)
    run_and_compare(ctx, a, 256, tag="2d_u8_grf")
    run_and_compare(ctx, a, 100, tag="2d_u8_L100_never")  # values >= 100 never enter
    run_and_compare(ctx, a, 1, tag="2d_u8_L1")


def test_2d_u16_identity_and_multipass(ctx):
    rng = np.random.default_rng(5)
    a = rng.integers(0, 12000, size=(70, 600)).astype(np.uint16)
    run_and_compare(ctx, a, 4096, tag="2d_u16_L4096")
    run_and_compare(ctx, a, 10000, tag="2d_u16_L10000_3pass")
    run_and_compare(ctx, a, 10000, conn=4, tag="2d_u16_L10000_4c")


def test_2d_f32_affine_thresholds(ctx):
    from paper_2311_11740_amd import synth
    z = synth.grf((300, 700), 8.0, 21)
    thr = synth.linspace_thresholds(-4.0, 4.0, 1024)
    idx = np.arange(0, z.size, 97)
    z.ravel()[idx] = thr[np.random.default_rng(1).integers(0, 1024, size=idx.size)]  # on thresholds
    z.ravel()[5] = np.nan
    z.ravel()[6] = np.inf
    z.ravel()[7] = -np.inf
    z.ravel()[8] = -0.0
    # far below the first threshold (level 0) and far above the last (never)
    z.ravel()[9::211] = np.float32(-4.0) - np.float32(8 / 1023) * (np.arange(z.ravel()[9::211].size) % 50)
    z.ravel()[10] = np.float32(-1e30)
    z.ravel()[14] = np.float32(1e30)
    z.ravel()[15] = np.float32(4.5)
    run_and_compare(ctx, z, 1024, thr=thr, tag="2d_f32_affine")
    run_and_compare(ctx, z, 1024, thr=thr, conn=4, tag="2d_f32_affine_4c")


def test_2d_f32_irregular_thresholds(ctx):
    rng = np.random.default_rng(8)
    z = rng.normal(size=(129, 257)).astype(np.float32)
    thr = np.sort(rng.normal(size=300)).astype(np.float32)
    thr[10:20] = thr[10]  # repeated thresholds
    z.ravel()[::50] = thr[rng.integers(0, 300, size=z.ravel()[::50].size)]
    z.ravel()[3] = np.nan
    run_and_compare(ctx, z, 300, thr=thr, tag="2d_f32_irregular")


def test_2d_integer_with_thresholds(ctx):
    rng = np.random.default_rng(9)
    a = rng.integers(0, 256, size=(100, 300)).astype(np.uint8)
    thr = np.array([3.5, 10, 10, 99.9, 100, 200, 254.5], np.float32)
    run_and_compare(ctx, a, len(thr), thr=thr, tag="2d_u8_thr")
    b = rng.integers(0, 65535, size=(90, 310)).astype(np.uint16)
    thr2 = np.linspace(0, 70000, 500).astype(np.float32)
    run_and_compare(ctx, b, 500, thr=thr2, tag="2d_u16_thr")


def test_2d_constant_and_never(ctx):
    run_and_compare(ctx, np.full((70, 530), 7, np.uint8), 256, tag="2d_const")
    run_and_compare(ctx, np.full((70, 530), 250, np.uint8), 100, tag="2d_all_never")
    run_and_compare(ctx, np.full((33, 33), np.nan, np.float32), 4,
                    thr=np.arange(4, dtype=np.float32), tag="2d_all_nan")


def test_2d_channel_subsets(ctx):
    rng = np.random.default_rng(10)
    a = rng.integers(0, 50, size=(77, 300)).astype(np.uint8)
    for ch in (("ec",), ("perimeter",), ("area",), ("ec", "area")):
        run_and_compare(ctx, a, 50, channels=ch, tag=f"2d_ch_{'_'.join(ch)}")


SHAPES_3D = [(1, 1, 1), (1, 1, 70), (70, 1, 1), (3, 5, 7), (17, 9, 130), (40, 33, 65), (1, 64, 64),
             (9, 7, 513), (5, 258, 300)]
# 3D paths: the z-marching kernel without the crease measure, with it (a
# second z-marching launch adds the crease), and the generic tile kernel with
# and without it (forced: by default small volumes take the tile kernel and
# large ones z-marching)
NO_CREASE = ("ec", "area", "volume")
ALL_3D = None
PATHS_3D = {"zmarch": (NO_CREASE, "zmarch"), "zmarch_crease": (ALL_3D, "zmarch"), "tile": (ALL_3D, "tile"),
            "tile_no_crease": (NO_CREASE, "tile")}


class kernel_choice:
    """Select the 3D kernel for the calls inside the block (ECC_3D_KERNEL)."""

    def __init__(self, which):
        self.which = which

    def __enter__(self):
        self.old = os.environ.pop("ECC_3D_KERNEL", None)
        if self.which:
            os.environ["ECC_3D_KERNEL"] = self.which

    def __exit__(self, *exc):
        os.environ.pop("ECC_3D_KERNEL", None)
        if self.old is not None:
            os.environ["ECC_3D_KERNEL"] = self.old


@pytest.mark.parametrize("shape", SHAPES_3D)
@pytest.mark.parametrize("conn", [26, 6])
@pytest.mark.parametrize("path", list(PATHS_3D))
def test_3d_u8(ctx, shape, conn, path):
    channels, which = PATHS_3D[path]
    rng = np.random.default_rng(hash((shape, conn, 3)) % 2**32)
    a = rng.integers(0, 40, size=shape).astype(np.uint8)
    with kernel_choice(which):
        run_and_compare(ctx, a, 36, conn=conn, channels=channels, tag=f"3d_u8_{path}")


@pytest.mark.parametrize("path", list(PATHS_3D))
def test_3d_u16_grf(ctx, path):
    from paper_2311_11740_amd import synth
    channels, which = PATHS_3D[path]
    a = synth.quantise(synth.grf((48, 40, 136), 3.0, 31), 4096)
    with kernel_choice(which):
        run_and_compare(ctx, a, 4096, tag="3d_u16_grf", channels=channels)
        run_and_compare(ctx, a, 3000, conn=6, tag="3d_u16_grf_6c_never", channels=channels)
        run_and_compare(ctx, a, 5000, tag="3d_u16_grf_2pass", channels=channels)
        run_and_compare(ctx, a, 5000, conn=6, tag="3d_u16_grf_2pass_6c", channels=channels)


@pytest.mark.parametrize("path", list(PATHS_3D))
def test_3d_f32_thresholds(ctx, path):
    from paper_2311_11740_amd import synth
    channels, which = PATHS_3D[path]
    z = synth.grf((20, 30, 70), 2.5, 41)
    z.ravel()[11] = np.nan
    z.ravel()[12] = np.inf
    z.ravel()[13] = -np.inf
    thr = synth.linspace_thresholds(-3, 3, 200)
    z.ravel()[100::37] = thr[np.arange(z.ravel()[100::37].size) % 200]  # values on thresholds
    z.ravel()[101::53] = np.float32(-3.0) - np.float32(0.03) * (np.arange(z.ravel()[101::53].size) % 40)
    z.ravel()[102::97] = np.float32(3.0) + np.float32(0.03) * (np.arange(z.ravel()[102::97].size) % 40)
    thr2 = np.sort(np.random.default_rng(2).normal(size=77)).astype(np.float32)
    with kernel_choice(which):
        run_and_compare(ctx, z, 200, thr=thr, tag="3d_f32_affine", channels=channels)
        run_and_compare(ctx, z, 77, thr=thr2, conn=6, tag="3d_f32_irregular_6c", channels=channels)


def test_3d_integer_with_thresholds(ctx):
    rng = np.random.default_rng(19)
    a = rng.integers(0, 256, size=(13, 21, 300)).astype(np.uint8)
    thr = np.array([3.5, 10, 10, 99.9, 100, 200, 254.5], np.float32)
    for conn in (26, 6):
        run_and_compare(ctx, a, len(thr), thr=thr, conn=conn, channels=NO_CREASE, tag="3d_u8_thr")
    b = rng.integers(0, 65535, size=(11, 17, 150)).astype(np.uint16)
    thr2 = np.linspace(0, 70000, 500).astype(np.float32)
    run_and_compare(ctx, b, 500, thr=thr2, channels=NO_CREASE, tag="3d_u16_thr")


def test_3d_channel_subsets(ctx):
    rng = np.random.default_rng(20)
    a = rng.integers(0, 30, size=(9, 20, 100)).astype(np.uint8)
    for ch in (("ec",), ("area",), ("volume",), ("perimeter",), ("ec", "perimeter")):
        run_and_compare(ctx, a, 30, channels=ch, tag=f"3d_ch_{'_'.join(ch)}")


@pytest.mark.parametrize("path", list(PATHS_3D))
def test_3d_constant(ctx, path):
    channels, which = PATHS_3D[path]
    with kernel_choice(which):
        run_and_compare(ctx, np.full((20, 6, 70), 3, np.uint16), 10, tag="3d_const", channels=channels)
        run_and_compare(ctx, np.full((5, 6, 270), 200, np.uint8), 100, tag="3d_all_never", channels=channels)


def test_repeat_is_deterministic(ctx):
    import torch
    rng = np.random.default_rng(12)
    a = torch.from_numpy(rng.integers(0, 256, size=(500, 700)).astype(np.uint8)).cuda()
    r1 = ctx.compute(a, 256)
    r2 = ctx.compute(a, 256)
    torch.cuda.synchronize()
    for k in r1:
        assert torch.equal(r1[k], r2[k])


def test_async_on_side_stream(ctx):
    """Work queued on a non-default stream is ordered after the previous call."""
    import torch
    import oracle
    rng = np.random.default_rng(13)
    a = rng.integers(0, 256, size=(300, 900)).astype(np.uint8)
    b = rng.integers(0, 256, size=(333, 444)).astype(np.uint8)
    da, db = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    s = torch.cuda.Stream()
    ra = ctx.compute(da, 256)
    with torch.cuda.stream(s):
        rb = ctx.compute(db, 256, stream=s)
    torch.cuda.synchronize()
    oa, ob = oracle.o2_curves(a, 256), oracle.o2_curves(b, 256)
    for k in ra:
        assert np.array_equal(ra[k].cpu().numpy(), oa[k])
        assert np.array_equal(rb[k].cpu().numpy(), ob[k])


@pytest.mark.parametrize("dtype", [np.uint8, np.uint16, np.float32])
@pytest.mark.parametrize("ndim", [2, 3])
def test_misaligned_base_and_buffer_end(ctx, dtype, ndim):
    """Fields that start one element into an allocation (unaligned vector loads)
    and whose last row ends exactly at the end of the buffer view (loads
    clamped to the buffer end and shifted back)."""
    import torch
    import oracle
    rng = np.random.default_rng(21 + ndim)
    shape = (97, 200) if ndim == 2 else (5, 7, 130)
    for sh in (shape, (3, 5) if ndim == 2 else (2, 1, 3)):
        n = int(np.prod(sh))
        if dtype == np.float32:
            a = rng.normal(size=sh).astype(np.float32)
            thr, L = np.linspace(-2, 2, 60).astype(np.float32), 60
        else:
            a = rng.integers(0, 60, size=sh).astype(dtype)
            thr, L = None, 50
        flat = torch.zeros(n + 1, dtype=getattr(torch, np.dtype(dtype).name)).cuda()
        flat[1:] = torch.from_numpy(a.ravel()).cuda()
        view = flat[1:].view(*sh)
        print(f"[case] misaligned ndim={ndim} dtype={np.dtype(dtype).name} shape={sh}", flush=True)
        ch = None if ndim == 2 else ("ec", "area", "volume")
        got = ctx.compute(view, L, thresholds=thr, channels=ch)
        torch.cuda.synchronize()
        ref = oracle.o2_curves(a, L, thresholds=thr, connectivity=8 if ndim == 2 else 26, channels=tuple(got))
        for k in got:
            assert np.array_equal(got[k].cpu().numpy(), ref[k]), (sh, k)


def test_first_call_of_fresh_context_on_side_stream():
    """The very first call of a new context, queued on a side stream, is exact
    (the context's one-time device state is ready before any stream uses it)."""
    import torch
    import oracle
    from paper_2311_11740_amd import ecc
    rng = np.random.default_rng(14)
    a = rng.integers(0, 300, size=(37, 13, 27)).astype(np.uint16)
    b = rng.integers(0, 256, size=(300, 500)).astype(np.uint8)
    print("[case] fresh context, side stream", flush=True)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        da, db = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    s.synchronize()
    c = ecc.Context(0)
    try:
        with torch.cuda.stream(s):
            ra = c.compute(da, 256, connectivity=26, stream=s)
            rb = c.compute(db, 256, stream=s)
        s.synchronize()
    finally:
        c.close()
    oa, ob = oracle.o2_curves(a, 256, connectivity=26), oracle.o2_curves(b, 256)
    for k in ra:
        assert np.array_equal(ra[k].cpu().numpy(), oa[k]), k
    for k in rb:
        assert np.array_equal(rb[k].cpu().numpy(), ob[k]), k


def test_stream_switch_keeps_calls_ordered():
    """A context's calls on one stream record no ordering events; the first
    call on a second stream (queued while the first stream is still busy) and
    the calls that alternate between the two afterwards are all exact."""
    import torch
    import oracle
    from paper_2311_11740_amd import ecc, synth
    vol = synth.quantise(synth.grf((96, 128, 256), 3.0, 31), 4096)
    imgs = [synth.quantise(synth.grf((700 + 37 * i, 900 - 41 * i), 4.0, 40 + i), 256) for i in range(5)]
    print("[case] stream switch: 3D then 2D fields alternating over two streams", flush=True)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    dv = torch.from_numpy(vol).cuda()
    di = [torch.from_numpy(a).cuda() for a in imgs]
    torch.cuda.synchronize()
    c = ecc.Context(0)
    try:
        got = []
        with torch.cuda.stream(s1):
            got.append(c.compute(dv, 4096, connectivity=26, stream=s1, channels=("ec", "area", "volume")))
            got.append(c.compute(di[0], 256, stream=s1))
        for i in range(1, 5):  # no host synchronisation between the calls
            s = s2 if i % 2 else s1
            with torch.cuda.stream(s):
                got.append(c.compute(di[i], 256, stream=s))
        with torch.cuda.stream(s2):
            got.append(c.compute(dv, 4096, connectivity=26, stream=s2, channels=("ec", "area", "volume")))
        torch.cuda.synchronize()
    finally:
        c.close()
    ref3 = oracle.o2_curves(vol, 4096, connectivity=26, channels=("ec", "area", "volume"))
    refs = [ref3] + [oracle.o2_curves(a, 256) for a in imgs] + [ref3]
    for k, (g, r) in enumerate(zip(got, refs)):
        for ch in g:
            assert np.array_equal(g[ch].cpu().numpy(), r[ch]), (k, ch)


def test_threshold_cache_eviction_on_one_stream():
    """More distinct threshold arrays than the cache holds, queued on one
    stream with no host synchronisation: evictions wait for the stream, and
    every result is exact."""
    import torch
    import oracle
    from paper_2311_11740_amd import ecc
    rng = np.random.default_rng(32)
    n = 300
    fields = [rng.normal(size=(40, 70)).astype(np.float32) for _ in range(n)]
    thrs = [np.sort(rng.normal(size=12)).astype(np.float32) for _ in range(n)]
    print(f"[case] {n} distinct threshold arrays on one stream", flush=True)
    dev = [torch.from_numpy(a).cuda() for a in fields]
    torch.cuda.synchronize()
    c = ecc.Context(0)
    try:
        got = [c.compute(dev[i], 12, thresholds=thrs[i]) for i in range(n)]
        torch.cuda.synchronize()
    finally:
        c.close()
    for i in range(n):
        ref = oracle.o2_curves(fields[i], 12, thresholds=thrs[i])
        for ch in got[i]:
            assert np.array_equal(got[i][ch].cpu().numpy(), ref[ch]), (i, ch)

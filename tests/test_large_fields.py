"""Fields of 2^28 cells and more (against closed forms that hold at any size).

The atomic drain packs the boundary measure and the cell count of a level
into one 64-bit word for fields below 2^28 cells and keeps them apart above.
The larger fields are too big for the oracle, so their curves are checked
against the cubical complex of closed cells written out with numpy: a
k-dimensional cell of the complex (vertex, edge, face, ...) enters at the
minimum level of the pixels or voxels that share it, the Euler characteristic
is the alternating count of cells present (Sec. 2, the sublevel complex of
closed cells, 8- and 26-connectivity), the perimeter or surface counts the
(n-1)-cells with exactly one side in the set, and the area or volume counts
the n-cells.  The CPU test pins these closed forms to the oracle on small
fields; the GPU tests run the large fields through the library.
"""
from __future__ import annotations

import itertools

import numpy as np
import pytest


def closed_form_curves(z, L):
    """EC, boundary measure and cell count of {z <= l} for l < L (closed cells)."""
    n = z.ndim
    z = z.astype(np.uint16)
    p = np.full(tuple(s + 2 for s in z.shape), L, np.uint16)  # L: never enters
    p[(slice(1, -1),) * n] = z

    def cells(axes):
        """the entry level of every cell thin along `axes` (min over its 2^|axes| neighbours)"""
        lo = hi = None
        for corner in itertools.product((0, 1), repeat=len(axes)):
            sl = [slice(1, -1)] * n
            for a, c in zip(axes, corner):
                sl[a] = slice(0, -1) if c == 0 else slice(1, None)
            v = p[tuple(sl)]
            lo = v if lo is None else np.minimum(lo, v)
            hi = v if hi is None else np.maximum(hi, v)
        return lo, hi

    def cumulative(v):
        return np.cumsum(np.bincount(v.ravel(), minlength=L + 1)[:L].astype(np.int64))

    ec = np.zeros(L, np.int64)
    boundary = np.zeros(L, np.int64)
    for k in range(n + 1):
        for axes in itertools.combinations(range(n), k):
            lo, hi = cells(axes)
            ec += (-1) ** (n - k) * cumulative(lo)
            if k == 1:  # (n-1)-cells: in the boundary for min <= l < max
                boundary += cumulative(lo) - cumulative(hi)
            del lo, hi
    area = cumulative(z)
    names = ("perimeter", "area") if n == 2 else ("area", "volume")
    return {"ec": ec, names[0]: boundary, names[1]: area}


@pytest.mark.parametrize("shape,L", [((37, 53), 16), ((64, 80), 256), ((5, 7), 4), ((9, 11, 13), 8),
                                     ((16, 12, 20), 64)])
def test_closed_forms_match_oracle(shape, L):
    import oracle
    z = np.random.default_rng(len(shape) * 100 + L).integers(0, L, size=shape).astype(np.uint8)
    cf = closed_form_curves(z, L)
    ref = oracle.o2_curves(z, L, connectivity=8 if z.ndim == 2 else 26, channels=tuple(cf), n_threads=4)
    for k in cf:
        assert np.array_equal(cf[k], ref[k]), (shape, k)


@pytest.mark.gpu
@pytest.mark.parametrize("shape", [(16384, 16384), (646, 646, 646)], ids=["2d_2^28", "3d_646^3"])
def test_gpu_unpacked_drain(shape):
    import torch
    from paper_2311_11740_amd import ecc
    assert np.prod(shape, dtype=np.int64) >= 1 << 28
    print(f"[case] large field {shape} u8, 256 levels", flush=True)
    # uniform values: every level holds boundary and count in every workgroup
    z = np.random.default_rng(5).integers(0, 256, size=shape, dtype=np.uint8)
    ctx = ecc.Context(0)
    try:
        got = ctx.compute(torch.from_numpy(np.ascontiguousarray(z)).cuda(), 256)
        torch.cuda.synchronize()
        got = {k: v.cpu().numpy() for k, v in got.items()}
    finally:
        ctx.close()
    ref = closed_form_curves(z, 256)
    for k in ref:
        assert np.array_equal(got[k], ref[k]), (shape, k, np.nonzero(got[k] != ref[k])[0][:4])

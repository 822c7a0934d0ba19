"""The paper's own benchmark inputs (Computational Results, Tables 3 and 4):
uniform and normal white noise translated to 0..255 at 1280 x 720,
1920 x 1080, 2048^2 and 4096^2 (2D, 8-connectivity, EC, perimeter and area)
and 128^3 and 256^3 (3D, 26-connectivity, EC, crease, surface and volume),
all 256 levels, in the launch configuration the benchmark times; every curve
against the all-levels oracle (O2).  White noise has the most events per level
of any input, the worst case for the LDS histograms.
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


@pytest.mark.parametrize("k", range(12))
def test_paper_workload(ctx, k):
    import torch
    import oracle
    from paper_2311_11740_amd import synth
    name = synth.PAPER_WORKLOADS[k][0]
    a = synth.paper_workload(k)
    conn = 8 if a.ndim == 2 else 26
    print(f"[case] {name} {a.shape} conn={conn}", flush=True)
    got = ctx.compute(torch.from_numpy(a).cuda(), 256, connectivity=conn)
    torch.cuda.synchronize()
    got = {c: v.cpu().numpy() for c, v in got.items()}
    ref = oracle.o2_curves(a, 256, connectivity=conn, channels=tuple(got), n_threads=NT)
    for c in got:
        bad = np.nonzero(got[c] != ref[c])[0]
        assert bad.size == 0, f"{name} {c}: {bad.size} levels differ, first {bad[:1]}"

"""Serving form: continuous batching of host requests.

* A mix of 2D and 3D requests (several dtypes and level modes, one with more
  than 4096 levels) submitted as fast as the server admits them: every result
  equals the oracle's.
* A request's result is the same alone and in the middle of a mix.
* Admission by memory: with a small budget, requests that do not fit are
  refused with BUSY and admitted later; one larger than the whole budget is
  rejected outright; the server's results stay exact throughout.
* Thresholds: many thresholded float32 requests ready at once (each with its
  own copy of an array), more distinct arrays than the context caches, and one
  array shared by the batched 2D stream and the single-field 3D stream.
"""
from __future__ import annotations

import os
import time

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


def oracle(a, L, thr, conn, channels):
    import oracle as O
    return O.o2_curves(a, L, thresholds=thr, connectivity=conn, channels=channels, n_threads=NT)


def serve_all(srv, reqs, timeout=60.0):
    """Submit every request (retrying on BUSY), poll until all complete."""
    results = [None] * len(reqs)
    tickets = {}
    nxt = 0
    busy = 0
    t0 = time.time()
    while (nxt < len(reqs) or tickets) and time.time() - t0 < timeout:
        while nxt < len(reqs):
            a, L, thr, conn = reqs[nxt]
            t = srv.submit(a, L, thresholds=thr, connectivity=conn)
            if t is None:
                busy += 1
                break
            tickets[t] = nxt
            nxt += 1
        for t in list(tickets):
            r = srv.poll(t)
            if r is not None:
                results[tickets.pop(t)] = r
        time.sleep(0.0002)
    assert nxt == len(reqs) and not tickets, "requests did not complete in time"
    return results, busy


def mixed_requests(rng, n):
    from paper_2311_11740_amd import synth
    thr_f = synth.linspace_thresholds(-3, 3, 200)
    reqs = []
    for k in range(n):
        kind = k % 5
        if kind in (0, 1):
            h, w = (int(x) for x in rng.integers(20, 600, size=2))
            reqs.append((synth.quantise(synth.grf((h, w), 3.0, int(rng.integers(1 << 30))), 256), 256, None,
                         8 if kind == 0 else 4))
        elif kind == 2:
            d, h, w = (int(x) for x in rng.integers(4, 40, size=3))
            reqs.append((rng.integers(0, 300, size=(d, h, w)).astype(np.uint16), 256, None, 26))
        elif kind == 3:
            z = synth.grf((int(rng.integers(10, 300)), int(rng.integers(10, 300))), 4.0, int(rng.integers(1 << 30)))
            reqs.append((z, 200, thr_f, 8))
        else:
            reqs.append((rng.integers(0, 6000, size=(37, 91)).astype(np.uint16), 5000, None, 8))
    return reqs


def check(results, reqs, tag):
    for i, ((a, L, thr, conn), got) in enumerate(zip(reqs, results)):
        ref = oracle(a, L, thr, conn, tuple(got))
        for k in got:
            assert np.array_equal(got[k], ref[k]), f"{tag}: request {i} {a.shape} {a.dtype} channel {k}"


def test_serving_mixed_exact(ctx):
    from paper_2311_11740_amd import ecc
    rng = np.random.default_rng(300)
    reqs = mixed_requests(rng, 60)
    print(f"[case] serving mixed n={len(reqs)}", flush=True)
    srv = ecc.Server(ctx, 256 << 20, max_slots=64, max_batch=32)
    try:
        results, _ = serve_all(srv, reqs)
        srv.drain()
    finally:
        srv.close()
    check(results, reqs, "mixed")


def test_serving_alone_equals_in_mix(ctx):
    from paper_2311_11740_amd import ecc, synth
    rng = np.random.default_rng(301)
    probe = (synth.quantise(synth.grf((333, 517), 5.0, 9), 256), 256, None, 8)
    probe3 = (rng.integers(0, 1000, size=(30, 41, 77)).astype(np.uint16), 1000, None, 26)
    print("[case] serving alone vs in mix", flush=True)
    srv = ecc.Server(ctx, 512 << 20, max_slots=128, max_batch=64)
    try:
        alone, _ = serve_all(srv, [probe, probe3])
        mix = mixed_requests(rng, 40)
        reqs = mix[:20] + [probe] + mix[20:] + [probe3]
        in_mix, _ = serve_all(srv, reqs)
    finally:
        srv.close()
    for k in alone[0]:
        assert np.array_equal(alone[0][k], in_mix[20][k]), k
    for k in alone[1]:
        assert np.array_equal(alone[1][k], in_mix[-1][k]), k
    check(alone, [probe, probe3], "alone")
    check(in_mix, reqs, "in_mix")


def test_serving_admission_by_memory(ctx):
    from paper_2311_11740_amd import ecc
    rng = np.random.default_rng(302)
    budget = 1 << 20  # 1 MiB: one of the requests below (0.5-0.7 MB each) at a time
    reqs = [(rng.integers(0, 256, size=(int(rng.integers(700, 800)), int(rng.integers(700, 900)))).astype(np.uint8),
             256, None, 8) for _ in range(40)]
    print("[case] serving admission, 1 MiB budget", flush=True)
    srv = ecc.Server(ctx, budget, max_slots=8, max_batch=8)
    try:
        with pytest.raises(ecc.EccError) as ei:
            srv.submit(np.zeros((1100, 1100), np.uint8), 256)  # more than the whole budget
        assert ei.value.status == ecc.ECC_ERR_INVALID_ARG
        results, busy = serve_all(srv, reqs)
    finally:
        srv.close()
    assert busy > 0, "the budget never refused a request"
    check(results, reqs, "admission")


def test_serving_many_thresholded_requests(ctx):
    """More thresholded float32 2D requests ready at once than one launch of
    the batched kernel used to take (each request carries its own copy of one
    of three threshold arrays), then more distinct arrays than the context
    caches at once: every request completes and equals the oracle."""
    from paper_2311_11740_amd import ecc, synth
    rng = np.random.default_rng(303)
    thr_sets = [synth.linspace_thresholds(-3, 3, 64), synth.linspace_thresholds(-2, 2.5, 100),
                np.sort(rng.normal(size=50)).astype(np.float32)]
    reqs = []
    for k in range(120):
        thr = thr_sets[k % 3]
        h, w = (int(x) for x in rng.integers(8, 64, size=2))
        reqs.append((rng.normal(size=(h, w)).astype(np.float32), len(thr), thr.copy(), 8 if k % 2 else 4))
    print(f"[case] serving {len(reqs)} thresholded f32 requests, max_batch 256", flush=True)
    srv = ecc.Server(ctx, 256 << 20, max_slots=256, max_batch=256)
    try:
        results, _ = serve_all(srv, reqs)
        srv.drain()
        many = []
        for k in range(300):  # 300 distinct arrays: more than the 256 cached at once
            thr = np.sort(rng.normal(size=int(rng.integers(5, 40)))).astype(np.float32)
            many.append((rng.normal(size=(int(rng.integers(4, 30)), int(rng.integers(4, 30)))).astype(np.float32),
                         len(thr), thr, 8))
        print(f"[case] serving {len(many)} requests with distinct threshold arrays", flush=True)
        results2, _ = serve_all(srv, many, timeout=120.0)
        srv.drain()
    finally:
        srv.close()
    check(results, reqs, "thresholded")
    check(results2, many, "distinct_thresholds")


def test_serving_shared_thresholds_2d_and_3d(ctx):
    """One threshold array used by batched 2D float32 requests and by 3D
    requests on the single-field stream (float32, and uint16 with its
    value -> level table), submitted interleaved, twice over."""
    from paper_2311_11740_amd import ecc, synth
    rng = np.random.default_rng(304)
    thr = synth.linspace_thresholds(-2.5, 2.5, 150)
    thr_int = np.linspace(0.5, 900.5, 150).astype(np.float32)
    reqs = []
    for k in range(40):
        kind = k % 4
        if kind in (0, 1):
            h, w = (int(x) for x in rng.integers(16, 200, size=2))
            reqs.append((synth.grf((h, w), 3.0, int(rng.integers(1 << 30))), 150, thr.copy(), 8))
        elif kind == 2:
            d, h, w = (int(x) for x in rng.integers(4, 30, size=3))
            reqs.append((synth.grf((d, h, w), 2.0, int(rng.integers(1 << 30))), 150, thr.copy(), 26))
        else:
            d, h, w = (int(x) for x in rng.integers(4, 30, size=3))
            reqs.append((rng.integers(0, 1000, size=(d, h, w)).astype(np.uint16), 150, thr_int.copy(), 26))
    print(f"[case] serving shared thresholds 2D+3D n={len(reqs)}", flush=True)
    srv = ecc.Server(ctx, 256 << 20, max_slots=64, max_batch=64)
    try:
        res_a, _ = serve_all(srv, reqs)
        res_b, _ = serve_all(srv, reqs[::-1])
        srv.drain()
    finally:
        srv.close()
    check(res_a, reqs, "shared_thresholds")
    check(res_b, reqs[::-1], "shared_thresholds_rev")

#!/usr/bin/env python3
"""EC-curve throughput on one MI355X.

A step is one ecc_curves_compute over one synthetic field already resident in
HBM: level index, per-cell vertex-contribution deltas, workgroup histograms,
merge and prefix scan.  Consecutive steps read different copies of the field
(4 copies by default, more than the 256 MB last-level cache) so every step
streams its field from HBM.

Default workload: 2D 8192 x 8192 float32 smoothed Gaussian random field
(sigma 16 px), 1024 thresholds on [-4, 4], 8-connectivity, EC + perimeter +
area curves.  `--workload 3d` runs the 512^3 uint16 volume (4096 levels, 26-C,
EC + surface + volume).  The default run also measures the 3D volume as a
secondary figure.

Prints one JSON line (rank 0).  The roofline object uses the field-reading
kernel's own duration, timed with HIP events on the stream it is launched on.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "EC-curve Gvoxels/s & % HBM peak; batched vs per-field launch; p99 latency"


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for name in ("ecc_device.h", "ecc_k2d.hip", "ecc_k3d.hip", "ecc_kmerge.hip", "ecc_internal.h"):
        with open(os.path.join(ROOT, "paper_2311_11740_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_profile(kernel: str, workload: str):
    """HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE runs) and the
    kernel's average duration under rocprofv3 --kernel-trace, from the
    committed profiles, if they were taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None, None
    try:
        with open(path) as f:
            d = json.load(f)
        e = d.get(workload, {})
        if e.get("kernel") == kernel and e.get("source_hash") == kernel_source_hash():
            return e.get("bytes_per_launch"), e.get("kernel_avg_us")
    except (OSError, ValueError):
        pass
    return None, None


def make_workload(name: str):
    from paper_2311_11740_amd import synth
    if name == "2d":
        return synth.large_2d_f32()
    if name == "3d":
        return synth.large_3d_u16()
    if name == "2d-small":
        return synth.small_2d_u8()
    raise ValueError(name)


def channels_for(spec):
    return ("ec", "perimeter", "area") if spec.data.ndim == 2 else ("ec", "area", "volume")


def time_field(ctx, spec, steps: int, warmup: int, copies: int):
    """Whole-call time per step (no profiling events in the stream), then the
    field-reading kernel's own time per launch from HIP events around it."""
    import torch
    dev0 = torch.from_numpy(spec.data).cuda()
    bufs = [dev0] + [dev0.clone() for _ in range(copies - 1)]
    ch = channels_for(spec)
    out = {c: torch.empty(spec.n_levels, dtype=torch.int64, device="cuda") for c in ch}
    thr = spec.thresholds
    stream = torch.cuda.current_stream()

    def run(i):
        ctx.compute(bufs[i % copies], spec.n_levels, thresholds=thr, connectivity=spec.connectivity,
                    out=out, stream=stream)

    for i in range(warmup):
        run(i)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t0.record(stream)
    for i in range(steps):
        run(i)
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    total_ms = t0.elapsed_time(t1)
    ctx.profile(True)
    ctx.profile_read(reset=True)
    for i in range(steps):
        run(i)
    torch.cuda.synchronize()
    k_ms, k_n = ctx.profile_read(reset=True)
    ctx.profile(False)
    res = {c: v.cpu().numpy() for c, v in out.items()}
    del bufs
    return dict(ms_per_step=total_ms / steps, wall_s=wall, kernel_ms=k_ms / max(k_n, 1),
                kernel_ms_per_step=k_ms / steps, kernel_launches=k_n, curves=res)


def host_cpu():
    """CPU model, logical CPUs of the host and those this process may run on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return model, os.cpu_count() or 1, usable


def cpu_baseline(spec, gpu_curves):
    """The oracle timed on the host: the all-levels C oracle on the whole field
    with one thread per usable CPU (the reported value, also the parity check
    of the full curves), the same oracle single-threaded on the first 2048 rows,
    and the per-level oracle on the 256 x 256 uint8 field at all 256 levels."""
    import oracle
    from paper_2311_11740_amd import synth
    model, nproc, usable = host_cpu()
    t = time.perf_counter()
    ref = oracle.o2_curves(spec.data, spec.n_levels, thresholds=spec.thresholds,
                           connectivity=spec.connectivity, channels=tuple(gpu_curves), n_threads=usable)
    dt = time.perf_counter() - t
    ok = all((ref[c] == gpu_curves[c]).all() for c in gpu_curves)
    cells = spec.data.size
    part = np.ascontiguousarray(spec.data[:2048])
    t = time.perf_counter()
    oracle.o2_curves(part, spec.n_levels, thresholds=spec.thresholds, connectivity=spec.connectivity,
                     channels=tuple(gpu_curves), n_threads=1)
    dt1 = time.perf_counter() - t
    small = synth.small_2d_u8()
    t = time.perf_counter()
    oracle.o1_curves(small.data, small.n_levels, connectivity=8)
    dt_o1 = time.perf_counter() - t
    return dict(value=round(cells / dt / 1e9, 4), unit="Gvoxels/s", cores=usable, kind="oracle",
                sample=f"whole field ({'x'.join(map(str, spec.data.shape))}, all {spec.n_levels} levels), "
                       f"all-levels C oracle, {usable} threads, one run of {dt:.2f} s",
                cpu_model=model, nproc=nproc,
                single_thread=dict(value=round(part.size / dt1 / 1e9, 4), unit="Gvoxels/s", cores=1,
                                   sample=f"rows 0-2047 of the field ({part.size} cells), one run of {dt1:.2f} s"),
                per_level_oracle_c1=dict(value=round(small.data.size * small.n_levels / dt_o1 / 1e9, 5),
                                         unit="Gvoxel-levels/s", cores=1,
                                         sample=f"256 x 256 uint8, all 256 levels binarised and counted, "
                                                f"{dt_o1:.2f} s")), ok


def measure(ctx, spec, steps, warmup, copies, with_cpu):
    r = time_field(ctx, spec, steps, warmup, copies)
    cells = spec.data.size
    elem = spec.data.dtype.itemsize
    value = cells / (r["ms_per_step"] / 1e3) / 1e9
    kernel = "ecc2d_stream" if spec.data.ndim == 2 else "ecc3d_stream"
    alg_bytes = cells * elem  # the field-reading kernel reads every cell once per step
    launches_per_step = r["kernel_launches"] / max(1, steps)
    achieved = alg_bytes / (r["kernel_ms_per_step"] / 1e3) / 1e9
    traffic, prof_us = load_profile(kernel, spec.meta["name"])
    out = dict(
        workload=spec.meta["name"], cells=cells, bytes=alg_bytes,
        gvox_s=round(value, 3), ms_per_step=round(r["ms_per_step"], 4),
        hbm_frac_step=round(alg_bytes / (r["ms_per_step"] / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
        roofline=dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                      frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic, kernel=kernel,
                      kernel_ms_per_launch=round(r["kernel_ms"], 4),
                      timing="HIP events passed to the kernel's own dispatch (hipExtLaunchKernel) on its "
                             "stream; the interval also holds the marker packets HIP adds for the events "
                             "(rocprofv3 shows them as 4-5 us between dispatches), so it is longer than "
                             "the kernel's duration under rocprofv3 (rocprof_kernel_us)",
                      rocprof_kernel_us=prof_us,
                      launches_per_step=launches_per_step,
                      alg_bytes_per_launch=int(alg_bytes / launches_per_step)),
        spec=spec, curves=r["curves"])
    if with_cpu:
        cb, ok = cpu_baseline(spec, r["curves"])
        out["cpu_baseline"] = cb
        out["parity_vs_oracle"] = bool(ok)
    return out


def measure_vertex_classes(ctx, spec, steps, warmup, copies, curves):
    """The contribution map (vertex counts per Table 1 class and level) of the
    main 2D field: per-call time with the field in HBM, the class-count
    kernel's own time, and the check that its Table 1 weightings reproduce the
    main run's EC, perimeter and area curves."""
    import numpy as np
    import torch
    dev0 = torch.from_numpy(spec.data).cuda()
    bufs = [dev0] + [dev0.clone() for _ in range(copies - 1)]
    out = torch.empty((5, spec.n_levels), dtype=torch.int64, device="cuda")
    it = [0]

    def call(stream):
        ctx.vertex_classes(bufs[it[0] % copies], spec.n_levels, thresholds=spec.thresholds, out=out,
                           stream=stream)
        it[0] += 1

    for _ in range(warmup):
        call(torch.cuda.current_stream())
    ms, _ = timed_calls(call, steps)
    ctx.profile(True)
    ctx.profile_read(reset=True)
    for _ in range(steps):
        call(torch.cuda.current_stream())
    torch.cuda.synchronize()
    k_ms, k_n = ctx.profile_read(reset=True)
    ctx.profile(False)
    one, adj, diag, three, four = out.cpu().numpy()
    ok = (np.array_equal(one - 2 * diag - three, 4 * curves["ec"]) and
          np.array_equal(2 * one + 2 * adj + 4 * diag + 2 * three, 2 * curves["perimeter"]) and
          np.array_equal(one + 2 * adj + 2 * diag + 3 * three + 4 * four, 4 * curves["area"]))
    cells = spec.data.size
    alg = cells * spec.data.dtype.itemsize
    kern = k_ms / max(k_n, 1)
    del bufs
    return dict(workload=spec.meta["name"], classes=["one", "adjacent", "diagonal", "three", "four"],
                ms_per_call=round(ms, 4), gvox_s=round(cells / ms / 1e6, 2),
                kernel="ecc2d_stream (class counts)", kernel_ms_per_launch=round(kern, 4),
                kernel_hbm_frac=round(alg / (kern / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                weightings_equal_curves=bool(ok))


def measure_vertex_classes_3d(ctx, spec, curves, steps=3):
    """The 3D contribution map (21 octant classes) of a volume: per-call time
    with the volume in HBM, and the check that weighting the class counts by
    the library's per-vertex table (Table 2, x8) gives the EC (26-C), surface
    and volume curves of the curves call."""
    import numpy as np
    import torch
    from paper_2311_11740_amd import ecc
    dev = torch.from_numpy(spec.data).cuda()
    out = torch.empty((21, spec.n_levels), dtype=torch.int64, device="cuda")

    def call(stream):
        ctx.vertex_classes(dev, spec.n_levels, thresholds=spec.thresholds, out=out, stream=stream)

    call(torch.cuda.current_stream())
    ms, _ = timed_calls(call, steps)
    n = out.cpu().numpy()
    vt = np.array(ecc.vertex_table(3, spec.connectivity), dtype=np.int64)  # [256][4] x8 EC, x2 crease, x4 surface, x8 vol
    cls = np.array(ecc.vertex_class_table(3))
    rep = {c: int(np.nonzero(cls == c)[0][0]) for c in range(21)}
    w = np.array([vt[rep[c]] for c in range(21)])  # per-class contributions
    ok = (np.array_equal((w[:, 0:1] * n).sum(0), 8 * curves["ec"]) and
          np.array_equal((w[:, 2:3] * n).sum(0), 4 * curves["area"]) and
          np.array_equal((w[:, 3:4] * n).sum(0), 8 * curves["volume"]))
    cells = spec.data.size
    return dict(workload=spec.meta["name"], classes=21, ms_per_call=round(ms, 3),
                gvox_s=round(cells / ms / 1e6, 2), weightings_equal_curves=bool(ok))


def measure_streamed(ctx, spec, curves, steps=3, slab_mib=64):
    """The main field from host memory through ecc_curves_compute_streamed
    (slabs of slab_mib MiB, copies overlapped with the slab kernels), from
    pageable and from pinned host memory, against uploading the whole field
    and then computing.  Host-to-device copies are inside every time here."""
    import numpy as np
    import torch
    a = np.ascontiguousarray(spec.data)
    pinned_t = torch.empty(a.shape, dtype=torch.from_numpy(a[:1]).dtype, pin_memory=True)
    pinned = pinned_t.numpy()
    pinned[...] = a
    res = {"workload": spec.meta["name"], "slab_mib": slab_mib, "field_bytes": int(a.nbytes)}
    ok = True
    for name, host in (("pageable", a), ("pinned", pinned)):
        out = None
        ctx.compute_streamed(host, spec.n_levels, thresholds=spec.thresholds, connectivity=spec.connectivity,
                             slab_bytes=slab_mib << 20)
        t0 = time.perf_counter()
        for _ in range(steps):
            out = ctx.compute_streamed(host, spec.n_levels, thresholds=spec.thresholds,
                                       connectivity=spec.connectivity, slab_bytes=slab_mib << 20)
        ms = (time.perf_counter() - t0) * 1e3 / steps
        ok = ok and all(np.array_equal(out[k], curves[k]) for k in curves)
        res[name] = dict(ms_per_call=round(ms, 2), gvox_s=round(a.size / ms / 1e6, 2),
                         host_gb_s=round(a.nbytes / ms / 1e6, 2))
    # the copy alone: the whole field from pinned memory in one transfer
    dst = torch.empty(pinned_t.shape, dtype=pinned_t.dtype, device="cuda")
    dst.copy_(pinned_t, non_blocking=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        dst.copy_(pinned_t, non_blocking=True)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    res["pinned_copy_only"] = dict(ms_per_call=round(ms, 2), host_gb_s=round(a.nbytes / ms / 1e6, 2))
    del dst
    t0 = time.perf_counter()
    for _ in range(steps):
        dev = torch.from_numpy(a).cuda()
        c = ctx.compute(dev, spec.n_levels, thresholds=spec.thresholds, connectivity=spec.connectivity)
        {k: v.cpu() for k, v in c.items()}
        del dev
    ms = (time.perf_counter() - t0) * 1e3 / steps
    res["upload_then_compute_pageable"] = dict(ms_per_call=round(ms, 2), gvox_s=round(a.size / ms / 1e6, 2))
    res["equal_to_device_curves"] = bool(ok)
    del pinned, pinned_t
    return res


def timed_calls(fn, steps):
    """(ms per call on the GPU clock, ms per call on the host clock) of `steps` calls."""
    import torch
    stream = torch.cuda.current_stream()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    t0.record(stream)
    for _ in range(steps):
        fn(stream)
    t1.record(stream)
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / steps, (time.perf_counter() - w0) * 1e3 / steps


def measure_batch(ctx, specs, steps, warmup, workload=None):
    """Batched call vs one call per field over the same fields (already in HBM)."""
    import numpy as np
    import torch
    import oracle
    sizes = [s.data.size for s in specs]
    offs = np.cumsum([0] + sizes)
    host = np.empty(int(offs[-1]), np.uint8)
    for i, s in enumerate(specs):
        host[offs[i]:offs[i + 1]] = s.data.ravel()
    dev = torch.from_numpy(host).cuda()
    views = [dev[int(offs[i]):int(offs[i + 1])].view(*specs[i].data.shape) for i in range(len(specs))]
    L = specs[0].n_levels
    conn = specs[0].connectivity
    b = ctx.batch(views, L, connectivity=conn)
    ref = ctx.batch(views, L, connectivity=conn)
    for _ in range(warmup):
        ref.run_per_field(torch.cuda.current_stream())
    pf_ms, pf_wall = timed_calls(ref.run_per_field, max(3, steps // 4))
    for _ in range(warmup):
        b.run(torch.cuda.current_stream())
    ctx.profile(True)
    ctx.profile_read(reset=True)
    bd_ms, bd_wall = timed_calls(b.run, steps)
    k_ms, k_n = ctx.profile_read(reset=True)
    ctx.profile(False)
    equal_default = bool(torch.equal(b.buffer, ref.buffer))
    t = time.perf_counter()
    b.tune(torch.cuda.current_stream())
    tune_s = time.perf_counter() - t
    b.buffer.zero_()
    for _ in range(warmup):
        b.run(torch.cuda.current_stream())
    ctx.profile(True)
    ctx.profile_read(reset=True)
    bt_ms, bt_wall = timed_calls(b.run, steps)
    kt_ms, kt_n = ctx.profile_read(reset=True)
    ctx.profile(False)
    torch.cuda.synchronize()
    equal = equal_default and bool(torch.equal(b.buffer, ref.buffer))
    # a sample of the fields against the oracle
    sample = list(range(0, len(specs), max(1, len(specs) // 16)))
    ok = True
    for i in sample:
        r = oracle.o2_curves(specs[i].data, L, connectivity=conn, channels=tuple(b.outputs[i]),
                             n_threads=min(16, os.cpu_count() or 1))
        ok &= all(np.array_equal(b.outputs[i][c].cpu().numpy(), r[c]) for c in r)
    px = float(sum(sizes))
    best = min(bd_ms, bt_ms)
    return dict(lane_occupancy=lane_occupancy(specs), **dict(
        workload=workload or f"batch_{len(specs)}x_u8_side64-2048_L{L}", fields=len(specs),
        gpx=round(px / 1e9, 4),
        per_field_ms=round(pf_ms, 3), per_field_host_ms=round(pf_wall, 3),
        batched_ms=round(bd_ms, 3), batched_tuned_ms=round(bt_ms, 3), batched_host_ms=round(bt_wall, 3),
        per_field_gvox_s=round(px / pf_ms / 1e6, 2), batched_gvox_s=round(px / best / 1e6, 2),
        speedup=round(pf_ms / best, 2),
        batched_kernel_ms=round((kt_ms / max(kt_n, 1)) if bt_ms <= bd_ms else (k_ms / max(k_n, 1)), 4),
        hbm_frac_batched=round(px / best / 1e6 / HBM_PEAK_GBS, 4),
        tune_seconds=round(tune_s, 2), equal_to_per_field=equal, parity_vs_oracle_sample=bool(ok),
        oracle_sample_fields=len(sample)))


def lane_occupancy(specs):
    """Share of the batched kernels' lane slots that hold cells of the fields.
    2D: a wave covers a strip of 64 lanes x one 16-byte block per row (lanes 0
    and 63 only load the neighbouring columns), so a field of width w fills
    w / (ceil(w / (62 VEC)) * 64 VEC) of its lane slots (VEC cells per 16
    bytes).  3D: tiles of the tile pass; reported for 2D batches only."""
    cells = slots = 0
    for s in specs:
        a = s.data
        if a.ndim != 2:
            return None
        vec = 16 // a.dtype.itemsize
        h, w = a.shape
        strips = -(-w // (62 * vec))
        cells += h * w
        slots += h * strips * 64 * vec
    return round(cells / slots, 4) if slots else None


# The paper's own synthetic workloads (white noise translated to 0..255, 8-C
# in 2D and 26-C in 3D) and its 24-core CPU throughput for them (Computational
# Results, Tables 3 and 4), as context for the same inputs here.


def measure_4d(ctx, spec, small, steps=10):
    """A 4D field (a, d, h, w) per call, both constructions, field in HBM; a
    small 4D field of the same recipe is checked against the any-dimension
    oracle (the large one is too big for it)."""
    import numpy as np
    import torch
    from oracle import ec_oracle_nd as ND
    out = {"workload": spec.meta["name"], "cells": int(spec.data.size)}
    dev = torch.from_numpy(spec.data).cuda()
    sdev = torch.from_numpy(small.data).cuda()
    for conn in (80, 8):
        for _ in range(2):
            ctx.compute_4d(dev, spec.n_levels, connectivity=conn)
        ms, _ = timed_calls(lambda s: ctx.compute_4d(dev, spec.n_levels, connectivity=conn, stream=s), steps)
        got = ctx.compute_4d(sdev, small.n_levels, connectivity=conn)
        torch.cuda.synchronize()
        ref = ND.curves_all_levels(small.data, small.n_levels, None, conn)
        ok = all(np.array_equal(got[k].cpu().numpy(), ref[k]) for k in ref)
        out[f"{conn}c"] = dict(ms_per_call=round(ms, 4), gcells_s=round(spec.data.size / ms / 1e6, 2),
                               parity_vs_oracle_small=bool(ok), small_field=list(small.data.shape))
    return out


def measure_paper_workloads(ctx, steps):
    """Per-call throughput on the paper's white-noise inputs (field resident in
    HBM, all 256 levels, every output channel the paper computes: EC,
    perimeter and area in 2D; EC, perimeter (crease), surface and volume in 3D,
    and in 3D also without the crease measure), checked against the oracle."""
    import torch
    import oracle
    from paper_2311_11740_amd import synth
    rows = []
    for k, (name, shape, kind, paper_mps, table) in enumerate(synth.PAPER_WORKLOADS):
        a = synth.paper_workload(k)
        dev = torch.from_numpy(a).cuda()
        conn = 8 if a.ndim == 2 else 26
        variants = [None] if a.ndim == 2 else [None, ("ec", "area", "volume")]
        row = dict(workload=name, cells=int(a.size), paper_cpu_24_cores_mcells_s=paper_mps, paper_source=table)
        for ch in variants:
            out = ctx.compute(dev, 256, connectivity=conn, channels=ch)

            def call(stream, _ch=ch, _out=out):
                ctx.compute(dev, 256, connectivity=conn, channels=_ch, out=_out, stream=stream)

            for _ in range(3):
                call(torch.cuda.current_stream())
            ms, _ = timed_calls(call, steps)
            got = {c: v.cpu().numpy() for c, v in out.items()}
            ref = oracle.o2_curves(a, 256, connectivity=conn, channels=tuple(got),
                                   n_threads=min(16, os.cpu_count() or 1))
            ok = all(np.array_equal(got[c], ref[c]) for c in got)
            key = "all_channels" if ch is None else "no_crease"
            row[key] = dict(ms_per_call=round(ms, 4), gcells_s=round(a.size / ms / 1e6, 2),
                            x_paper=round(a.size / ms / 1e3 / paper_mps, 1), parity_vs_oracle=bool(ok))
        rows.append(row)
    return rows


def serve_trace(submit, poll, t_arr, ids, pool, warm):
    """Replay a Poisson trace: requests are offered at their arrival times,
    retried while the server is full, and polled until done.  Returns the
    latencies (s, arrival to result on the host) of the requests after the
    first `warm`, the elapsed time of those, and the results by request."""
    from collections import deque
    n = len(t_arr)
    lat = np.zeros(n)
    results = [None] * n
    backlog, pending = deque(), {}
    i = 0
    start = time.perf_counter()
    while i < n or backlog or pending:
        now = time.perf_counter() - start
        progressed = False
        while i < n and t_arr[i] <= now:
            backlog.append(i)
            i += 1
        while backlog:
            k = backlog[0]
            t = submit(pool[ids[k]])
            if t is None:
                break
            pending[t] = k
            backlog.popleft()
            progressed = True
        for t in list(pending):
            r = poll(t)
            if r is not None:
                k = pending.pop(t)
                lat[k] = time.perf_counter() - start - t_arr[k]
                results[k] = r
                progressed = True
        if not progressed:
            time.sleep(2e-5)
    elapsed = time.perf_counter() - start - t_arr[warm]
    return lat[warm:], elapsed, results


def measure_serving(ctx, pool, n_requests, rates, warm=100):
    """Continuous-batching server vs the plain path (copy in, one call, copy
    out, one request at a time) on the same Poisson traces."""
    import torch
    from paper_2311_11740_amd import ecc, synth
    n2d = sum(1 for p in pool if p.data.ndim == 2)
    ch = lambda p: ("ec", "perimeter", "area") if p.data.ndim == 2 else ("ec", "area", "volume")  # noqa: E731
    # reference curves of every pool field from the single-field call
    ref = []
    for p in pool:
        r = ctx.compute(torch.from_numpy(p.data).cuda(), p.n_levels, connectivity=p.connectivity, channels=ch(p))
        ref.append({c: v.cpu().numpy() for c, v in r.items()})
    srv = ecc.Server(ctx, 2 << 30, max_slots=256, max_batch=128)

    def srv_submit(p):
        return srv.submit(p.data, p.n_levels, connectivity=p.connectivity, channels=ch(p))

    plain_state = {}

    def plain_submit(p):  # synchronous: the request is complete when this returns
        d = torch.from_numpy(p.data).cuda()
        r = ctx.compute(d, p.n_levels, connectivity=p.connectivity, channels=ch(p))
        t = len(plain_state) + 1
        plain_state[t] = {c: v.cpu().numpy() for c, v in r.items()}
        return t

    out = []
    equal = True
    try:
        for rate in rates:
            t_arr, ids = synth.poisson_trace(n_requests + warm, rate, len(pool), 0.7, n2d)
            row = {"rate_rps": rate}
            for name, sub, pol in (("server", srv_submit, srv.poll),
                                   ("per_field", plain_submit, lambda t: plain_state.pop(t, None))):
                lat, el, res = serve_trace(sub, pol, t_arr, ids, pool, warm)
                vox = float(sum(pool[k].data.size for k in ids[warm:]))
                row[name] = dict(throughput_rps=round(n_requests / el, 1), gvox_s=round(vox / el / 1e9, 3),
                                 p50_ms=round(float(np.percentile(lat, 50)) * 1e3, 3),
                                 p99_ms=round(float(np.percentile(lat, 99)) * 1e3, 3))
                for k in range(len(res)):
                    equal &= all(np.array_equal(res[k][c], ref[ids[k]][c]) for c in res[k])
            out.append(row)
            print(f"[bench] serving {rate} req/s: {row}", file=sys.stderr, flush=True)
    finally:
        srv.close()
    return dict(workload=f"serving_pool{n2d}x2d_u8+{len(pool) - n2d}x3d_u16_poisson",
                requests_per_rate=n_requests, warmup_requests=warm, rates=out,
                results_equal_single_field=bool(equal))


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=["2d", "3d", "2d-small"], default="2d")
    ap.add_argument("--copies", type=int, default=4)
    ap.add_argument("--no-secondary", action="store_true", help="skip the 3D secondary measurement")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched vs per-field comparison")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving comparison")
    ap.add_argument("--no-streamed", action="store_true",
                    help="skip the host-resident (streamed in slabs) measurement")
    ap.add_argument("--no-vertex-classes", action="store_true",
                    help="skip the contribution-map (vertex class counts) measurement")
    ap.add_argument("--no-4d", action="store_true", help="skip the 4D field measurement")
    ap.add_argument("--no-paper-workloads", action="store_true",
                    help="skip the paper's white-noise workloads (context against its CPU timings)")
    ap.add_argument("--serving-requests", type=int, default=2000)
    ap.add_argument("--serving-rates", type=str, default="500,2000,4000,8000,16000",
                    help="Poisson arrival rates (requests/s), comma separated")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--gen-workers", type=int, default=min(16, os.cpu_count() or 1),
                    help="processes that draw the synthetic inputs")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="also run a plain device copy of MIB MiB (for counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the EC-curve path has no "
                                   "multi-GPU form in this build (see DESIGN.md for how it would shard)",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    # every host input is drawn before the GPU is touched
    from paper_2311_11740_amd import synth
    t_gen = time.perf_counter()
    spec = make_workload(args.workload)
    sec_spec = make_workload("3d") if args.workload == "2d" and not args.no_secondary else None
    batch_specs = None if args.no_batch else synth.batch_2d_u8(workers=args.gen_workers)
    grid_specs = None if args.no_batch else synth.batch_3d_grids(workers=args.gen_workers)
    f4 = None if args.no_4d else (synth.field_4d(), synth.field_4d((6, 10, 14, 18), seed=8))
    pool = None if args.no_serving else synth.serving_pool(workers=args.gen_workers)
    print(f"[bench] inputs drawn in {time.perf_counter() - t_gen:.1f} s", file=sys.stderr, flush=True)

    import torch
    from paper_2311_11740_amd import ecc
    ctx = ecc.Context(0)

    if args.calibrate_copy:
        n = args.calibrate_copy << 20
        a = torch.empty(n, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()

    main_r = measure(ctx, spec, args.steps, args.warmup, args.copies, with_cpu=not args.no_cpu_baseline)
    print(f"[bench] {spec.meta['name']}: {main_r['gvox_s']} Gvox/s", file=sys.stderr, flush=True)
    line = {
        "metric": METRIC,
        "value": main_r["gvox_s"],
        "unit": "Gvoxels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"float32": "f32", "uint8": "u8", "uint16": "u16"}[str(spec.data.dtype)],
        "data": "synthetic",
        "config": {"workload": spec.meta["name"], "shape": list(spec.data.shape),
                   "n_levels": spec.n_levels, "connectivity": spec.connectivity,
                   "channels": list(channels_for(spec)), "field_copies": args.copies,
                   "parallelism": "single-gpu"},
        "hbm_frac_step": main_r["hbm_frac_step"],
        "roofline": main_r["roofline"],
    }
    if "cpu_baseline" in main_r:
        line["cpu_baseline"] = main_r["cpu_baseline"]
        line["parity_vs_oracle"] = main_r["parity_vs_oracle"]
    if spec.data.ndim == 2 and spec.connectivity == 8 and not args.no_vertex_classes:
        line["vertex_classes"] = measure_vertex_classes(ctx, spec, args.steps, args.warmup, args.copies,
                                                        main_r["curves"])
        print(f"[bench] vertex classes: {line['vertex_classes']['gvox_s']} Gvox/s", file=sys.stderr, flush=True)
    if not args.no_streamed:
        line["streamed_from_host"] = measure_streamed(ctx, spec, main_r["curves"])
        print(f"[bench] streamed from host: {line['streamed_from_host']['pinned']['gvox_s']} Gvox/s (pinned)",
              file=sys.stderr, flush=True)
    del main_r
    if sec_spec is not None:
        sec = measure(ctx, sec_spec, max(3, args.steps // 2), 2, 2, with_cpu=False)
        line["secondary"] = {k: sec[k] for k in ("workload", "gvox_s", "ms_per_step", "hbm_frac_step",
                                                  "roofline")}
        if not args.no_vertex_classes:
            line["secondary"]["vertex_classes"] = measure_vertex_classes_3d(ctx, sec_spec, sec["curves"])
        print(f"[bench] {sec_spec.meta['name']}: {sec['gvox_s']} Gvox/s", file=sys.stderr, flush=True)
        del sec
    if batch_specs is not None:
        line["batched"] = measure_batch(ctx, batch_specs, max(5, args.steps // 2), 2)
        print(f"[bench] batched: {line['batched']['batched_gvox_s']} Gvox/s", file=sys.stderr, flush=True)
    if grid_specs is not None:
        line["batched_3d"] = measure_batch(ctx, grid_specs, max(5, args.steps // 2), 2,
                                           workload=f"batch_{len(grid_specs)}x_u8_20^3_L256_26c")
        print(f"[bench] batched 3D: {line['batched_3d']['batched_gvox_s']} Gvox/s "
              f"({line['batched_3d']['speedup']}x per-field)", file=sys.stderr, flush=True)
        del grid_specs
    if f4 is not None:
        line["field_4d"] = measure_4d(ctx, *f4)
        print(f"[bench] 4D: {line['field_4d']['80c']['gcells_s']} Gcells/s (80-C)", file=sys.stderr, flush=True)
        del f4
    if not args.no_paper_workloads:
        line["paper_workloads"] = measure_paper_workloads(ctx, max(5, args.steps // 2))
        print("[bench] paper workloads done", file=sys.stderr, flush=True)
    if pool is not None:
        del batch_specs
        rates = [float(r) for r in args.serving_rates.split(",") if r]
        line["serving"] = measure_serving(ctx, pool, args.serving_requests, rates)
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

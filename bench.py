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

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "EC-curve Gvoxels/s & % HBM peak; batched vs per-field launch; p99 latency"


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for name in ("ecc_kernels.hip", "ecc_internal.h"):
        with open(os.path.join(ROOT, "paper_2311_11740_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(kernel: str, workload: str):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were
    taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            d = json.load(f)
        e = d.get(workload, {})
        if e.get("kernel") == kernel and e.get("source_hash") == kernel_source_hash():
            return e.get("bytes_per_launch")
    except (OSError, ValueError):
        pass
    return None


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
    import torch
    dev0 = torch.from_numpy(spec.data).cuda()
    bufs = [dev0] + [dev0.clone() for _ in range(copies - 1)]
    ch = channels_for(spec)
    out = {c: torch.empty(spec.n_levels, dtype=torch.int64, device="cuda") for c in ch}
    thr = spec.thresholds
    for i in range(warmup):
        ctx.compute(bufs[i % copies], spec.n_levels, thresholds=thr, connectivity=spec.connectivity,
                    out=out)
    torch.cuda.synchronize()
    ctx.profile(True)
    ctx.profile_read(reset=True)
    stream = torch.cuda.current_stream()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t0.record(stream)
    for i in range(steps):
        ctx.compute(bufs[i % copies], spec.n_levels, thresholds=thr, connectivity=spec.connectivity,
                    out=out, stream=stream)
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    total_ms = t0.elapsed_time(t1)
    k_ms, k_n = ctx.profile_read(reset=True)
    ctx.profile(False)
    res = {c: v.cpu().numpy() for c, v in out.items()}
    del bufs
    return dict(ms_per_step=total_ms / steps, wall_s=wall, kernel_ms=k_ms / max(k_n, 1),
                kernel_ms_per_step=k_ms / steps, kernel_launches=k_n, curves=res)


def cpu_baseline(spec, gpu_curves):
    import oracle
    nt = min(16, os.cpu_count() or 1)
    t = time.perf_counter()
    ref = oracle.o2_curves(spec.data, spec.n_levels, thresholds=spec.thresholds,
                           connectivity=spec.connectivity, channels=tuple(gpu_curves), n_threads=nt)
    dt = time.perf_counter() - t
    ok = all((ref[c] == gpu_curves[c]).all() for c in gpu_curves)
    cells = spec.data.size
    return dict(value=round(cells / dt / 1e9, 4), unit="Gvoxels/s", cores=nt, kind="oracle",
                sample=f"whole field ({'x'.join(map(str, spec.data.shape))}, all {spec.n_levels} levels), "
                       f"all-levels C oracle, one run of {dt:.2f} s"), ok


STEPS_CTX = {"steps": 1}


def measure(ctx, name, steps, warmup, copies, with_cpu):
    STEPS_CTX["steps"] = steps
    spec = make_workload(name)
    r = time_field(ctx, spec, steps, warmup, copies)
    cells = spec.data.size
    elem = spec.data.dtype.itemsize
    value = cells / (r["ms_per_step"] / 1e3) / 1e9
    kernel = "ecc2d_stream" if spec.data.ndim == 2 else "ecc3d_stream"
    alg_bytes = cells * elem  # the field-reading kernel reads every cell once per step
    launches_per_step = r["kernel_launches"] / max(1, STEPS_CTX["steps"])
    achieved = alg_bytes / (r["kernel_ms_per_step"] / 1e3) / 1e9
    traffic = load_traffic(kernel, spec.meta["name"])
    out = dict(
        workload=spec.meta["name"], cells=cells, bytes=alg_bytes,
        gvox_s=round(value, 3), ms_per_step=round(r["ms_per_step"], 4),
        hbm_frac_step=round(alg_bytes / (r["ms_per_step"] / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
        roofline=dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                      frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic, kernel=kernel,
                      kernel_ms_per_launch=round(r["kernel_ms"], 4),
                      launches_per_step=launches_per_step,
                      alg_bytes_per_launch=int(alg_bytes / launches_per_step)),
        spec=spec, curves=r["curves"])
    if with_cpu:
        cb, ok = cpu_baseline(spec, r["curves"])
        out["cpu_baseline"] = cb
        out["parity_vs_oracle"] = bool(ok)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=["2d", "3d", "2d-small"], default="2d")
    ap.add_argument("--copies", type=int, default=4)
    ap.add_argument("--no-secondary", action="store_true", help="skip the 3D secondary measurement")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="also run a plain device copy of MIB MiB (for counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the EC-curve path has no "
                                   "multi-GPU form in this build (see DESIGN.md for how it would shard)",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

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

    main_r = measure(ctx, args.workload, args.steps, args.warmup, args.copies,
                     with_cpu=not args.no_cpu_baseline)
    spec = main_r["spec"]
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
    if args.workload == "2d" and not args.no_secondary:
        sec = measure(ctx, "3d", max(3, args.steps // 2), 2, 2, with_cpu=False)
        line["secondary"] = {k: sec[k] for k in ("workload", "gvox_s", "ms_per_step", "hbm_frac_step",
                                                  "roofline")}
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

"""Benchmark of the Voronoi particle-merging hot path on one MI355X.

One step = one merge event (vpm_run: bin cells, partition every cell, merge, compact) over the whole
synthetic two-stream population: 256 x 256 cells, Poisson(512) electrons per cell (33.5M particles),
two drifting Maxwellians, tolerances T_X 0.1, T_P 0.05, minimum subset 4.  Inputs are resident in
HBM before timing.  The batched fixed-point FP32 form is the measured line; the plain FP64 form
(one wavefront per cell) is timed on the same population for the speedup, and both forms' conserved
totals (weight, momentum, energy) are compared with their inputs.

Prints one JSON line.  `--copy-calib` instead runs a plain device copy of known size (for scaling
rocprofv3 FETCH_SIZE / WRITE_SIZE counters to bytes).
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

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, published
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_fixed_cells_two_stream.json")
KERNEL_SOURCE = os.path.join(ROOT, "paper_1504_00636_amd", "csrc", "vpm_fixed.hip")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def conservation_error(arrs_in, arrs_out, n_out, mass):
    """Largest relative change of the totals W, Px, Py, Pz, E (momentum normalised by sum w|p|)."""
    import torch

    def totals(a, n):
        x, y, z, px, py, pz, w = [t[:n].double() for t in a]
        e = torch.sqrt(mass * mass + px * px + py * py + pz * pz)
        return torch.stack([w.sum(), (w * px).sum(), (w * py).sum(), (w * pz).sum(), (w * e).sum()]), \
            torch.stack([w.sum(), (w * px.abs()).sum(), (w * py.abs()).sum(), (w * pz.abs()).sum(), (w * e).sum()])
    tin, scale = totals(arrs_in, arrs_in[0].numel())
    tout, _ = totals(arrs_out, n_out)
    rel = ((tout - tin).abs() / scale).cpu().numpy()
    return dict(weight=float(rel[0]), momentum=float(rel[1:4].max()), energy=float(rel[4]))


def traffic_from_profiles():
    """HBM bytes per launch of the dominant kernel from committed rocprofv3 counter runs, if they were
    taken on the current kernel source; else None."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    try:
        t = json.load(open(TRAFFIC_FILE))
        sha = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
        if t.get("kernel_source_sha256") != sha:
            return None
        return float(t["fetch_bytes_per_launch"]) + float(t["write_bytes_per_launch"])
    except Exception:
        return None


def copy_calibration(nbytes=1 << 30, reps=5):
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": nbytes, "copy_calibration_bytes_written": nbytes,
                      "launches": reps}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--fp64-steps", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 form")
    ap.add_argument("--copy-calib", action="store_true")
    ap.add_argument("--seed", type=int, default=0)
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: a merge event is cell-local, and this benchmark times the "
              "single-MI355X form; run it without --gpus or with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1504_00636_amd import vpm, workloads as W

    if args.copy_calib:
        copy_calibration()
        return

    t0 = time.time()
    wl64 = W.two_stream_grid(nx=256, ny=256, mean=512, seed=args.seed)
    wl32 = wl64.astype(np.float32)
    prm = dict(wl64.params)
    n, n_cells = wl64.n, wl64.n_cells
    log(f"[bench] generated {n} particles in {n_cells} cells ({time.time() - t0:.1f}s)")

    ctx = vpm.Context(0)
    ctx.reserve(n, n_cells)
    arrs32, off = vpm.upload(wl32)
    out32 = [torch.empty_like(a) for a in arrs32]
    out_off = torch.empty(n_cells + 1, dtype=torch.int64, device="cuda")
    out_total = torch.empty(1, dtype=torch.int64, device="cuda")
    p32 = vpm.make_params(decide=vpm.VPM_DECIDE_FIXED, **prm)
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        ctx.run(arrs32, off, n, p32, out32, out_off, out_total, stream)
    torch.cuda.synchronize()
    log("[bench] warmup done")

    ctx.profile_enable(True)
    ctx.profile_read(reset=True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        ctx.run(arrs32, off, n, p32, out32, out_off, out_total, stream)
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    prof = ctx.profile_read(reset=True)
    ctx.profile_enable(False)
    ms_step = (t_end - t_start) * 1e3 / args.steps
    n_out = int(out_total.item())
    rho = n_out / n
    flags = ctx.device_status(clear=True)
    log(f"[bench] fixed-point FP32: {ms_step:.3f} ms/step, out {n_out} (rho {rho:.4f}), flags {flags}")

    kernels = {k: dict(launches=v[0], avg_ms=v[1] / max(v[0], 1)) for k, v in prof.items()}
    # the dominant kernel: the partition/merge kernel with the largest time per step
    dom_name = max((k for k in kernels if k.startswith("fixed_cells")), key=lambda k: kernels[k]["avg_ms"])
    dom = kernels[dom_name]
    # algorithmic bytes: read every input particle (7 x FP32), write every output particle (7 x FP32)
    bytes_per_step = 28.0 * n * (1.0 + rho)
    achieved = bytes_per_step / (dom["avg_ms"] * 1e-3) / 1e9
    traffic = traffic_from_profiles()

    cons32 = conservation_error(arrs32, out32, n_out, prm["mass"])

    plain = None
    if not args.no_fp64:
        arrs64, _ = vpm.upload(wl64)
        out64 = [torch.empty_like(a) for a in arrs64]
        p64 = vpm.make_params(decide=vpm.VPM_DECIDE_FP64, **prm)
        ctx.run(arrs64, off, n, p64, out64, out_off, out_total, stream)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        for _ in range(args.fp64_steps):
            ctx.run(arrs64, off, n, p64, out64, out_off, out_total, stream)
        torch.cuda.synchronize()
        ms64 = (time.perf_counter() - ta) * 1e3 / args.fp64_steps
        n_out64 = int(out_total.item())
        cons64 = conservation_error(arrs64, out64, n_out64, prm["mass"])
        plain = dict(ms_per_step=ms64, value=n / (ms64 * 1e-3), n_out=n_out64, conservation=cons64,
                     speedup_batched_over_plain=ms64 / ms_step)
        log(f"[bench] plain FP64: {ms64:.3f} ms/step, speedup {ms64 / ms_step:.1f}x")
        del arrs64, out64

    cpu = None
    if not args.no_cpu:
        import oracle
        cores = min(os.cpu_count() or 1, int(os.environ.get("OMP_NUM_THREADS", "0") or 16))
        ta = time.perf_counter()
        oracle.run_workload(wl32, decide=oracle.FIXED, n_threads=cores)
        dt = time.perf_counter() - ta
        cpu = dict(value=n / dt, unit="particles/s", cores=cores, kind="oracle",
                   sample=f"all {n_cells} cells ({n} particles), fixed-point decisions, pair merge, "
                          f"{dt:.2f} s wall on {cores} threads")
        log(f"[bench] oracle: {dt:.2f} s on {cores} threads")

    line = {
        "metric": "input particles merged/sec + % HBM peak; batched-FP32 vs plain-FP64 at equal cons. err",
        "value": n / (ms_step * 1e-3),
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "two_stream_256x256_poisson512", "n_particles": n, "n_cells": n_cells,
                   "tol_x": prm["tol_x"], "tol_p": prm["tol_p"], "min_subset": prm["min_subset"],
                   "n_min_cell": prm["n_min_cell"], "decide": "fixed", "merge": "pair", "seed": args.seed},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": dom_name,
                     "kernel_avg_ms": dom["avg_ms"], "algorithmic_bytes_per_launch": bytes_per_step},
        "cpu_baseline": cpu,
        "merge_ratio": rho,
        "pipeline_GBps": bytes_per_step / (ms_step * 1e-3) / 1e9,
        "kernels": kernels,
        "conservation": cons32,
        "plain_fp64": plain,
        "device_flags": flags,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()

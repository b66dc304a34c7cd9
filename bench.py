"""Benchmark of the Voronoi particle-merging hot path on one MI355X.

One step = one merge event (vpm_run: bin cells, partition every cell, merge, compact) over the whole
synthetic two-stream population: 256 x 256 cells, Poisson(512) electrons per cell (33.5M particles),
two drifting Maxwellians, tolerances T_X 0.1, T_P 0.05, minimum subset 4.  Inputs are resident in
HBM before timing.  The batched fixed-point FP32 form is the measured line; the same event from the
FP64 particle arrays (rounded as they are loaded) and the plain FP64 form (one wavefront per cell,
FP64 statistics) are timed on the same population, and each form's conserved totals (weight,
momentum, energy) are compared with its input.  More workloads are reported beside the headline,
each with a roofline per size-bin kernel and the oracle timed on a sample of its cells: the
two-stream population at the paper's own two-stream tolerances (with the paper's blind method
beside the Voronoi merge), the shower-shaped 64^3 population (lognormal cell occupancy up to
32,768, gamma^-2 momenta; with the fixed-point vs FP64 partition agreement), its three-species
form, 50 graph-replayed events of the 512 x 512 cascade and the fixed-point vs FP64 comparison at
five densities.

Prints one JSON line.  Tooling modes: `--copy-calib` runs a plain device copy of known size (for
scaling rocprofv3 FETCH_SIZE / WRITE_SIZE counters to bytes); `--traffic-summary` turns four
rocprofv3 counter runs into the traffic record under profiles/.
"""
from __future__ import annotations

import argparse
import csv
import glob
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
# every source compiled into the kernels (a counter record taken on other sources is stale)
KERNEL_SOURCES = sorted(f for f in glob.glob(os.path.join(ROOT, "paper_1504_00636_amd", "csrc", "*"))
                        if f.endswith((".hip", ".h", ".hpp", ".cpp"))) + [os.path.join(ROOT, "include", "vpm.h")]
DOMINANT = "fixed_cells_576"          # the one-wavefront-per-cell bin: every two-stream cell but ~0.2 %
DOMINANT_SYMBOL = "k_fixed_cells<576"  # how rocprofv3 names it
COPY_BYTES = 1 << 30
VALU_FILE = os.path.join(ROOT, "profiles", "valu_fixed_cells_two_stream.json")
# VALU issue peak: 256 CUs x 4 SIMDs, one 64-lane VALU instruction per SIMD every 4 cycles at 2.4 GHz
VALU_PEAK_INSTS = 256 * 4 * 2.4e9 / 4
# int32 lane operations: 256 CUs x 64 lanes x 2.4 GHz
ALU_PEAK_LANE_OPS = 256 * 64 * 2.4e9
# least lane operations per particle-level (moment sums of the smaller child, the cut and the
# compaction), the algorithmic unit of the ALU figure
LANE_OPS_PER_PARTICLE_LEVEL = 40


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_sha():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(os.path.relpath(f, ROOT).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def host_cpu():
    """The host's processor model, its logical CPU count and the CPUs this process may run on."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return dict(model=model, logical_cpus=os.cpu_count(), usable_cpus=usable)


def conservation_error(arrs_in, arrs_out, n_out, mass, mass_out=None):
    """Largest relative change of the totals W, Px, Py, Pz, E (momentum normalised by sum w|p|).
    mass: a number, or a per-particle tensor (then mass_out gives the output particles' masses)."""
    import torch

    def totals(a, n, mass):
        x, y, z, px, py, pz, w = [t[:n].double() for t in a]
        e = torch.sqrt(mass * mass + px * px + py * py + pz * pz)
        return torch.stack([w.sum(), (w * px).sum(), (w * py).sum(), (w * pz).sum(), (w * e).sum()]), \
            torch.stack([w.sum(), (w * px.abs()).sum(), (w * py.abs()).sum(), (w * pz.abs()).sum(), (w * e).sum()])
    tin, scale = totals(arrs_in, arrs_in[0].numel() if mass_out is None else mass.numel(), mass)
    tout, _ = totals(arrs_out, n_out, mass if mass_out is None else mass_out)
    rel = ((tout - tin).abs() / scale).cpu().numpy()
    return dict(weight=float(rel[0]), momentum=float(rel[1:4].max()), energy=float(rel[4]))


def traffic_from_profiles():
    """HBM bytes per launch of the dominant kernel from committed rocprofv3 counter runs, if they were
    taken on the current kernel source; else None."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    try:
        t = json.load(open(TRAFFIC_FILE))
        if t.get("kernel_source_sha256") != kernel_source_sha():
            return None
        return float(t["fetch_bytes_per_launch"]) + float(t["write_bytes_per_launch"])
    except Exception:
        return None


def copy_calibration(reps=5):
    import torch
    a = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": COPY_BYTES, "copy_calibration_bytes_written": COPY_BYTES,
                      "launches": reps}))


def _counter_means(d, counter, kernel_pred):
    vals = []
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            if r["Counter_Name"] == counter and kernel_pred(r["Kernel_Name"]):
                vals.append(float(r["Counter_Value"]))
    if not vals:
        raise SystemExit(f"no {counter} rows for the kernel in {d}")
    return sum(vals) / len(vals), len(vals)


def traffic_summary(fetch_dir, write_dir, calib_fetch_dir, calib_write_dir):
    """Scale FETCH_SIZE / WRITE_SIZE of the dominant kernel by the same counters on a plain copy of
    COPY_BYTES bytes, and write the traffic record (bytes per launch) under profiles/."""
    is_dom = lambda k: DOMINANT_SYMBOL in k.replace(" ", "")
    is_copy = lambda k: "copy" in k.lower() and "fill" not in k.lower()
    f_k, nf = _counter_means(fetch_dir, "FETCH_SIZE", is_dom)
    w_k, nw = _counter_means(write_dir, "WRITE_SIZE", is_dom)
    f_c, _ = _counter_means(calib_fetch_dir, "FETCH_SIZE", is_copy)
    w_c, _ = _counter_means(calib_write_dir, "WRITE_SIZE", is_copy)
    fetch_scale = COPY_BYTES / f_c
    write_scale = COPY_BYTES / w_c
    rec = {
        "kernel": DOMINANT, "workload": "two_stream_256x256_poisson512",
        "kernel_source_sha256": kernel_source_sha(),
        "fetch_bytes_per_launch": f_k * fetch_scale, "write_bytes_per_launch": w_k * write_scale,
        "fetch_counter_per_launch": f_k, "write_counter_per_launch": w_k, "launches": [nf, nw],
        "copy_calibration": {"bytes": COPY_BYTES, "fetch_counter": f_c, "write_counter": w_c,
                             "fetch_bytes_per_count": fetch_scale, "write_bytes_per_count": write_scale},
        "commands": [
            "rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir> -o run -- python3 bench.py --no-cpu --no-fp64 --no-extra --no-autotune --steps 3 --warmup 1",
            "rocprofv3 --pmc WRITE_SIZE --output-format csv -d <dir> -o run -- python3 bench.py --no-cpu --no-fp64 --no-extra --no-autotune --steps 3 --warmup 1",
            "rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir> -o run -- python3 bench.py --copy-calib",
            "rocprofv3 --pmc WRITE_SIZE --output-format csv -d <dir> -o run -- python3 bench.py --copy-calib",
            "python3 bench.py --traffic-summary <fetch> <write> <calib-fetch> <calib-write>",
        ],
    }
    os.makedirs(os.path.dirname(TRAFFIC_FILE), exist_ok=True)
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec))


def valu_summary(pmc_dir):
    """Instruction counts of the dominant kernel per launch (SQ_INSTS_VALU, SQ_INSTS_SALU,
    SQ_INSTS_LDS, SQ_WAVES from one rocprofv3 --pmc pass), written under profiles/."""
    is_dom = lambda k: DOMINANT_SYMBOL in k.replace(" ", "")
    rec = {"kernel": DOMINANT, "workload": "two_stream_256x256_poisson512",
           "kernel_source_sha256": kernel_source_sha()}
    for c in ("SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_WAVES"):
        v, k = _counter_means(pmc_dir, c, is_dom)
        rec[c.lower() + "_per_launch"] = v
        rec["launches"] = k
    rec["command"] = ("rocprofv3 --pmc SQ_INSTS_VALU SQ_INSTS_SALU SQ_INSTS_LDS SQ_WAVES --output-format csv "
                      "-d <dir> -o run -- python3 bench.py --no-cpu --no-fp64 --no-extra --no-autotune "
                      "--steps 3 --warmup 1; python3 bench.py --valu-summary <dir>")
    os.makedirs(os.path.dirname(VALU_FILE), exist_ok=True)
    with open(VALU_FILE, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec))


def valu_from_profiles():
    """VALU wave-instructions per launch of the dominant kernel from the committed counter run, if it
    was taken on the current kernel source; else None."""
    if not os.path.exists(VALU_FILE):
        return None
    try:
        t = json.load(open(VALU_FILE))
        if t.get("kernel_source_sha256") != kernel_source_sha():
            return None
        return float(t["sq_insts_valu_per_launch"])
    except Exception:
        return None


# the size-bin kernels, in the order of their upper limits in the tuning (the last has none)
BINS = [("fixed_cells_small", "bin_s_max"), ("fixed_cells_576", "bin_a_max"), ("fixed_cells_1144", "bin_d_max"),
        ("fixed_cells_2288", "bin_b_max"), ("fixed_cells_4592", "bin_c_max"), ("fixed_cells_big", None)]
ORACLE_KEYS = ("tol_x", "tol_p", "n_min_cell", "min_subset", "cell_len", "mass")


def bin_of_cells(counts, tuning, n_min_cell):
    """The size bin of every cell as the library assigns it (-1: left untouched)."""
    lims = [tuning[k] for _, k in BINS[:-1]]
    b = np.searchsorted(np.asarray(lims), counts, side="left")      # first bin whose limit >= count
    proc = (counts > n_min_cell) & (counts > 0) & (counts <= (1 << 24))
    return np.where(proc, b, -1)


def oracle_threads():
    """Threads for the oracle: the CPUs this process may use, capped by OMP_NUM_THREADS when set."""
    usable = host_cpu()["usable_cpus"]
    env = os.environ.get("OMP_NUM_THREADS")
    return max(1, min(usable, int(env))) if env and env.isdigit() else usable


def oracle_sample(wl, prm, bins, per_bin, seed):
    """The CPU baseline of a workload on a bounded sample: the oracle (fixed-point decisions, pair
    merge) on up to per_bin seeded cells of every size bin, timed; returns its rate and, per bin,
    the particle-levels of the tree (particles times levels they pass through) per particle."""
    import oracle
    r = np.random.Generator(np.random.Philox(seed + 7))
    counts = np.diff(wl.cell_off)
    threads = oracle_threads()
    pick = []
    for i in range(len(BINS)):
        cells = np.nonzero(bins == i)[0]
        if cells.size:
            pick.append(np.sort(r.choice(cells, min(per_bin, cells.size), replace=False)))
    pick = np.concatenate(pick) if pick else np.zeros(0, np.int64)
    sub = wl.cells(pick)
    t0 = time.perf_counter()
    ref = oracle.run(sub.arrays(), sub.cell_off, decide=oracle.FIXED, n_threads=threads,
                     **{k: prm[k] for k in ORACLE_KEYS})
    dt = time.perf_counter() - t0
    per_bin_pl = {}
    for i, (name, _) in enumerate(BINS):
        m = bins[pick] == i
        if m.any():
            per_bin_pl[name] = float(ref.stats["particle_levels"][m].sum()) / float(counts[pick][m].sum())
    return dict(value=sub.n / dt, unit="particles/s", cores=threads, kind="oracle",
                sample=f"{pick.size} seeded cells (up to {per_bin} per size bin, {sub.n} particles), "
                       f"{dt:.2f} s wall on {threads} threads"), per_bin_pl


def bin_rooflines(counts, out_counts, bins, kernels, in_bytes=28.0, pl_per_particle=None):
    """Per size-bin kernel: its cells' algorithmic bytes (in_bytes per input particle read, 28 per
    output particle written) over the kernel's average duration against the HBM peak and, given the
    particle-levels per particle of the bin, its algorithmic integer work against the int32 lane
    peak.  Returns the per-bin records and the name of the longest-running kernel."""
    rec = {}
    for i, (name, _) in enumerate(BINS):
        m = bins == i
        if not m.any() or name not in kernels:
            continue
        ms = kernels[name]["avg_ms"]
        byt = in_bytes * float(counts[m].sum()) + 28.0 * float(out_counts[m].sum())
        r = dict(cells=int(m.sum()), particles=int(counts[m].sum()), avg_ms=ms, algorithmic_bytes=byt,
                 roofline=dict(bound="hbm", achieved=byt / (ms * 1e-3) / 1e9, peak=HBM_PEAK_GBS, unit="GB/s",
                               frac=byt / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS))
        if pl_per_particle and name in pl_per_particle:
            pl = pl_per_particle[name] * float(counts[m].sum())
            ops = pl * LANE_OPS_PER_PARTICLE_LEVEL / (ms * 1e-3)
            r["alu"] = dict(particle_levels_per_launch=pl, lane_ops_per_particle_level=LANE_OPS_PER_PARTICLE_LEVEL,
                            achieved=ops, peak=ALU_PEAK_LANE_OPS, unit="int32 lane-ops/s",
                            frac=ops / ALU_PEAK_LANE_OPS, estimate="particle-levels per particle of the bin "
                            "from the oracle's sample, times the bin's particles")
        rec[name] = r
    dominant = max(rec, key=lambda k: rec[k]["avg_ms"]) if rec else None
    return rec, dominant


def autotune(ctx, vpm, arrs, off, n, p):
    """Let the library pick lane-group sizing and bin limits for this population (timed on the GPU),
    through the persistent tuning cache (keyed by device, ROCm, dtype, sources and the population's
    shape); returns (tuning dict, seconds spent).  The dict notes whether the cache held it."""
    import torch
    from paper_1504_00636_amd import tuning_cache
    out = [torch.empty_like(a, dtype=torch.float32) for a in arrs]
    out_off = torch.empty(off.numel(), dtype=torch.int64, device="cuda")
    out_total = torch.empty(1, dtype=torch.int64, device="cuda")
    t0 = time.perf_counter()
    best, hit, _ = tuning_cache.autotune_cached(ctx, arrs, off, n, p, out, out_off, out_total)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    del out
    return dict(best.as_dict(), from_cache=hit), dt


def time_fixed(ctx, vpm, arrs, off, n, p, steps, warmup, profile, graph=False):
    """Time `steps` merge events of one form; returns (ms/step, outputs, out_off, n_out, kernels, extra).

    graph: the event is captured once in a HIP graph and the timed steps replay it (the library's
    launches have no host-side dependencies, so the graph holds the whole event); the replayed
    output must equal an eager call's bit for bit.  profile: a separate eager pass after the timed
    steps records every internal kernel with HIP events on the stream it runs on (never inside the
    timed steps)."""
    import torch
    n_cells = off.numel() - 1
    odt = torch.float32 if p.decide == vpm.VPM_DECIDE_FIXED else arrs[0].dtype    # the fixed-point path writes FP32
    out = [torch.empty_like(a, dtype=odt) for a in arrs]
    out_off = torch.empty(n_cells + 1, dtype=torch.int64, device="cuda")
    out_total = torch.empty(1, dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream()
    extra = {}
    for _ in range(warmup):
        ctx.run(arrs, off, n, p, out, out_off, out_total, stream)
    torch.cuda.synchronize()
    if graph:
        eager = [t.clone() for t in out], out_off.clone(), int(out_total.item())
        t0 = time.perf_counter()
        for _ in range(steps):
            ctx.run(arrs, off, n, p, out, out_off, out_total, stream)
        torch.cuda.synchronize()
        extra["eager_ms_per_step"] = (time.perf_counter() - t0) * 1e3 / steps
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            ctx.run(arrs, off, n, p, out, out_off, out_total)
        for _ in range(max(warmup, 1)):
            g.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            g.replay()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        tot = int(out_total.item())
        same = tot == eager[2] and torch.equal(out_off, eager[1]) and all(
            torch.equal(a[:tot].view(torch.int32), b[:tot].view(torch.int32)) for a, b in zip(out, eager[0]))
        if not same:
            raise RuntimeError("graph-replayed merge event differs from the eager call")
        extra["graph_replay_equals_eager"] = True
        del g
    else:
        t0 = time.perf_counter()
        for _ in range(steps):
            ctx.run(arrs, off, n, p, out, out_off, out_total, stream)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
    kernels = {}
    if profile:
        ctx.profile_enable(True)
        ctx.profile_read(reset=True)
        for _ in range(steps):
            ctx.run(arrs, off, n, p, out, out_off, out_total, stream)
        torch.cuda.synchronize()
        prof = ctx.profile_read(reset=True)
        ctx.profile_enable(False)
        kernels = {k: dict(launches=v[0], avg_ms=v[1] / max(v[0], 1)) for k, v in prof.items()}
    return ms, out, out_off, int(out_total.item()), kernels, extra


def time_plain(ctx, vpm, wl64, prm, steps):
    import torch
    arrs64, off64 = vpm.upload(wl64)
    n = wl64.n
    p64 = vpm.make_params(decide=vpm.VPM_DECIDE_FP64, **prm)
    ms, out64, _, n_out, _, _ = time_fixed(ctx, vpm, arrs64, off64, n, p64, steps, 1, False)
    cons = conservation_error(arrs64, out64, n_out, prm["mass"])
    del arrs64, out64
    torch.cuda.empty_cache()
    return dict(ms_per_step=ms, value=n / (ms * 1e-3), n_out=n_out, conservation=cons)


def extra_workload(ctx, vpm, name, wl32, wl64, prm, steps, fp64_steps, tune=True, cv=True, cpu=True,
                   agreement=False, seed=0):
    """One more population: FIXED FP32 timing with a roofline per size-bin kernel and, unless
    fp64_steps == 0, the plain FP64 form.  tune = False keeps the context's batching configuration;
    cv = False leaves out the merged-subset CVs (a vpm_partition launch of their own); cpu: the
    oracle timed on a bounded sample of the workload's cells (its CPU baseline, whose tree also
    gives each bin's particle-levels for the ALU figure); agreement: the fraction of particles whose
    final subset is the same under the fixed-point and the FP64 decisions (on the same FP32 values)."""
    import torch
    n = wl32.n
    arrs, off = vpm.upload(wl32)
    p32 = vpm.make_params(decide=vpm.VPM_DECIDE_FIXED, **prm)
    if tune:
        tuning, tune_s = autotune(ctx, vpm, arrs, off, n, p32)
    else:
        tuning, tune_s = ctx.get_tuning().as_dict(), 0.0
    ms, out, out_off, n_out, kernels, _ = time_fixed(ctx, vpm, arrs, off, n, p32, steps, 2, True)
    counts = np.diff(wl32.cell_off)
    bins = bin_of_cells(counts, tuning, prm["n_min_cell"])
    out_counts = np.diff(out_off.cpu().numpy())
    cpu_rec, pl = (oracle_sample(wl32, prm, bins, 2048, seed) if cpu else (None, None))
    per_bin, dominant = bin_rooflines(counts, out_counts, bins, kernels, 28.0, pl)
    rec = dict(workload=name, n_particles=n, n_cells=wl32.n_cells, ms_per_step=ms, value=n / (ms * 1e-3),
               tuning=tuning, autotune_s=tune_s,
               unit="particles/s", merge_ratio=n_out / n,
               pipeline_GBps=28.0 * (n + n_out) / (ms * 1e-3) / 1e9,
               roofline=dict(per_bin[dominant]["roofline"], kernel=dominant) if dominant else None,
               alu=dict(per_bin[dominant]["alu"], kernel=dominant) if dominant and "alu" in per_bin[dominant] else None,
               bins=per_bin, cpu_baseline=cpu_rec,
               conservation=conservation_error(arrs, out, n_out, prm["mass"]),
               merged_cv=merged_cv(ctx, vpm, arrs, off, n, p32, prm) if cv else None,
               kernels={k: round(v["avg_ms"], 4) for k, v in kernels.items()},
               params={k: prm[k] for k in ("tol_x", "tol_p", "n_min_cell", "min_subset")})
    del out
    if agreement:
        perm = torch.empty(n, dtype=torch.int32, device="cuda")
        sid = torch.empty(n, dtype=torch.int32, device="cuda")
        nsub = torch.empty(wl32.n_cells, dtype=torch.int32, device="cuda")
        ctx.partition(arrs, off, n, p32, perm, sid, nsub)
        lab32 = subset_labels(perm, sid, off)
        del arrs
        torch.cuda.empty_cache()
        arrs64, off64 = vpm.upload(wl32, dtype=torch.float64)
        p64 = vpm.make_params(decide=vpm.VPM_DECIDE_FP64, **prm)
        ctx.partition(arrs64, off64, n, p64, perm, sid, nsub)
        lab64 = subset_labels(perm, sid, off64)
        same = lab32 == lab64
        cid = torch.repeat_interleave(torch.arange(wl32.n_cells, device="cuda"), off64[1:] - off64[:-1],
                                      output_size=n)
        differ = torch.zeros(wl32.n_cells, dtype=torch.int32, device="cuda").index_add_(0, cid, (~same).int())
        rec["fixed_vs_fp64_partition"] = dict(particle_agreement=float(same.double().mean().item()),
                                              identical_cells=float((differ == 0).double().mean().item()))
        del arrs64, perm, sid, nsub, lab32, lab64, same, cid, differ
    else:
        del arrs
    torch.cuda.empty_cache()
    if fp64_steps > 0 and wl64 is not None:
        pl = time_plain(ctx, vpm, wl64, prm, fp64_steps)
        pl["speedup_batched_over_plain"] = pl["ms_per_step"] / ms
        rec["plain_fp64"] = pl
    log(f"[bench] {name}: {ms:.3f} ms/step ({rec['value']:.3g} particles/s), rho {rec['merge_ratio']:.4f}")
    return rec


def whole_box(ctx, vpm, W, seed, steps=3, cpu=True):
    """Global merging: a whole simulation box passed as one cell (the method's first subset is the
    box), in three populations: the counter-propagating blocks at 4,000 and at 16,000 electrons per
    unit cell (4 M and 16 M particles in a 100 x 20 box; the largest cell is 2^24 = 16.8 M) and a
    64 x 64 patch of the two-stream population (2.1 M particles).
    Each is timed per merge event; the oracle is timed on the same box (its CPU baseline), and that
    run's partition is compared with the GPU's (bit-exact)."""
    import torch
    import oracle
    recs = {}
    # the default batching (bins in sequence): a lone large cell needs every workgroup of the
    # large-cell kernel to wait for its subsets, which the concurrent-bin mode does not do
    saved = ctx.get_tuning()
    ctx.set_tuning(vpm.make_tuning())
    blocks = W.counter_blocks(per_cell=4000, seed=seed)
    blocks16 = W.counter_blocks(per_cell=16000, seed=seed + 1)     # 16 M particles: near the largest cell
    ts = W.two_stream_grid(nx=64, ny=64, mean=512, seed=seed)
    cases = [("counter_blocks_4M", blocks, dict(blocks.params, cell_len=(100.0, 20.0, 1.0), tol_x=0.02)),
             ("counter_blocks_16M", blocks16, dict(blocks16.params, cell_len=(100.0, 20.0, 1.0), tol_x=0.02)),
             ("two_stream_64x64", ts, dict(ts.params, cell_len=(64.0, 64.0, 1.0), tol_x=0.02))]
    for name, wl, prm in cases:
        box = W.Workload(name, *[getattr(wl, f).astype(np.float32) for f in W.FIELDS],
                         cell_off=np.array([0, wl.n], np.int64), cell_id=None, params=prm)
        n = box.n
        arrs, off = vpm.upload(box)
        p32 = vpm.make_params(decide=vpm.VPM_DECIDE_FIXED, **prm)
        ctx.device_status(clear=True)
        ms, out, out_off, n_out, kernels, _ = time_fixed(ctx, vpm, arrs, off, n, p32, steps, 1, True)
        rec = dict(workload=f"{name}_as_one_cell", n_particles=n, ms_per_step=ms, value=n / (ms * 1e-3),
                   unit="particles/s", n_out=n_out, device_flags=ctx.device_status(clear=True),
                   tuning=ctx.get_tuning().as_dict(),
                   conservation=conservation_error(arrs, out, n_out, prm["mass"]),
                   kernels={k: round(v["avg_ms"], 4) for k, v in kernels.items()},
                   params={k: prm[k] for k in ("tol_x", "tol_p", "n_min_cell", "min_subset", "cell_len")})
        del out
        perm = torch.empty(n, dtype=torch.int32, device="cuda")
        sid = torch.empty(n, dtype=torch.int32, device="cuda")
        nsub = torch.empty(1, dtype=torch.int32, device="cuda")
        ctx.partition(arrs, off, n, p32, perm, sid, nsub)
        torch.cuda.synchronize()
        rec["subsets"] = int(nsub.item())
        if cpu:
            keys = ("tol_x", "tol_p", "n_min_cell", "min_subset", "cell_len", "mass")
            t0 = time.perf_counter()
            ref = oracle.run_workload(box, decide=oracle.FIXED, merge_mode=oracle.PAIR,
                                      **{k: prm[k] for k in keys})
            t_orc = time.perf_counter() - t0
            same = bool(int(ref.n_subsets[0]) == rec["subsets"] and ref.out_total == n_out and
                        np.array_equal(perm.cpu().numpy(), ref.perm) and
                        np.array_equal(sid.cpu().numpy(), ref.subset_id))
            rec["cpu_baseline"] = dict(value=n / t_orc, unit="particles/s", cores=1, kind="oracle",
                                       sample=f"the whole box ({n} particles), {t_orc:.2f} s wall (one cell: one thread)",
                                       gpu_partition_equal=same)
        del arrs, perm, sid, nsub
        torch.cuda.empty_cache()
        log(f"[bench] whole box {name}: {n} particles, {ms:.2f} ms/event, {rec['subsets']} subsets, "
            f"oracle equal: {(rec.get('cpu_baseline') or {}).get('gpu_partition_equal')}")
        recs[name] = rec
    ctx.set_tuning(saved)
    return recs


def blind_vs_voronoi(ctx, vpm, wl32, prm, alphas, seed, steps=5):
    """The paper's comparison on one population: the Voronoi merge (vpm_run) against the blind method
    (vpm_blind: random pairs merged until at most ceil(alpha N) particles remain per cell), each
    with its particle count, time and conserved-total errors; the blind method runs at the paper's
    fraction(s) and at the Voronoi merge's own output fraction (the same particle count)."""
    import torch
    n = wl32.n
    arrs, off = vpm.upload(wl32)
    p = vpm.make_params(decide=vpm.VPM_DECIDE_FIXED, **prm)
    out = [torch.empty_like(a) for a in arrs]
    oo = torch.empty(off.numel(), dtype=torch.int64, device="cuda")
    ot = torch.empty(1, dtype=torch.int64, device="cuda")

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps

    ms = timed(lambda: ctx.run(arrs, off, n, p, out, oo, ot))
    n_v = int(ot.item())
    recs = {"voronoi": dict(n_out=n_v, merge_ratio=n_v / n, ms_per_step=ms,
                            conservation=conservation_error(arrs, out, n_v, prm["mass"]))}
    for a in list(alphas) + [n_v / n]:
        ms = timed(lambda: ctx.blind(arrs, off, n, p, a, seed, out, oo, ot))
        k = int(ot.item())
        recs[f"blind_alpha_{a:.6g}"] = dict(alpha=a, n_out=k, merge_ratio=k / n, ms_per_step=ms,
                                          conservation=conservation_error(arrs, out, k, prm["mass"]))
    flags = ctx.device_status(clear=True)
    del arrs, out
    torch.cuda.empty_cache()
    log(f"[bench] blind vs Voronoi: " + ", ".join(f"{k}: {v['n_out']} out, dE {v['conservation']['energy']:.2e}"
                                                   for k, v in recs.items()))
    return dict(workload="two_stream_256x256_poisson512_T0.8_0.15_Nmin200", seed=seed, device_flags=flags,
                params={k: prm[k] for k in ("tol_x", "tol_p", "n_min_cell", "min_subset")}, methods=recs,
                note="energy: relative change of the total energy; the blind method conserves weight and "
                     "momentum and loses energy, the Voronoi pair merge conserves all three")


def species_shower(ctx, vpm, W, seed, steps=5, warmup=2):
    """The shower population with three species (electrons, positrons and photons: masses 1, 1, 0),
    one drawn per cell, merged in one launch by vpm_run_species with the batching tuned for the
    shower."""
    import torch
    sh = W.shower_grid(nc=64, seed=seed)
    prm = dict(sh.params)
    masses = [1.0, 1.0, 0.0]
    species = np.random.Generator(np.random.Philox(seed + 100)).integers(0, 3, sh.n_cells).astype(np.uint8)
    n, n_cells = sh.n, sh.n_cells
    arrs, off = vpm.upload(sh)
    del sh
    sp = torch.from_numpy(species).cuda()
    p = vpm.make_params(decide=vpm.VPM_DECIDE_FIXED, **prm)
    out = [torch.empty_like(a) for a in arrs]
    out_off = torch.empty(n_cells + 1, dtype=torch.int64, device="cuda")
    out_total = torch.empty(1, dtype=torch.int64, device="cuda")
    ctx.device_status(clear=True)
    for _ in range(warmup):
        ctx.run_species(arrs, off, n, p, sp, masses, out, out_off, out_total)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.run_species(arrs, off, n, p, sp, masses, out, out_off, out_total)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    n_out = int(out_total.item())
    m_cell = torch.tensor(masses, dtype=torch.float64, device="cuda")[sp.long()]
    m_in = torch.repeat_interleave(m_cell, off[1:] - off[:-1], output_size=n)
    m_out = torch.repeat_interleave(m_cell, out_off[1:] - out_off[:-1], output_size=n_out)
    cons = conservation_error(arrs, out, n_out, m_in, m_out)
    flags = ctx.device_status(clear=True)
    del arrs, out, m_in, m_out
    torch.cuda.empty_cache()
    log(f"[bench] shower, three species: {ms:.3f} ms/step")
    return dict(workload="shower_64cubed_three_species", n_particles=n, n_cells=n_cells, species_mass=masses,
                cells_per_species=np.bincount(species, minlength=3).tolist(), ms_per_step=ms,
                value=n / (ms * 1e-3), unit="particles/s", merge_ratio=n_out / n, conservation=cons,
                device_flags=flags, tuning=ctx.get_tuning().as_dict(),
                params={k: prm[k] for k in ("tol_x", "tol_p", "n_min_cell", "min_subset")})


def merged_cv(ctx, vpm, arrs, off, n, p, prm):
    """Largest real-valued coefficients of variation (Eqs. cv_x and cv_p, in FP64 from the FP32
    values) over the subsets that the fixed-point partition merges, per kind of axis, against the
    tolerances: the fixed-point rule decides on the particles' codes, so a merged subset's CV may
    exceed its tolerance by the codes' quantisation."""
    import torch
    n_cells = off.numel() - 1
    perm = torch.empty(n, dtype=torch.int32, device="cuda")
    sid = torch.empty(n, dtype=torch.int32, device="cuda")
    nsub = torch.empty(n_cells, dtype=torch.int32, device="cuda")
    ctx.partition(arrs, off, n, p, perm, sid, nsub)
    cid = torch.repeat_interleave(torch.arange(n_cells, device="cuda"), off[1:] - off[:-1], output_size=n)
    ok = sid >= 0
    key = (cid * (1 << 20) + sid.long())[ok]
    src = perm.long()[ok]
    del cid, sid, nsub
    _, inv = torch.unique_consecutive(key, return_inverse=True)
    ns = int(inv.max().item()) + 1 if inv.numel() else 0
    cnt = torch.bincount(inv, minlength=ns)
    w = arrs[6][src].double()
    W = torch.zeros(ns, dtype=torch.float64, device="cuda").index_add_(0, inv, w)
    merged = cnt >= prm["min_subset"]
    worst = []
    for l in range(6):
        v = arrs[l][src].double()
        s1 = torch.zeros(ns, dtype=torch.float64, device="cuda").index_add_(0, inv, w * v)
        mean = s1 / W
        s2 = torch.zeros(ns, dtype=torch.float64, device="cuda").index_add_(0, inv, w * (v - mean[inv]) ** 2)
        sigma = torch.sqrt(s2 / W)
        if l < 3:
            cv = sigma / prm["cell_len"][l]
        else:
            cv = torch.where(sigma == 0, torch.zeros_like(sigma), sigma / mean.abs())
        worst.append(float(cv[merged].max().item()) if bool(merged.any()) else 0.0)
    del perm, key, src, inv, w
    torch.cuda.empty_cache()
    return dict(merged_subsets=int(merged.sum().item()), max_cv_position=max(worst[:3]),
                max_cv_momentum=max(worst[3:]), tol_x=prm["tol_x"], tol_p=prm["tol_p"])


def subset_labels(perm, sid, n_subsets_cell_off):
    """Canonical label of every particle's final subset: the smallest input index among its members
    (-1 for particles of cells that were not processed).  perm / subset_id as vpm_partition writes
    them (subsets contiguous per cell)."""
    import torch
    cell_off = n_subsets_cell_off
    n = perm.numel()
    counts = (cell_off[1:] - cell_off[:-1])
    cid = torch.repeat_interleave(torch.arange(counts.numel(), device=perm.device), counts, output_size=n)
    key = cid * (1 << 20) + sid.long().clamp(min=0)                  # (cell, subset) -> one key
    uniq, inv = torch.unique_consecutive(key, return_inverse=True)
    first = torch.full((uniq.numel(),), 1 << 62, dtype=torch.int64, device=perm.device)
    first.scatter_reduce_(0, inv, perm.long(), reduce="amin")
    lab = torch.empty(n, dtype=torch.int64, device=perm.device)
    lab[perm.long()] = first[inv]
    lab[perm.long()[sid < 0]] = -1
    return lab


def precision_sweep(ctx, vpm, W, means, seed):
    """The two-stream population at several densities: the batched fixed-point FP32 form against the
    plain FP64 form on the same particles: time, conserved-total error of each against the exact
    input totals, the fraction of particles whose final subset is the same in both, and the
    fraction of cells partitioned identically."""
    import torch
    recs = []
    for mean in means:
        wl64 = W.two_stream_grid(nx=256, ny=256, mean=mean, seed=seed)
        wl32 = wl64.astype(np.float32)
        prm = dict(wl64.params)
        n = wl64.n
        ctx.reserve(n, wl64.n_cells)
        arrs, off = vpm.upload(wl32)
        p32 = vpm.make_params(decide=vpm.VPM_DECIDE_FIXED, **prm)
        ms32, out32, _, n_out32, _, _ = time_fixed(ctx, vpm, arrs, off, n, p32, 5, 1, False)
        cons32 = conservation_error(arrs, out32, n_out32, prm["mass"])
        del out32
        perm = torch.empty(n, dtype=torch.int32, device="cuda")
        sid = torch.empty(n, dtype=torch.int32, device="cuda")
        nsub = torch.empty(wl64.n_cells, dtype=torch.int32, device="cuda")
        ctx.partition(arrs, off, n, p32, perm, sid, nsub)
        lab32 = subset_labels(perm, sid, off)
        del arrs
        torch.cuda.empty_cache()
        # the plain FP64 form runs on the FP32-rounded particles, so both see the same input
        arrs64, off64 = vpm.upload(wl32, dtype=torch.float64)
        p64 = vpm.make_params(decide=vpm.VPM_DECIDE_FP64, **prm)
        ms64, out64, _, n_out64, _, _ = time_fixed(ctx, vpm, arrs64, off64, n, p64, 1, 1, False)
        cons64 = conservation_error(arrs64, out64, n_out64, prm["mass"])
        del out64
        ctx.partition(arrs64, off64, n, p64, perm, sid, nsub)
        lab64 = subset_labels(perm, sid, off64)
        same = lab32 == lab64
        agree = float(same.double().mean().item())
        cid = torch.repeat_interleave(torch.arange(wl64.n_cells, device="cuda"), off64[1:] - off64[:-1],
                                      output_size=n)
        differ = torch.zeros(wl64.n_cells, dtype=torch.int32, device="cuda").index_add_(0, cid, (~same).int())
        cells_agree = float((differ == 0).double().mean().item())
        del arrs64, lab32, lab64, perm, sid, nsub, same, cid, differ
        torch.cuda.empty_cache()
        recs.append(dict(mean_per_cell=mean, n_particles=n, fixed_fp32_ms=ms32, plain_fp64_ms=ms64,
                         speedup=ms64 / ms32, fixed_fp32_conservation=cons32, plain_fp64_conservation=cons64,
                         merge_ratio_fp32=n_out32 / n, merge_ratio_fp64=n_out64 / n, partition_agreement=agree,
                         identical_cells=cells_agree))
        log(f"[bench] precision sweep, mean {mean}: FP32 {ms32:.2f} ms, FP64 {ms64:.2f} ms, agreement {agree:.5f}")
    return dict(workload="two_stream_256x256_poisson_mean", tolerances=[0.1, 0.05], points=recs)


CASCADE_TOL_P = 0.6   # merged cells fall to a few hundred particles and grow back: cells stay near N_min


def cascade(ctx, vpm, W, steps, seed):
    """Repeated merge events: the 512 x 512 cascade (256 particles per cell at the start, every particle
    split in two between events, cells above 1,024 particles merged) at T_P 0.6, which holds the
    cells near 1,024 particles.  The merge event is captured once in a HIP graph and replayed for
    every step; the population size is read on the device."""
    import torch
    cap = 540_000_000
    wl = W.cascade_initial(seed=seed)
    prm = dict(wl.params, tol_p=CASCADE_TOL_P)
    n_cells = wl.n_cells
    ctx.reserve(cap, n_cells)
    ctx.set_tuning(vpm.make_tuning())       # default batching (the early steps merge nothing to tune on)
    P = [torch.empty(cap, dtype=torch.float32, device="cuda") for _ in range(7)]
    Q = [torch.empty(cap, dtype=torch.float32, device="cuda") for _ in range(7)]
    offP = torch.from_numpy(wl.cell_off).cuda()
    offQ = torch.empty_like(offP)
    for t, a in zip(P, wl.arrays()):
        t[:wl.n].copy_(torch.from_numpy(a))
    n = wl.n
    del wl
    out_total = torch.empty(1, dtype=torch.int64, device="cuda")
    p = vpm.make_params(decide=vpm.VPM_DECIDE_FIXED, **prm)
    g = None
    recs = []
    for step in range(steps):
        if 2 * n > cap:
            break
        n2 = W.cascade_split_device(P, offP, n, step, Q, offQ, seed=seed)
        torch.cuda.synchronize()
        if g is None:                       # capture the merge event once (capturing runs nothing)
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                ctx.run(Q, offQ, cap, p, P, offP, out_total)
            torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        g.replay()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        n_out = int(out_total.item())
        counts = (offQ[1:] - offQ[:-1])
        recs.append(dict(step=step, n_in=n2, n_out=n_out, cells_merged=int((counts > prm["n_min_cell"]).sum().item()),
                         ms=ms, value=n2 / (ms * 1e-3)))
        log(f"[bench] cascade step {step}: {n2} -> {n_out} particles, {ms:.2f} ms")
        n = n_out
    flags = ctx.device_status(clear=True)
    del P, Q
    torch.cuda.empty_cache()
    tot_ms = sum(r["ms"] for r in recs)
    tot_in = sum(r["n_in"] for r in recs)
    return dict(workload="cascade_512x512_from256", params={k: prm[k] for k in ("tol_x", "tol_p", "n_min_cell", "min_subset")},
                capacity=cap, graph_replayed=True, steps_run=len(recs), total_merge_ms=tot_ms,
                value=tot_in / (tot_ms * 1e-3) if tot_ms > 0 else None, unit="input particles/s over all events",
                max_population=max((r["n_in"] for r in recs), default=0), steps=recs, device_flags=flags,
                note="every particle is split in two between events; each event merges the cells above "
                     "N_min, and the run stops early only if the next split would exceed the capacity")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--fp64-steps", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 form")
    ap.add_argument("--no-extra", action="store_true", help="skip the shower and paper-tolerance workloads")
    ap.add_argument("--copy-calib", action="store_true")
    ap.add_argument("--traffic-summary", nargs=4, metavar=("FETCH", "WRITE", "CALIB_FETCH", "CALIB_WRITE"))
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cascade-steps", type=int, default=50)
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default batching configuration (profiling runs: one kernel configuration only)")
    ap.add_argument("--valu-summary", metavar="PMC_DIR")
    ap.add_argument("--shower-only", action="store_true",
                    help="time only the shower population (every size bin) and print its record (profiling runs)")
    ap.add_argument("--whole-box-only", action="store_true",
                    help="time only the whole-box populations (each merged as one cell) and print their record")
    ap.add_argument("--bins-in-sequence", action="store_true",
                    help="with --shower-only --no-autotune: run the size bins one after another (per-bin times)")
    ap.add_argument("--graph", action="store_true",
                    help="time replays of the merge event captured in a HIP graph (checked against an eager call)")
    args = ap.parse_args()

    if args.traffic_summary:
        traffic_summary(*args.traffic_summary)
        return
    if args.valu_summary:
        valu_summary(args.valu_summary)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: a merge event is cell-local, and this benchmark times the "
              "single-MI355X form; run it without --gpus or with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1504_00636_amd import vpm, workloads as W

    if args.copy_calib:
        copy_calibration()
        return
    if args.whole_box_only:
        ctx = vpm.Context(0)
        ctx.reserve(17_000_000, 4096)
        print(json.dumps(whole_box(ctx, vpm, W, args.seed, steps=args.steps, cpu=not args.no_cpu)))
        return
    if args.shower_only:
        ctx = vpm.Context(0)
        ctx.reserve(52_000_000, 64 ** 3)
        sh = W.shower_grid(nc=64, seed=args.seed)
        if args.no_autotune:        # the configuration the autotuner usually picks for this population
            ctx.set_tuning(vpm.make_tuning(ppl=16, concurrent_bins=0 if args.bins_in_sequence else 1))
        print(json.dumps(extra_workload(ctx, vpm, "shower_64cubed_lognormal64", sh, None, dict(sh.params),
                                        args.steps, 0, tune=not args.no_autotune, cv=False)))
        return

    t0 = time.time()
    wl64 = W.two_stream_grid(nx=256, ny=256, mean=512, seed=args.seed)
    wl32 = wl64.astype(np.float32)
    prm = dict(wl64.params)
    n, n_cells = wl64.n, wl64.n_cells
    log(f"[bench] generated {n} particles in {n_cells} cells ({time.time() - t0:.1f}s)")

    ctx = vpm.Context(0)
    ctx.reserve(52_000_000, 64 ** 3)
    arrs32, off = vpm.upload(wl32)
    p32 = vpm.make_params(decide=vpm.VPM_DECIDE_FIXED, **prm)
    if args.no_autotune:
        tuning, tune_s = ctx.get_tuning().as_dict(), 0.0
    else:
        tuning, tune_s = autotune(ctx, vpm, arrs32, off, n, p32)
    log(f"[bench] tuning ({tune_s:.2f}s autotune): {tuning}")
    ms_step, out32, out_off, n_out, kernels, timing = time_fixed(ctx, vpm, arrs32, off, n, p32, args.steps,
                                                                 args.warmup, True, graph=args.graph)
    rho = n_out / n
    flags = ctx.device_status(clear=True)
    log(f"[bench] fixed-point FP32: {ms_step:.3f} ms/step, out {n_out} (rho {rho:.4f}), flags {flags}")

    # Roofline of the dominant kernel (the one-wavefront-per-cell bin): algorithmic bytes of the cells
    # it processes (read 7 x FP32 per input particle, write 7 x FP32 per output particle) over its
    # average duration, timed with HIP events on the stream it runs on.
    counts = np.diff(wl32.cell_off)
    gpu_out_off = out_off.cpu().numpy()
    out_counts = np.diff(gpu_out_off)
    in_a = bin_of_cells(counts, tuning, prm["n_min_cell"]) == 1
    bytes_dom = 28.0 * float(counts[in_a].sum() + out_counts[in_a].sum())
    dom = kernels[DOMINANT]
    achieved = bytes_dom / (dom["avg_ms"] * 1e-3) / 1e9
    traffic = traffic_from_profiles()
    bytes_step = 28.0 * n * (1.0 + rho)
    cons32 = conservation_error(arrs32, out32, n_out, prm["mass"])
    # (a vpm_partition launch of its own: left out of the counter and trace runs, which pass
    # --no-extra, so that they see the timed form's launches only)
    cv32 = None if args.no_extra else merged_cv(ctx, vpm, arrs32, off, n, p32, prm)

    # The same event from the FP64 particle arrays (the fixed-point kernels round each value to FP32
    # as they load it; FP32 output): its time, its roofline on 56 bytes read per input particle, and
    # whether its output equals the FP32 run's bit for bit.
    fp64_in = None
    if not args.no_fp64:
        arrs64, off64 = vpm.upload(wl64)
        p64in = vpm.make_params(decide=vpm.VPM_DECIDE_FIXED, dtype=vpm.VPM_F64, **prm)
        ms64i, out64i, oo64i, n64i, k64i, _ = time_fixed(ctx, vpm, arrs64, off64, n, p64in, args.steps,
                                                         args.warmup, True)
        same = n64i == n_out and torch.equal(oo64i, out_off) and all(
            torch.equal(a[:n_out].view(torch.int32), b[:n_out].view(torch.int32)) for a, b in zip(out64i, out32))
        b64 = 56.0 * float(counts[in_a].sum()) + 28.0 * float(out_counts[in_a].sum())
        d64 = k64i[DOMINANT]["avg_ms"]
        fp64_in = dict(ms_per_step=ms64i, value=n / (ms64i * 1e-3), unit="particles/s", dtype_in="f64",
                       output_equals_fp32_input=bool(same),
                       pipeline_GBps=(56.0 * n + 28.0 * n64i) / (ms64i * 1e-3) / 1e9,
                       roofline=dict(bound="hbm", achieved=b64 / (d64 * 1e-3) / 1e9, peak=HBM_PEAK_GBS, unit="GB/s",
                                     frac=b64 / (d64 * 1e-3) / 1e9 / HBM_PEAK_GBS, kernel=DOMINANT,
                                     kernel_avg_ms=d64, algorithmic_bytes_per_launch=b64),
                       kernels={k: round(v["avg_ms"], 4) for k, v in k64i.items()})
        log(f"[bench] fixed-point from FP64 input: {ms64i:.3f} ms/step, output equal to the FP32 run: {same}")
        del arrs64, out64i
    # The same event with every decision taken by the exact integer rule (the certified FP64
    # evaluation skipped): its output must equal the fast form's bit for bit.
    exact_check = None
    if not args.no_extra:
        saved = ctx.get_tuning()
        t = vpm.make_tuning(**{k: v for k, v in saved.as_dict().items() if k != "exact_decisions"}, exact_decisions=1)
        ctx.set_tuning(t)
        try:
            msx, outx, oox, nx, _, _ = time_fixed(ctx, vpm, arrs32, off, n, p32, 2, 1, False)
        finally:
            ctx.set_tuning(saved)
        same = nx == n_out and torch.equal(oox, out_off) and all(
            torch.equal(a[:n_out].view(torch.int32), b[:n_out].view(torch.int32)) for a, b in zip(outx, out32))
        exact_check = dict(ms_per_step=msx, output_equals_fast_form=bool(same),
                           note="every Step 3-5 decision by the exact 128/256/320-bit rule")
        log(f"[bench] exact decisions everywhere: {msx:.3f} ms/step, output equal: {same}")
        del outx
    del out32
    torch.cuda.empty_cache()

    plain = None
    if not args.no_fp64:
        plain = time_plain(ctx, vpm, wl64, prm, args.fp64_steps)
        plain["speedup_batched_over_plain"] = plain["ms_per_step"] / ms_step
        log(f"[bench] plain FP64: {plain['ms_per_step']:.3f} ms/step, speedup {plain['speedup_batched_over_plain']:.1f}x")

    cpu = None
    pl_dom = None
    if not args.no_cpu:
        import oracle
        cores = oracle_threads()
        ta = time.perf_counter()
        ref = oracle.run_workload(wl32, decide=oracle.FIXED, n_threads=cores)
        dt = time.perf_counter() - ta
        cpu = dict(value=n / dt, unit="particles/s", cores=cores, kind="oracle", host=host_cpu(),
                   sample=f"all {n_cells} cells ({n} particles) of the same workload, fixed-point decisions, "
                          f"pair merge, {dt:.2f} s wall on {cores} threads (every CPU the process may use, "
                          f"capped by OMP_NUM_THREADS when set)")
        log(f"[bench] oracle: {dt:.2f} s on {cores} threads")
        # The tree the method builds on this workload, from the same oracle run, and whether the GPU's
        # per-cell output counts equal the oracle's over every cell.
        st = ref.stats
        done = st["n_nodes"] > 0
        pl_dom = float(st["particle_levels"][in_a].sum())
        cpu["tree"] = dict(cells_processed=int(done.sum()),
                           visited_subsets_per_cell=float(st["n_nodes"][done].mean()),
                           mean_max_depth=float(st["max_depth"][done].mean()),
                           max_depth=int(st["max_depth"].max()),
                           particle_levels_per_particle=float(st["particle_levels"].sum()) / n,
                           gpu_out_counts_equal=bool(np.array_equal(np.asarray(ref.out_off), gpu_out_off)))
        del ref
        # The same oracle on one thread, over every 16th cell.
        part = wl32.cells(np.arange(0, n_cells, 16))
        ta = time.perf_counter()
        oracle.run_workload(part, decide=oracle.FIXED, n_threads=1)
        d1 = time.perf_counter() - ta
        cpu["single_thread"] = dict(value=part.n / d1, unit="particles/s",
                                    sample=f"every 16th cell ({part.n} particles), {d1:.2f} s wall on 1 thread")
        log(f"[bench] oracle: {d1:.2f} s on 1 thread for {part.n} particles; tree {cpu['tree']}")
        del part

    extra = None
    if not args.no_extra:
        del arrs32
        torch.cuda.empty_cache()
        extra = {}
        ts_paper = W.two_stream_grid(nx=256, ny=256, mean=512, seed=args.seed, params=W.TWO_STREAM_PAPER_PARAMS)
        extra["two_stream_paper_tolerances"] = extra_workload(
            ctx, vpm, "two_stream_256x256_poisson512_T0.8_0.15_Nmin200", ts_paper.astype(np.float32),
            None if args.no_fp64 else ts_paper, dict(ts_paper.params), 10, 0 if args.no_fp64 else 2,
            cpu=not args.no_cpu, agreement=not args.no_fp64, seed=args.seed)
        extra["blind_vs_voronoi"] = blind_vs_voronoi(ctx, vpm, ts_paper.astype(np.float32), dict(ts_paper.params),
                                                     [0.965, 0.88], args.seed)
        del ts_paper
        sh = W.shower_grid(nc=64, seed=args.seed)
        sh64 = sh.astype(np.float64) if not args.no_fp64 else None
        extra["shower"] = extra_workload(ctx, vpm, "shower_64cubed_lognormal64", sh, sh64, dict(sh.params), 5,
                                         0 if args.no_fp64 else 1, cpu=not args.no_cpu,
                                         agreement=not args.no_fp64, seed=args.seed)
        del sh, sh64
        extra["shower_three_species"] = species_shower(ctx, vpm, W, args.seed)
        extra["whole_box"] = whole_box(ctx, vpm, W, args.seed, cpu=not args.no_cpu)
        if args.cascade_steps > 0:
            extra["cascade"] = cascade(ctx, vpm, W, args.cascade_steps, args.seed)
        if not args.no_fp64:
            extra["precision_sweep"] = precision_sweep(ctx, vpm, W, [128, 256, 512, 1024, 2048], args.seed)

    # The ALU side of the dominant kernel: issued VALU instructions (committed counter run) against
    # the VALU issue peak, and the algorithmic integer work (particle-levels of its cells, from the
    # oracle run, times the least lane operations per particle-level) against the int32 lane peak.
    t_dom = dom["avg_ms"] * 1e-3
    valu = valu_from_profiles()
    alu = {"issue": None if valu is None else
           {"valu_insts_per_launch": valu, "achieved": valu / t_dom, "peak": VALU_PEAK_INSTS,
            "unit": "VALU wave-instructions/s", "frac": valu / t_dom / VALU_PEAK_INSTS},
           "algorithmic": None if pl_dom is None else
           {"particle_levels_per_launch": pl_dom, "lane_ops_per_particle_level": LANE_OPS_PER_PARTICLE_LEVEL,
            "achieved": pl_dom * LANE_OPS_PER_PARTICLE_LEVEL / t_dom, "peak": ALU_PEAK_LANE_OPS,
            "unit": "int32 lane-ops/s", "frac": pl_dom * LANE_OPS_PER_PARTICLE_LEVEL / t_dom / ALU_PEAK_LANE_OPS}}

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
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": DOMINANT,
                     "kernel_avg_ms": dom["avg_ms"], "algorithmic_bytes_per_launch": bytes_dom},
        "alu": alu,
        "cpu_baseline": cpu,
        "timing": dict(mode="HIP graph replay of the whole merge event" if args.graph else
                       "eager calls, no profiling events in the timed steps", **timing),
        "tuning": tuning,
        "autotune_s": tune_s,
        "merge_ratio": rho,
        "pipeline_GBps": bytes_step / (ms_step * 1e-3) / 1e9,
        "kernels": kernels,
        "conservation": cons32,
        "merged_cv": cv32,
        "plain_fp64": plain,
        "fp64_input": fp64_in,
        "exact_decisions_check": exact_check,
        "device_flags": flags,
        "workloads": extra,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()

"""Repeated merge events replayed from one captured HIP graph.

vpm_run reads the population size from cell_off on the device, so a graph captured once over fixed
buffers can be replayed for events whose particle counts differ.  Every replay is checked bit for bit
against an eager call on the same population; eager library work and host synchronisation run
between the replays.  Offsets that are invalid are reported through the device flags.
"""
import numpy as np
import pytest

import oracle
from paper_1504_00636_amd import vpm, workloads as W
from tests.gpu_common import ctx, oracle_params

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

PARAMS = dict(tol_x=0.3, tol_p=0.08, n_min_cell=0, min_subset=4, cell_len=(1.0, 1.0, 1.0), mass=1.0)


def population(sizes, seed):
    r = np.random.Generator(np.random.Philox(seed))
    cells = []
    for k in sizes:
        cells.append(np.stack([r.random(k), r.random(k), r.random(k), 1.0 + 0.1 * r.standard_normal(k),
                               0.5 + 0.05 * r.standard_normal(k), -0.3 + 0.05 * r.standard_normal(k),
                               0.5 + r.random(k)], axis=1))
    return W.from_cells(cells, params=dict(PARAMS), dtype=np.float32)


def eager(c, wl, merge):
    arrs, off = vpm.upload(wl)
    res = vpm.run_population(c, arrs, off, vpm.make_params(merge_mode=merge, **PARAMS))
    torch.cuda.synchronize()
    return [t[:res.out_total].clone() for t in res.out], res.out_off.clone(), res.out_total


def load(wl, bufs, off_buf):
    for t, a in zip(bufs, wl.arrays()):
        t[:wl.n].copy_(torch.from_numpy(np.ascontiguousarray(a)))
    off_buf.copy_(torch.from_numpy(wl.cell_off))


@pytest.mark.parametrize("merge,concurrent", [(vpm.VPM_MERGE_PAIR, 0), (vpm.VPM_MERGE_CENTROID, 0),
                                              (vpm.VPM_MERGE_PAIR, 1), (vpm.VPM_MERGE_PAIR, 2)])
def test_graph_replay_matches_eager(merge, concurrent):
    """concurrent = 1 or 2: size bins run on forked side streams inside the captured graph."""
    sizes1 = [300, 40, 3, 0, 700, 2100, 64, 5000, 17]
    sizes2 = [20, 600, 0, 1, 580, 900, 4400, 12, 64]          # same cell count, other sizes
    wl1, wl2 = population(sizes1, 11), population(sizes2, 12)
    cap = max(wl1.n, wl2.n) + 37
    c = ctx(cap, len(sizes1))
    default = c.get_tuning()
    c.set_tuning(vpm.make_tuning(concurrent_bins=concurrent))
    try:
        _graph_replay(c, wl1, wl2, sizes1, cap, merge)
    finally:
        c.set_tuning(default)


def test_graph_replay_with_cells_above_2_16():
    """Whole-box cells inside a captured graph: their chunk and output tasks, and the job counters
    that each event resets, replay like the rest."""
    sizes1 = [300, 90000, 700, 5000]
    sizes2 = [70000, 40, 20000, 66000]
    wl1, wl2 = population(sizes1, 13), population(sizes2, 14)
    cap = max(wl1.n, wl2.n) + 37
    c = ctx(cap, len(sizes1))
    _graph_replay(c, wl1, wl2, sizes1, cap, vpm.VPM_MERGE_PAIR)


def _graph_replay(c, wl1, wl2, sizes1, cap, merge):
    refs = {1: eager(c, wl1, merge), 2: eager(c, wl2, merge)}
    # the eager result is the oracle's (so a replay that matches it matches the oracle)
    orc = oracle.run_workload(wl1, decide=oracle.FIXED, merge_mode=merge, **oracle_params(PARAMS))
    assert refs[1][2] == orc.out_total

    bufs = [torch.zeros(cap, dtype=torch.float32, device="cuda") for _ in range(7)]
    off_buf = torch.zeros(len(sizes1) + 1, dtype=torch.int64, device="cuda")
    out = [torch.zeros(cap, dtype=torch.float32, device="cuda") for _ in range(7)]
    out_off = torch.zeros(len(sizes1) + 1, dtype=torch.int64, device="cuda")
    out_total = torch.zeros(1, dtype=torch.int64, device="cuda")
    p = vpm.make_params(merge_mode=merge, **PARAMS)

    load(wl1, bufs, off_buf)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):                                # warm-up outside the capture
        c.run(bufs, off_buf, cap, p, out, out_off, out_total)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        c.run(bufs, off_buf, cap, p, out, out_off, out_total)
    torch.cuda.synchronize()

    for rep, k in enumerate([1, 2, 1, 2, 2, 1]):
        wl = wl1 if k == 1 else wl2
        load(wl, bufs, off_buf)
        for t in out:
            t.fill_(-1.0)
        g.replay()
        torch.cuda.synchronize()
        ref_out, ref_off, ref_tot = refs[k]
        assert int(out_total.item()) == ref_tot, rep
        assert torch.equal(out_off, ref_off), rep
        for a, b in zip(out, ref_out):
            assert torch.equal(a[:ref_tot].view(torch.int32), b.view(torch.int32)), rep
        # eager work between replays
        eager(c, wl2 if k == 1 else wl1, merge)
    assert c.device_status(clear=True) == 0


def test_bad_offsets_flagged_and_skipped():
    wl = population([50, 60, 70], 13)
    c = ctx(wl.n + 10, 3)
    arrs, off = vpm.upload(wl)
    bad = off.clone()
    bad[2] = bad[1] - 5                                            # cell 1 decreasing, cell 2 widened
    out = [torch.empty_like(a) for a in arrs]
    out_off = torch.empty(4, dtype=torch.int64, device="cuda")
    out_total = torch.empty(1, dtype=torch.int64, device="cuda")
    c.device_status(clear=True)
    c.run(arrs, bad, wl.n, vpm.make_params(**PARAMS), out, out_off, out_total)
    torch.cuda.synchronize()
    assert c.device_status(clear=True) & vpm.VPM_FLAG_BAD_OFFSETS
    oo = out_off.cpu().numpy()
    assert oo[2] - oo[1] == 0                                      # the decreasing cell emits nothing
    # offsets past the arrays are rejected the same way
    past = off.clone()
    past[3] = wl.n + 5
    c.run(arrs, past, wl.n, vpm.make_params(**PARAMS), out, out_off, out_total)
    torch.cuda.synchronize()
    assert c.device_status(clear=True) & vpm.VPM_FLAG_BAD_OFFSETS


def test_two_contexts_on_two_streams():
    """Two contexts (each with its own workspace) run at the same time on two streams of default
    priority; each result equals the same population's eager run on the shared context."""
    wl1 = population([300, 40, 3, 700, 2100, 64, 5000, 17], 21)
    wl2 = population([20, 600, 1, 580, 900, 4400, 12, 64, 129], 22)
    ref1 = eager(ctx(max(wl1.n, wl2.n), 16), wl1, vpm.VPM_MERGE_PAIR)
    ref2 = eager(ctx(), wl2, vpm.VPM_MERGE_PAIR)
    p = vpm.make_params(**PARAMS)
    runs = []
    for wl in (wl1, wl2):
        c = vpm.Context(0)
        c.reserve(wl.n, wl.n_cells)
        arrs, off = vpm.upload(wl)
        out = [torch.empty_like(a) for a in arrs]
        out_off = torch.empty(wl.n_cells + 1, dtype=torch.int64, device="cuda")
        out_total = torch.empty(1, dtype=torch.int64, device="cuda")
        runs.append((c, arrs, off, wl.n, out, out_off, out_total, torch.cuda.Stream()))
    torch.cuda.synchronize()
    for c, arrs, off, n, out, out_off, out_total, s in runs:
        with torch.cuda.stream(s):
            c.run(arrs, off, n, p, out, out_off, out_total)
    torch.cuda.synchronize()
    for (c, arrs, off, n, out, out_off, out_total, s), (r_out, r_off, r_tot) in zip(runs, (ref1, ref2)):
        tot = int(out_total.item())
        assert tot == r_tot and torch.equal(out_off, r_off)
        for a, b in zip(out, r_out):
            assert torch.equal(a[:tot].view(torch.int32), b.view(torch.int32))
        assert c.device_status(clear=True) == 0


def test_overlapping_offsets_write_nothing_past_n_particles():
    """Offsets that decrease let later cells overlap earlier ones ([0, 80, 30, 100]: cells 0 and 2
    share particles 30..79).  Their counts would add up past the arrays; out_total and out_off are
    clamped to n_particles and canaries past it stay untouched."""
    wl = population([80, 0, 70], 14)                  # 150 particles; only 100 are the call's
    n = 100
    c = ctx(n + 64, 3)
    arrs, _ = vpm.upload(wl)
    bad = torch.tensor([0, 80, 30, 100], dtype=torch.int64, device="cuda")
    canary = 64
    out = [torch.full((n + canary,), 7.0, dtype=torch.float32, device="cuda") for _ in range(7)]
    out_off = torch.empty(4, dtype=torch.int64, device="cuda")
    out_total = torch.empty(1, dtype=torch.int64, device="cuda")
    p = vpm.make_params(**dict(PARAMS, n_min_cell=1000))     # every cell copied: counts 80 + 0 + 70
    c.device_status(clear=True)
    c.run([a[:n] for a in arrs], bad, n, p, [o[:n] for o in out], out_off, out_total)
    torch.cuda.synchronize()
    assert c.device_status(clear=True) & vpm.VPM_FLAG_BAD_OFFSETS
    assert int(out_total.item()) <= n
    oo = out_off.cpu().numpy()
    assert np.all(np.diff(oo) >= 0) and oo[-1] <= n
    for o in out:
        assert torch.all(o[n:] == 7.0)

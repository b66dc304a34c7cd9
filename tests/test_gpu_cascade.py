"""The repeated-merge cascade: one merge event captured in a HIP graph and replayed on a population
that changes between replays (every particle split in two before each event, cells above N_min =
1,024 merged), each replay checked against the oracle on the same input.  The next event's input is
the oracle's output of this one (rounded to FP32), so no input comes from the GPU."""
import numpy as np
import pytest

import oracle
from paper_1504_00636_amd import vpm, workloads as W
from tests.gpu_common import FIELDS, check_merged_values, ctx, oracle_params

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

NX = 16
CAP = NX * NX * 16384                   # the largest population below (cells of 16,384 particles)


def _next_input(wl, ref, params):
    return W.Workload(wl.name, *[ref.out[f] for f in ("x", "y", "z", "px", "py", "pz", "w")],
                      cell_off=np.asarray(ref.out_off, np.int64), cell_id=None,
                      params=dict(params)).astype(np.float32)


@pytest.mark.parametrize("tol_p,steps", [(0.02, 6), (0.3, 5), (0.6, 50)])
def test_cascade_graph_replays(tol_p, steps):
    """tol_p 0.02 (the shower's tolerance) splits almost every subset down to single particles, so
    the population doubles up to cells of 16,384 (the global-slab bin); tol_p 0.3 merges, so the
    population size and the cell sizes (1,800 to 2,500 particles) change between replays; tol_p 0.6
    (the benchmark's cascade) holds the cells near N_min = 1,024 over 50 events (merged cells fall
    to a few hundred particles and grow back), every event checked on every cell."""
    wl = W.cascade_initial(nx=NX, ny=NX, seed=4)
    params = dict(wl.params, tol_p=tol_p)
    n_cells = wl.n_cells
    c = ctx(CAP, n_cells)
    Q = [torch.zeros(CAP, dtype=torch.float32, device="cuda") for _ in range(7)]
    P = [torch.zeros(CAP, dtype=torch.float32, device="cuda") for _ in range(7)]
    offQ = torch.zeros(n_cells + 1, dtype=torch.int64, device="cuda")
    offP = torch.full((n_cells + 1,), -1, dtype=torch.int64, device="cuda")
    out_total = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    p = vpm.make_params(decide=vpm.VPM_DECIDE_FIXED, merge_mode=vpm.VPM_MERGE_PAIR, **params)
    c.device_status(clear=True)
    g = None
    merged_steps = 0
    for step in range(steps):
        wl = W.cascade_split(wl, step, seed=4)
        assert wl.n <= CAP
        for t, a in zip(Q, wl.arrays()):
            t[:wl.n].copy_(torch.from_numpy(np.ascontiguousarray(a)))
        offQ.copy_(torch.from_numpy(wl.cell_off))
        offP.fill_(-1)
        out_total.fill_(-1)
        torch.cuda.synchronize()
        if g is None:                               # capture once; capturing runs nothing
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                c.run(Q, offQ, CAP, p, P, offP, out_total)
            torch.cuda.synchronize()
        print(f"cascade tol_p={tol_p} step {step}: {wl.n} particles, cells up to "
              f"{int(np.diff(wl.cell_off).max())}", flush=True)
        g.replay()
        torch.cuda.synchronize()
        ref = oracle.run_workload(wl, decide=oracle.FIXED, merge_mode=oracle.PAIR, **oracle_params(params))
        tot = int(out_total.item())
        assert tot == ref.out_total
        got = {f: P[i][:tot].cpu().numpy().astype(np.float64) for i, f in enumerate(FIELDS)}
        check_merged_values(wl, params, vpm.VPM_MERGE_PAIR, got, offP.cpu().numpy(), ref)
        merged_steps += int(ref.out_total < wl.n)
        wl = _next_input(wl, ref, params)
    assert c.device_status(clear=True) == 0
    if tol_p > 0.1:
        assert merged_steps >= 3

"""Launch configurations (lane-group sizing and size-bin limits) change how the work is batched, never
the result: every tuning, and the autotuner's choice, must reproduce the oracle's partition and the
default configuration's output bit for bit."""
import numpy as np
import pytest

import oracle
from paper_1504_00636_amd import vpm
from tests.gpu_common import ctx, oracle_params
from tests.test_gpu_graph import PARAMS, population

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SIZES = [1, 2, 5, 17, 64, 200, 575, 577, 900, 2047, 2049, 3000, 4353, 6000, 300, 12, 128, 129, 255, 256, 257,
         3, 4, 9, 33, 90, 110, 7, 40, 60, 1140, 2280, 4590]
TUNINGS = [(16, 576, 2048, 4352), (8, 64, 512, 1024, 1), (32, 320, 1024, 2560), (8, 1, 1, 1, 0, 0),
           (32, 576, 576, 576, 1), (16, 100, 2048, 2048), (16, 576, 2048, 4352, 1), (16, 576, 2048, 4352, 0, 0),
           (8, 576, 2048, 4352, 0, 256), (32, 576, 2048, 4352, 1, 17), (16, 576, 2048, 4352, 0, 128, 1),
           (8, 320, 1024, 2560, 1, 64, 1), (16, 576, 2048, 4352, 0, 128, 0, 576), (8, 200, 2048, 4352, 1, 64, 0, 700),
           (32, 576, 1144, 1144, 0, 128, 0, 1144), (16, 576, 2288, 4592, 1), (16, 576, 2288, 4592, 2),
           (8, 320, 1024, 2560, 2, 64, 0, 700)]


def _run(c, arrs, off, n, p):
    out = [torch.empty_like(a) for a in arrs]
    out_off = torch.empty(off.numel(), dtype=torch.int64, device="cuda")
    out_total = torch.empty(1, dtype=torch.int64, device="cuda")
    c.run(arrs, off, n, p, out, out_off, out_total)
    torch.cuda.synchronize()
    tot = int(out_total.item())
    return [t[:tot].clone() for t in out], out_off.clone(), tot


def _partition(c, arrs, off, n, n_cells, p):
    perm = torch.empty(n, dtype=torch.int32, device="cuda")
    sid = torch.empty(n, dtype=torch.int32, device="cuda")
    nsub = torch.empty(n_cells, dtype=torch.int32, device="cuda")
    c.partition(arrs, off, n, p, perm, sid, nsub)
    torch.cuda.synchronize()
    return perm.cpu().numpy(), sid.cpu().numpy(), nsub.cpu().numpy()


def _same(a, b):
    (oa, fa, ta), (ob, fb, tb) = a, b
    assert ta == tb and torch.equal(fa, fb)
    for x, y in zip(oa, ob):
        assert torch.equal(x.view(torch.int32), y.view(torch.int32))


@pytest.mark.parametrize("merge", [vpm.VPM_MERGE_PAIR, vpm.VPM_MERGE_CENTROID])
def test_every_tuning_gives_identical_results(merge):
    wl = population(SIZES, 21)
    c = ctx(wl.n, wl.n_cells)
    default = c.get_tuning()
    p = vpm.make_params(merge_mode=merge, **PARAMS)
    arrs, off = vpm.upload(wl)
    ref = oracle.run_workload(wl, decide=oracle.FIXED, merge_mode=merge, **oracle_params(PARAMS))
    try:
        base = _run(c, arrs, off, wl.n, p)
        assert base[2] == ref.out_total
        for t in TUNINGS:
            c.set_tuning(vpm.make_tuning(*t))
            assert c.get_tuning().as_dict() == vpm.make_tuning(*t).as_dict()
            perm, sid, nsub = _partition(c, arrs, off, wl.n, wl.n_cells, p)
            np.testing.assert_array_equal(nsub, ref.n_subsets, err_msg=str(t))
            np.testing.assert_array_equal(perm, ref.perm, err_msg=str(t))
            np.testing.assert_array_equal(sid, ref.subset_id, err_msg=str(t))
            _same(_run(c, arrs, off, wl.n, p), base)
    finally:
        c.set_tuning(default)
    assert c.device_status(clear=True) == 0


def test_autotune_choice_is_valid_and_exact():
    wl = population(SIZES * 8, 22)
    c = ctx(wl.n, wl.n_cells)
    default = c.get_tuning()
    p = vpm.make_params(**PARAMS)
    arrs, off = vpm.upload(wl)
    try:
        base = _run(c, arrs, off, wl.n, p)
        out = [torch.empty_like(a) for a in arrs]
        out_off = torch.empty(off.numel(), dtype=torch.int64, device="cuda")
        out_total = torch.empty(1, dtype=torch.int64, device="cuda")
        best = c.autotune(arrs, off, wl.n, p, out, out_off, out_total)
        torch.cuda.synchronize()
        assert vpm.vpm_check_tuning(best) == vpm.VPM_OK
        assert c.get_tuning().as_dict() == best.as_dict()
        tot = int(out_total.item())
        _same(([t[:tot] for t in out], out_off, tot), base)
        _same(_run(c, arrs, off, wl.n, p), base)
    finally:
        c.set_tuning(default)


@pytest.mark.parametrize("axis_rule", [0, 1])
def test_exact_rule_everywhere_gives_identical_results(axis_rule):
    """Every decision taken by the exact integer rule (exact_decisions = 1, the certified FP64
    evaluation skipped) on populations where the FP64 filter decides nearly everything: the
    two-stream grid (64 x 64 cells, Poisson(512)) and the shower shape (16^3 cells, every size bin),
    each at its own tolerances.  Partition and output must equal the fast form's bit for bit."""
    from paper_1504_00636_amd import workloads as W
    pops = [W.two_stream_grid(nx=64, ny=64, seed=5).astype(np.float32), W.shower_grid(nc=16, seed=6)]
    for wl in pops:
        c = ctx(wl.n, wl.n_cells)
        default = c.get_tuning()
        prm = dict(wl.params, axis_rule=axis_rule)
        p = vpm.make_params(**prm)
        arrs, off = vpm.upload(wl)
        try:
            c.set_tuning(vpm.make_tuning())
            fast = _run(c, arrs, off, wl.n, p), _partition(c, arrs, off, wl.n, wl.n_cells, p)
            c.set_tuning(vpm.make_tuning(exact_decisions=1))
            exact = _run(c, arrs, off, wl.n, p), _partition(c, arrs, off, wl.n, wl.n_cells, p)
        finally:
            c.set_tuning(default)
        _same(exact[0], fast[0])
        for a, b in zip(exact[1], fast[1]):
            np.testing.assert_array_equal(a, b)
        assert c.device_status(clear=True) == 0

"""FP64 particles on the fixed-point path: the kernels round each value to FP32 as they load it, so an
FP64 population must give exactly the output of the same population rounded to FP32 on the host
(vpm_run over every size bin and both merges, vpm_partition, vpm_merge, vpm_blind).  The output of
the fixed-point path is FP32 in both cases."""
import numpy as np
import pytest

from paper_1504_00636_amd import vpm, workloads as W
from tests.gpu_common import ctx

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

PARAMS = dict(tol_x=0.3, tol_p=0.08, n_min_cell=2, min_subset=4, cell_len=(1.0, 1.0, 1.0), mass=1.0)


def population(sizes, seed):
    r = np.random.Generator(np.random.Philox(seed))
    cells = []
    for k in sizes:
        cells.append(np.stack([r.random(k), r.random(k), r.random(k), 1.0 + 0.1 * r.standard_normal(k),
                               0.5 + 0.05 * r.standard_normal(k), -0.3 + 0.05 * r.standard_normal(k),
                               0.5 + r.random(k)], axis=1))
    return W.from_cells(cells, params=dict(PARAMS), dtype=np.float64)


def _run(c, wl, dtype, **kw):
    arrs, off = vpm.upload(wl, dtype=dtype)
    p = vpm.make_params(dtype=vpm.VPM_F64 if dtype == torch.float64 else vpm.VPM_F32, **dict(PARAMS, **kw))
    res = vpm.run_population(c, arrs, off, p)
    torch.cuda.synchronize()
    assert all(t.dtype == torch.float32 for t in res.out)
    return [t[:res.out_total].clone() for t in res.out], res.out_off.clone(), res.out_total


def _same(a, b):
    assert a[2] == b[2] and torch.equal(a[1], b[1])
    for x, y in zip(a[0], b[0]):
        assert torch.equal(x.view(torch.int32), y.view(torch.int32))


@pytest.mark.parametrize("merge", [vpm.VPM_MERGE_PAIR, vpm.VPM_MERGE_CENTROID])
@pytest.mark.parametrize("concurrent", [0, 1, 2])
def test_fp64_input_equals_host_rounded_fp32(merge, concurrent):
    wl = population([300, 40, 3, 0, 700, 2100, 64, 5000, 17, 9000, 130, 1, 577, 4400], 51)
    c = ctx(wl.n, wl.n_cells)
    default = c.get_tuning()
    c.set_tuning(vpm.make_tuning(concurrent_bins=concurrent))
    try:
        a = _run(c, wl, torch.float64, merge_mode=merge)
        b = _run(c, wl.astype(np.float32), torch.float32, merge_mode=merge)
    finally:
        c.set_tuning(default)
    _same(a, b)
    assert a[2] < wl.n


def test_fp64_two_stream_grid():
    wl = W.two_stream_grid(nx=48, ny=48, seed=3)
    c = ctx(wl.n, wl.n_cells)
    _same(_run(c, wl, torch.float64), _run(c, wl.astype(np.float32), torch.float32))


def test_fp64_partition_merge_and_blind():
    wl = population([500, 64, 3000, 9, 6000], 52)
    c = ctx(wl.n, wl.n_cells)
    outs = {}
    for dt in (torch.float64, torch.float32):
        w = wl if dt == torch.float64 else wl.astype(np.float32)
        arrs, off = vpm.upload(w, dtype=dt)
        p = vpm.make_params(dtype=vpm.VPM_F64 if dt == torch.float64 else vpm.VPM_F32, **PARAMS)
        perm = torch.empty(wl.n, dtype=torch.int32, device="cuda")
        sid = torch.empty_like(perm)
        nsub = torch.empty(wl.n_cells, dtype=torch.int32, device="cuda")
        c.partition(arrs, off, wl.n, p, perm, sid, nsub)
        out = [torch.empty(wl.n, dtype=torch.float32, device="cuda") for _ in range(7)]
        oo = torch.empty(wl.n_cells + 1, dtype=torch.int64, device="cuda")
        ot = torch.empty(1, dtype=torch.int64, device="cuda")
        c.merge(arrs, off, wl.n, p, perm, sid, nsub, out, oo, ot)
        bout = [torch.empty(wl.n, dtype=torch.float32, device="cuda") for _ in range(7)]
        boo = torch.empty_like(oo)
        bot = torch.empty_like(ot)
        grp = torch.empty_like(perm)
        c.blind(arrs, off, wl.n, p, 0.7, 9, bout, boo, bot, grp)
        torch.cuda.synchronize()
        k, bk = int(ot.item()), int(bot.item())
        outs[dt] = (perm, sid, nsub, [t[:k] for t in out], oo, [t[:bk] for t in bout], boo, grp)
    a, b = outs[torch.float64], outs[torch.float32]
    for x, y in zip(a[:3], b[:3]):
        assert torch.equal(x, y)
    assert torch.equal(a[4], b[4]) and torch.equal(a[6], b[6]) and torch.equal(a[7], b[7])
    for x, y in zip(a[3] + a[5], b[3] + b[5]):
        assert torch.equal(x.view(torch.int32), y.view(torch.int32))


def test_fp64_input_cells_above_2_16():
    """Whole-box cells from FP64 arrays: the frame and codes chunk tasks round as they load, so the
    output equals that of the host-rounded FP32 population."""
    wl = population([90000, 500, 140000], 53)
    c = ctx(wl.n, wl.n_cells)
    a = _run(c, wl, torch.float64)
    b = _run(c, wl.astype(np.float32), torch.float32)
    _same(a, b)
    assert a[2] < wl.n

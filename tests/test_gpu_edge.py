"""Degenerate inputs on the GPU, each against the oracle: empty calls, cells of identical particles
(every coefficient of variation zero), cells where one particle carries almost all the weight (the
others get weight code 0), zero tolerances, a minimum subset size above every cell, and single
particles, in every size bin."""
import numpy as np
import pytest

from paper_1504_00636_amd import vpm, workloads as W
from tests.gpu_common import ctx
from tests.test_gpu_parity import full_check

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

BASE = dict(tol_x=0.3, tol_p=0.08, n_min_cell=0, min_subset=4, cell_len=(1.0, 1.0, 1.0), mass=1.0)
SIZES = [1, 2, 5, 64, 129, 600, 2100, 4400]        # small batches, every bin


@pytest.mark.parametrize("n_cells", [0, 3])
def test_empty_call(n_cells):
    """No cells, or only empty cells: offsets all zero, total zero, no flags raised."""
    c = ctx()
    inp = [torch.zeros(1, dtype=torch.float32, device="cuda") for _ in range(7)]
    out = [torch.zeros(1, dtype=torch.float32, device="cuda") for _ in range(7)]
    off = torch.zeros(n_cells + 1, dtype=torch.int64, device="cuda")
    out_off = torch.full((n_cells + 1,), -1, dtype=torch.int64, device="cuda")
    out_total = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    c.device_status(clear=True)
    c.run(inp, off, 0, vpm.make_params(**BASE), out, out_off, out_total)
    torch.cuda.synchronize()
    assert int(out_total.item()) == 0 and not out_off.any()
    assert c.device_status(clear=True) == 0


@pytest.mark.parametrize("merge", [vpm.VPM_MERGE_PAIR, vpm.VPM_MERGE_CENTROID])
def test_identical_particles(merge):
    r = np.random.Generator(np.random.Philox(31))
    cells = []
    for k in SIZES:
        row = np.array([r.random(), r.random(), r.random(), 0.7, -0.2, 0.1, 0.9])
        cells.append(np.tile(row, (k, 1)))
    wl = W.from_cells(cells, params=dict(BASE), dtype=np.float32)
    ref = full_check(wl, dict(BASE), merge)
    big = [i for i, k in enumerate(SIZES) if k >= 4]
    assert all(ref.n_subsets[i] == 1 for i in big)              # one subset: every CV is zero


def test_heavy_particles_among_weightless():
    r = np.random.Generator(np.random.Philox(32))
    cells = []
    for k in SIZES:
        c = np.stack([r.random(k), r.random(k), r.random(k), 1.0 + 0.1 * r.standard_normal(k),
                      0.5 + 0.05 * r.standard_normal(k), 0.2 + 0.05 * r.standard_normal(k),
                      np.full(k, 1e-7)], axis=1)
        c[k // 2, 6] = 1.0                                      # the others code to weight 0
        c[0, 6] = 0.75 if k > 2 else c[0, 6]                    # a second heavy one: cuts between them
        cells.append(c)
    wl = W.from_cells(cells, params=dict(BASE), dtype=np.float32)
    ref = full_check(wl, dict(BASE))
    assert ref.n_subsets[-1] > 1


def test_zero_tolerances_and_large_min_subset():
    r = np.random.Generator(np.random.Philox(33))
    cells = [np.stack([np.floor(4 * r.random(k)) / 4, np.zeros(k), np.zeros(k),
                       np.floor(3 * r.random(k)), np.ones(k), np.ones(k), np.ones(k)], axis=1) for k in SIZES]
    wl = W.from_cells(cells, params=dict(BASE), dtype=np.float32)
    full_check(wl, dict(BASE, tol_x=0.0, tol_p=0.0, min_subset=2))
    ref = full_check(wl, dict(BASE, min_subset=5000))            # nothing is merged
    assert ref.out_total == wl.n


def test_unbalanced_splits():
    """Cells whose heavy particles pull the weighted mean to one side, so that splits peel off a few
    particles at a time: some subsets keep most of the cell for several levels (the lane groups of
    the top levels then hold far more particles than usual, and the scheduler takes over early)."""
    r = np.random.Generator(np.random.Philox(34))
    cells = []
    for k in [140, 300, 520, 570]:
        light = np.stack([0.4 * r.random(k), r.random(k), r.random(k), 1.0 + 0.01 * r.standard_normal(k),
                          0.5 + 0.01 * r.standard_normal(k), 0.2 + 0.01 * r.standard_normal(k), np.ones(k)], axis=1)
        h = 6
        heavy = np.stack([0.95 - 0.05 * np.arange(h), r.random(h), r.random(h), np.full(h, 1.0), np.full(h, 0.5),
                          np.full(h, 0.2), 2.0 ** (12 - np.arange(h))], axis=1)
        c = np.concatenate([light, heavy])
        r.shuffle(c)
        cells.append(c[:k])
    params = dict(BASE, tol_x=0.05, tol_p=0.005)
    wl = W.from_cells(cells, params=params, dtype=np.float32)
    for ms in (2, 4):
        ref = full_check(wl, dict(params, min_subset=ms))
        assert ref.stats["max_depth"].max() >= 10                  # deeper than a balanced tree


def test_massless_photons():
    """Photons (mass 0, energy |p|) in shower-shaped cells, tolerances loose enough that subsets
    merge: both merges on the fixed-point path, and the pair merge on the FP64 path."""
    from tests.test_gpu_parity import _fp64_check, _sampled_check
    wl = W.shower_grid(nc=10, seed=5)
    params = dict(wl.params, mass=0.0, tol_p=1.0, tol_x=0.5)
    sample = np.arange(0, wl.n_cells, 3)
    for merge in (vpm.VPM_MERGE_PAIR, vpm.VPM_MERGE_CENTROID):
        _sampled_check(wl, params, sample, merge)
    small = W.shower_grid(nc=5, seed=6, dtype=np.float64)
    assert _fp64_check(small, dict(params)) <= 1

"""Cells above 2^16 particles on the GPU (a whole simulation box merged as one cell) against the oracle.

The method's first subset may be the whole box (the paper's remark after the algorithm on merging
globally).  The fixed-point library takes cells of up to 2^24 particles: subsets above 2^16 are split
by one workgroup each with exact integer moments (their |S1| can pass 2^53), and their unfinished
children are handed to other workgroups.  Bar: final-subset membership and order bit-exact, output
counts exact, copied particles bit-identical, merged particles within 1e-6, as for the other cells.
"""
import numpy as np
import pytest

import oracle
from paper_1504_00636_amd import vpm, workloads as W
from tests.gpu_common import ctx, gpu_partition, gpu_run, oracle_params
from tests.test_gpu_parity import CLOUD, cloud_cells, full_check

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def heavy_cell(n, seed):
    """Weights within 10 % of the largest and momenta near the top of their axis's code range, so
    that the root's S1 of px passes 2^53 once n is above about 70,000."""
    r = np.random.Generator(np.random.Philox(seed))
    return np.stack([r.random(n), r.random(n), r.random(n), 3.0 + r.random(n), 1.0 + 0.1 * r.random(n),
                     -2.1 + 0.1 * r.random(n), 0.9 + 0.1 * r.random(n)], axis=1)


HEAVY = dict(tol_x=0.25, tol_p=0.02, n_min_cell=0, min_subset=4, cell_len=(1.0, 1.0, 1.0), mass=1.0)


def root_s1_px(rows):
    """|S1| of the px codes over a whole cell, in exact integers (the fixed-point encoding of the
    weights and the px momenta, from the FP32 values)."""
    w = rows[:, 6].astype(np.float32)
    e_w = np.frexp(w.max())[1]
    om = np.rint(np.ldexp(w, 15 - e_w).astype(np.float32)).astype(np.int64)
    p = rows[:, 3].astype(np.float32)
    e_p = np.frexp(np.abs(p).max())[1]
    c = np.rint(np.ldexp(p, 22 - e_p).astype(np.float32)).astype(np.int64)
    return abs(sum(int(v) for v in om * c))


@pytest.mark.parametrize("merge", [vpm.VPM_MERGE_PAIR, vpm.VPM_MERGE_CENTROID])
def test_cells_above_2_16_with_small_ones(merge):
    """Cells of 65,537 and 150,000 particles in one launch with ordinary ones."""
    wl = cloud_cells([600, 65537, 3000, 150000, 40], seed=21)
    full_check(wl, CLOUD, merge)


def test_sums_past_2_53():
    """A 300,000-particle box whose top subsets have |S1| > 2^53: the exact wide moments decide."""
    rows = heavy_cell(300000, seed=22)
    assert root_s1_px(rows) > 2 ** 53
    wl = W.from_cells([rows], params=dict(HEAVY), dtype=np.float32)
    ref = full_check(wl, HEAVY)
    assert ref.n_subsets[0] > 8


def test_whole_box_counter_blocks():
    """The counter-propagating blocks, scaled to 120,000 electrons, merged as one box: the
    partition and the merged particles match the oracle and no subset mixes the blocks."""
    wl = W.counter_blocks(per_cell=120)
    assert wl.n == 120000
    params = dict(wl.params, cell_len=(100.0, 20.0, 1.0), tol_x=0.02)
    box = W.Workload("box", *[getattr(wl, f) for f in W.FIELDS], cell_off=np.array([0, wl.n], np.int64),
                     cell_id=None, params=params)
    ref = full_check(box, params)
    px = ref.out["px"]
    assert ref.out_total < box.n and np.all(np.abs(np.abs(px) - 150.0) < 1e-9)


def test_largest_cell_limits():
    """The fixed-point form takes a cell of 2^24 + 1 particles as too large (flagged, copied
    unchanged); the FP64 form keeps its limit of 2^16."""
    c = ctx()
    n = (1 << 24) + 1
    r = np.random.Generator(np.random.Philox(23))
    rows = np.empty((n, 7), np.float32)
    rows[:, :3] = r.random((n, 3), dtype=np.float32)
    rows[:, 3:6] = 1.0 + 0.01 * r.standard_normal((n, 3), dtype=np.float32)
    rows[:, 6] = 1.0
    wl = W.from_cells([rows[:5], rows], params={}, dtype=np.float32)
    c.device_status(clear=True)
    perm, sid, nsub = gpu_partition(wl, CLOUD)
    assert c.device_status(clear=True) & vpm.VPM_FLAG_CELL_TOO_LARGE
    assert nsub[1] == 0 and np.all(sid[5:] == -1)
    del perm, sid
    wl2 = cloud_cells([65537, 700], seed=24, dtype=np.float64)
    perm, sid, nsub = gpu_partition(wl2, CLOUD, decide=vpm.VPM_DECIDE_FP64)
    assert c.device_status(clear=True) & vpm.VPM_FLAG_CELL_TOO_LARGE
    assert nsub[0] == 0 and nsub[1] > 0


def test_wide_lattice_zero_tolerance():
    """T = 0 on a 90,000-particle cell drawn from a small lattice: the final subsets are the
    duplicate classes, reached through exact ties between axes (ties go to the lowest axis) and
    zero-variance axes, all decided on the exact wide moments at the top."""
    r = np.random.Generator(np.random.Philox(25))
    k = 90000
    base = r.integers(0, 3, size=(k, 6)).astype(np.float64)
    base[:, :3] *= 1000.0
    base[:, 3:] -= 1.0
    w = r.integers(1, 4, size=(k, 1)).astype(np.float64)
    params = dict(tol_x=0.0, tol_p=0.0, n_min_cell=0, min_subset=1, cell_len=(65536.0,) * 3, mass=1.0)
    wl = W.from_cells([np.concatenate([base, w], axis=1), np.concatenate([base[:500], w[:500]], axis=1)],
                      params=params, dtype=np.float32)
    ref = full_check(wl, params, vpm.VPM_MERGE_CENTROID)
    assert ref.n_subsets[0] == len({tuple(v) for v in base.tolist()})


@pytest.mark.parametrize("axis_rule", [0, 1])
def test_wide_normalised_rule_and_photons(axis_rule):
    """The tolerance-normalised axis rule and massless particles with one momentum axis all zero,
    on cells above 2^16 (the exact wide decisions weigh each CV by its tolerance)."""
    rows = heavy_cell(200000, seed=26)
    ph = heavy_cell(80000, seed=27)
    ph[:, 5] = 0.0                                   # pz = 0 throughout: a zero momentum axis
    prm = dict(HEAVY, tol_p=0.03, axis_rule=axis_rule, mass=0.0)
    wl = W.from_cells([rows, ph], params=dict(prm), dtype=np.float32)
    full_check(wl, prm)


def test_wide_cells_with_concurrent_bins():
    """With the size bins on concurrent streams, idle workgroups of the large-cell kernel leave
    instead of waiting for tasks: the chunk and output tasks of cells above 2^16 are then taken by
    the workgroups that spawn them.  Same bits as the default configuration."""
    c = ctx()
    wl = cloud_cells([70000, 3000, 130000, 500, 5000], seed=28)
    saved = c.get_tuning()
    try:
        c.set_tuning(vpm.make_tuning(concurrent_bins=1))
        got, got_off, tot = gpu_run(wl, CLOUD)
    finally:
        c.set_tuning(saved)
    ref, ref_off, ref_tot = gpu_run(wl, CLOUD)
    assert tot == ref_tot
    np.testing.assert_array_equal(got_off, ref_off)
    for f in got:
        np.testing.assert_array_equal(got[f], ref[f])


def test_wide_cell_with_a_bad_value_passes_through():
    """A NaN in a 100,000-particle cell: the cell is flagged and copied unchanged (its identity
    partition in vpm_partition), the other cells are merged as usual."""
    c = ctx()
    wl = cloud_cells([3000, 100000, 90000], seed=29)
    lo = int(wl.cell_off[1])
    wl.px[lo + 777] = np.nan
    c.device_status(clear=True)
    perm, sid, nsub = gpu_partition(wl, CLOUD)
    assert c.device_status(clear=True) & vpm.VPM_FLAG_BAD_VALUE
    hi = int(wl.cell_off[2])
    assert nsub[1] == 0 and np.all(sid[lo:hi] == -1) and np.array_equal(perm[lo:hi], np.arange(lo, hi))
    got, got_off, tot = gpu_run(wl, CLOUD)
    c.device_status(clear=True)
    o = int(got_off[1])
    assert got_off[2] - got_off[1] == hi - lo
    np.testing.assert_array_equal(got["w"][o:o + hi - lo], wl.w[lo:hi].astype(np.float32).astype(np.float64))
    good = wl.cells([0, 2])
    ref = oracle.run_workload(good, decide=oracle.FIXED, **oracle_params(CLOUD))
    assert nsub[0] == ref.n_subsets[0] and nsub[2] == ref.n_subsets[1]

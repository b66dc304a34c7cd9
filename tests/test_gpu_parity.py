"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Bar (fixed-point FP32 path): final-subset membership and order bit-exact, output counts exact,
copied particles bit-identical, merged particles within 1e-6 (relative to W, L, the merged energy)
plus one FP32 rounding of the stored value.  FP64 path: partitions equal except at certified
near-ties, merged values within 1e-12.
"""
import numpy as np
import pytest

import oracle
from paper_1504_00636_amd import vpm, workloads as W
from tests.gpu_common import (FIELDS, check_merged_values, check_partition_equal, gpu_partition, gpu_run,
                              oracle_params)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MERGES = [vpm.VPM_MERGE_PAIR, vpm.VPM_MERGE_CENTROID]
CLOUD = dict(tol_x=0.3, tol_p=0.08, n_min_cell=0, min_subset=4, cell_len=(1.0, 1.0, 1.0), mass=1.0)


def cloud_cells(sizes, seed=0, spread=0.05, dtype=np.float32):
    """Cells whose momenta have nonzero means, so that subsets merge."""
    r = np.random.Generator(np.random.Philox(seed))
    cells = []
    for k in sizes:
        px = 1.0 + 2 * spread * r.standard_normal(k)
        py = 0.5 + spread * r.standard_normal(k)
        pz = -0.3 + spread * r.standard_normal(k)
        cells.append(np.stack([r.random(k), r.random(k), r.random(k), px, py, pz, 0.5 + r.random(k)], axis=1))
    return W.from_cells(cells, params=dict(CLOUD), dtype=dtype)


def full_check(wl, params, merge=vpm.VPM_MERGE_PAIR):
    ref = oracle.run_workload(wl, decide=oracle.FIXED, merge_mode=merge, **oracle_params(params))
    check_partition_equal(wl, params, ref=ref, merge=merge)
    got, got_off, tot = gpu_run(wl, params, merge=merge)
    assert tot == ref.out_total
    check_merged_values(wl, params, merge, got, got_off, ref)
    return ref


def test_single_cell_two_beams():
    wl = W.single_cell_two_beams().astype(np.float32)
    full_check(wl, wl.params)


@pytest.mark.parametrize("merge", MERGES)
def test_merging_cloud(merge):
    wl = cloud_cells([300, 257, 64, 1000, 5, 4, 3, 2, 1, 0, 700], seed=1)
    params = dict(CLOUD, min_subset=4 if merge == vpm.VPM_MERGE_PAIR else 2)
    ref = full_check(wl, params, merge)
    assert ref.stats["n_merged"].sum() > 50


@pytest.mark.parametrize("merge", MERGES)
def test_size_bins_and_ragged_tails(merge):
    """Sizes around every lane-group size and size-bin boundary (576, 1144, 2288 and 4592 particles
    in LDS with 1, 2, 4 and 8 wavefronts per cell, larger cells in global slabs)."""
    sizes = [1, 2, 3, 4, 5, 7, 8, 9, 15, 16, 17, 31, 32, 33, 63, 64, 65, 255, 256, 257, 511, 512, 513,
             575, 576, 577, 1023, 1024, 1025, 1143, 1144, 1145, 2047, 2048, 2049, 2288, 2289, 4095, 4096,
             4097, 4352, 4353, 4591, 4592, 4593, 9001]
    wl = cloud_cells(sizes, seed=2, spread=0.08)
    full_check(wl, dict(CLOUD, min_subset=3), merge)


def test_untouched_and_empty_cells():
    wl = cloud_cells([0, 5, 20, 0, 21, 22, 0], seed=3)
    params = dict(CLOUD, n_min_cell=20)
    ref = full_check(wl, params)
    assert all(ref.n_subsets[c] == 0 for c in (0, 1, 2, 3, 6)) and ref.n_subsets[4] > 0
    perm, sid, nsub = gpu_partition(wl, params)
    lo, hi = wl.cell_off[2], wl.cell_off[3]
    assert np.all(sid[lo:hi] == -1) and np.all(perm[lo:hi] == np.arange(lo, hi))


def test_bad_values_flag_and_pass_through():
    wl = cloud_cells([50, 50, 50, 50], seed=4)
    wl.w[wl.cell_off[1] + 3] = -1.0
    wl.py[wl.cell_off[2] + 7] = np.nan
    c = __import__("tests.gpu_common", fromlist=["ctx"]).ctx()
    c.device_status(clear=True)
    got, got_off, tot = gpu_run(wl, CLOUD)
    assert c.device_status(clear=True) & vpm.VPM_FLAG_BAD_VALUE
    assert tot == int(got_off[-1])
    # cells 1 and 2 are copied unchanged, in input order
    for cc in (1, 2):
        lo, hi = wl.cell_off[cc], wl.cell_off[cc + 1]
        o = got_off[cc]
        assert got_off[cc + 1] - o == hi - lo
        for f in ("x", "w"):
            np.testing.assert_array_equal(got[f][o:o + hi - lo], getattr(wl, f)[lo:hi].astype(np.float64))
    # the healthy cells match the oracle
    sub = wl.cells([0, 3])
    ref = oracle.run_workload(sub, **oracle_params(CLOUD))
    for k, cc in enumerate((0, 3)):
        assert got_off[cc + 1] - got_off[cc] == ref.out_off[k + 1] - ref.out_off[k]


@pytest.mark.parametrize("seed", [0, 1])
def test_zero_tolerance_lattice(seed):
    """T = 0: subsets are the duplicate classes; exercises deep trees of tiny subsets and ties."""
    r = np.random.Generator(np.random.Philox(seed))
    cells = []
    for k in (40, 300, 900, 2500):
        base = r.integers(0, 3, size=(k, 6)).astype(np.float64)
        base[:, :3] *= 1000.0
        base[:, 3:] -= 1.0
        w = r.integers(1, 4, size=(k, 1)).astype(np.float64)
        cells.append(np.concatenate([base, w], axis=1))
    params = dict(tol_x=0.0, tol_p=0.0, n_min_cell=0, min_subset=1, cell_len=(65536.0,) * 3, mass=1.0)
    wl = W.from_cells(cells, params=params, dtype=np.float32)
    full_check(wl, params, vpm.VPM_MERGE_CENTROID)


def test_huge_tolerance_single_subset():
    wl = cloud_cells([100, 3000, 5000, 1], seed=5)
    params = dict(CLOUD, tol_x=100.0, tol_p=100.0)
    ref = full_check(wl, params)
    assert list(ref.n_subsets) == [1, 1, 1, 1]


def test_identical_particles():
    k = 777
    cell = np.tile(np.array([[0.25, 0.5, 0.75, 1.0, 0.0, -2.0, 1.5]]), (k, 1))
    wl = W.from_cells([cell, cell[:5]], params=dict(CLOUD, tol_x=0.0, tol_p=0.0), dtype=np.float32)
    full_check(wl, dict(CLOUD, tol_x=0.0, tol_p=0.0))


def test_cells_either_side_of_2_16():
    """65,536 particles is the largest cell decided through the FP64 filter; one more takes the exact
    wide path of the global-memory bin.  Both match the oracle, and nothing is flagged."""
    wl = cloud_cells([65536, 65537, 10], seed=6)
    c = __import__("tests.gpu_common", fromlist=["ctx"]).ctx()
    c.device_status(clear=True)
    check_partition_equal(wl, CLOUD)
    assert c.device_status(clear=True) == 0


def test_repeatable_bit_identical():
    wl = cloud_cells([800, 3000, 12000, 50], seed=7)
    a, ao, _ = gpu_run(wl, CLOUD)
    b, bo, _ = gpu_run(wl, CLOUD)
    np.testing.assert_array_equal(ao, bo)
    for f in FIELDS:
        np.testing.assert_array_equal(a[f], b[f])


def _autotune_for(wl, params, merge):
    """Set the context to the tuning vpm_autotune picks for this population, as the benchmark does
    before it times an event; returns the tuning that was set before."""
    import torch
    from tests.gpu_common import ctx
    c = ctx(max(wl.n, 1), max(wl.n_cells, 1))
    saved = c.get_tuning()
    arrs, off = vpm.upload(wl, dtype=torch.float32)
    out = [torch.empty_like(a) for a in arrs]
    oo = torch.empty(off.numel(), dtype=torch.int64, device="cuda")
    ot = torch.empty(1, dtype=torch.int64, device="cuda")
    best = c.autotune(arrs, off, wl.n, vpm.make_params(merge_mode=merge, **params), out, oo, ot)
    assert vpm.vpm_check_tuning(best) == vpm.VPM_OK
    return c, saved


def _sampled_check(wl, params, sample, merge=vpm.VPM_MERGE_PAIR, autotuned=False):
    """Run the whole population on the GPU and compare the sampled cells with the oracle run on
    those cells alone.  autotuned: in the launch configuration the benchmark times (the tuning
    vpm_autotune picks for the population), else the context's default."""
    if autotuned:
        c, saved = _autotune_for(wl, params, merge)
        try:
            perm, sid, nsub = gpu_partition(wl, params, merge=merge)
            got, got_off, tot = gpu_run(wl, params, merge=merge)
        finally:
            c.set_tuning(saved)
    else:
        perm, sid, nsub = gpu_partition(wl, params, merge=merge)
        got, got_off, tot = gpu_run(wl, params, merge=merge)
    sub = wl.cells(sample)
    ref = oracle.run_workload(sub, merge_mode=merge, **oracle_params(params))
    for k, c in enumerate(sample):
        lo, hi = int(wl.cell_off[c]), int(wl.cell_off[c + 1])
        slo = int(sub.cell_off[k])
        assert nsub[c] == ref.n_subsets[k]
        np.testing.assert_array_equal(perm[lo:hi] - lo, ref.perm[slo:slo + hi - lo] - slo)
        np.testing.assert_array_equal(sid[lo:hi], ref.subset_id[slo:slo + hi - lo])
        assert got_off[c + 1] - got_off[c] == ref.out_off[k + 1] - ref.out_off[k]
    # merged values of the sampled cells
    sel = np.concatenate([np.arange(got_off[c], got_off[c + 1]) for c in sample])
    g = {f: got[f][sel] for f in FIELDS}
    check_merged_values(sub, params, merge, g, ref.out_off, ref)
    return got, got_off, tot


def test_two_stream_full_size_sampled():
    """256 x 256 cells, Poisson(512) per cell (33.5M particles), FP32, sampled cells vs the oracle."""
    wl = W.two_stream_grid(seed=0).astype(np.float32)
    r = np.random.Generator(np.random.Philox(11))
    sample = np.sort(r.choice(wl.n_cells, 300, replace=False))
    _sampled_check(wl, wl.params, sample)


def test_two_stream_full_size_sampled_autotuned():
    """The same population and sample in the launch configuration the benchmark times."""
    wl = W.two_stream_grid(seed=0).astype(np.float32)
    r = np.random.Generator(np.random.Philox(13))
    sample = np.sort(r.choice(wl.n_cells, 300, replace=False))
    _sampled_check(wl, wl.params, sample, autotuned=True)


def test_two_stream_paper_tolerances_sampled():
    """Same population with the paper's two-stream tolerances (T_X 0.8, T_P 0.15, N_min 200): merges."""
    wl = W.two_stream_grid(nx=64, ny=64, seed=1).astype(np.float32)
    params = dict(W.TWO_STREAM_PAPER_PARAMS)
    sample = np.arange(0, wl.n_cells, 7)
    _sampled_check(wl, params, sample)


def test_shower_full_size_sampled():
    """64^3 cells, lognormal occupancy up to 32,768, gamma^-2 momenta: every size bin, sampled."""
    wl = W.shower_grid(seed=0)
    cnt = np.diff(wl.cell_off)
    r = np.random.Generator(np.random.Philox(12))
    big = np.nonzero(cnt > 4096)[0]
    mid = np.nonzero((cnt > 1024) & (cnt <= 4096))[0]
    small = np.nonzero((cnt > 10) & (cnt <= 1024))[0]
    tiny = np.nonzero(cnt <= 10)[0]
    sample = np.sort(np.concatenate([r.choice(big, 6, replace=False), [int(np.argmax(cnt))],
                                     r.choice(mid, 40, replace=False), r.choice(small, 200, replace=False),
                                     r.choice(tiny, 20, replace=False)]))
    sample = np.unique(sample)
    _sampled_check(wl, wl.params, sample, autotuned=True)


def test_shower_with_merging_sampled():
    """Shower-shaped cells with loose momentum tolerance so that subsets merge (lognormal weights,
    gamma up to 1e4): exercises the fixed-point merge sums over a wide dynamic range."""
    wl = W.shower_grid(nc=16, seed=3)
    params = dict(wl.params, tol_p=100.0, tol_x=0.5)
    sample = np.arange(0, wl.n_cells, 5)
    for merge in MERGES:
        _sampled_check(wl, params, sample, merge)


# ---------------------------------------------------------------------------- FP64 path

def _fp64_check(wl, params, merge=vpm.VPM_MERGE_PAIR):
    ref = oracle.run_workload(wl, decide=oracle.PAPER, merge_mode=merge, **oracle_params(params))
    perm, sid, nsub = gpu_partition(wl, params, decide=vpm.VPM_DECIDE_FP64)
    bad = []
    for c in range(wl.n_cells):
        lo, hi = wl.cell_off[c], wl.cell_off[c + 1]
        if not (np.array_equal(perm[lo:hi], ref.perm[lo:hi]) and np.array_equal(sid[lo:hi], ref.subset_id[lo:hi])):
            bad.append(c)
    for c in bad:
        assert ref.stats["min_margin"][c] < 1e-9, f"cell {c} differs without a near-tie"
    got, got_off, tot = gpu_run(wl, params, decide=vpm.VPM_DECIDE_FP64, merge=merge)
    good = [c for c in range(wl.n_cells) if c not in bad]
    sub = wl.cells(good)
    rsub = oracle.run_workload(sub, decide=oracle.PAPER, merge_mode=merge, **oracle_params(params))
    sel = np.concatenate([np.arange(got_off[c], got_off[c + 1]) for c in good]) if good else np.zeros(0, int)
    check_merged_values(sub, params, merge, {f: got[f][sel] for f in FIELDS}, rsub.out_off, rsub, rel=1e-12)
    return len(bad)


@pytest.mark.parametrize("merge", MERGES)
def test_fp64_path_cloud(merge):
    wl = cloud_cells([300, 257, 64, 1000, 5, 4, 3, 2, 1, 0, 700, 5000], seed=8, dtype=np.float64)
    params = dict(CLOUD, min_subset=4 if merge == vpm.VPM_MERGE_PAIR else 2)
    assert _fp64_check(wl, params, merge) <= 1


def test_fp64_path_two_stream():
    wl = W.two_stream_grid(nx=32, ny=32, seed=2)
    assert _fp64_check(wl, wl.params) <= 2


def test_fp64_path_two_stream_full_size_sampled():
    """The plain FP64 form on the whole 256 x 256 Poisson(512) two-stream population (33.5M particles,
    FP64, the population the benchmark times it on), 300 sampled cells against the PAPER oracle run
    on those cells alone: subset membership identical except in cells with a certified near-tie
    (oracle margin below 1e-9), merged particles to 1e-12."""
    wl = W.two_stream_grid(seed=0)
    params = dict(wl.params)
    r = np.random.Generator(np.random.Philox(13))
    sample = np.sort(r.choice(wl.n_cells, 300, replace=False))
    perm, sid, nsub = gpu_partition(wl, params, decide=vpm.VPM_DECIDE_FP64)
    got, got_off, _ = gpu_run(wl, params, decide=vpm.VPM_DECIDE_FP64)
    sub = wl.cells(sample)
    ref = oracle.run_workload(sub, decide=oracle.PAPER, **oracle_params(params))
    good, near = [], 0
    for k, c in enumerate(sample):
        lo, hi = int(wl.cell_off[c]), int(wl.cell_off[c + 1])
        slo = int(sub.cell_off[k])
        same = (nsub[c] == ref.n_subsets[k] and
                np.array_equal(perm[lo:hi] - lo, ref.perm[slo:slo + hi - lo] - slo) and
                np.array_equal(sid[lo:hi], ref.subset_id[slo:slo + hi - lo]))
        if not same:
            assert ref.stats["min_margin"][k] < 1e-9, f"cell {c} differs without a near-tie"
            near += 1
            continue
        assert got_off[c + 1] - got_off[c] == ref.out_off[k + 1] - ref.out_off[k]
        good.append(k)
    assert near <= 3
    cells = sample[good]
    rsub = oracle.run_workload(sub.cells(good), decide=oracle.PAPER, **oracle_params(params))
    sel = np.concatenate([np.arange(got_off[c], got_off[c + 1]) for c in cells])
    check_merged_values(sub.cells(good), params, vpm.VPM_MERGE_PAIR, {f: got[f][sel] for f in FIELDS},
                        rsub.out_off, rsub, rel=1e-12)


GOLDEN = ["px_bisection_6.txt", "corners_tie_4.txt", "px_ladder_8.txt", "pair_direction_2.txt",
          "pair_two_clusters_4.txt", "axis_rule_normalised_4.txt", "axis_rule_raw_4.txt"]


@pytest.mark.parametrize("decide", [vpm.VPM_DECIDE_FIXED, vpm.VPM_DECIDE_FP64])
@pytest.mark.parametrize("fname", GOLDEN)
def test_golden_cells_on_gpu(fname, decide):
    """The hand-worked cells (one holds an exact CV tie, which the FP64 filter cannot settle and
    hands to the exact integer rule; two derive pair momenta by hand) give the expected subsets and
    particles on the GPU, on both decision paths."""
    from tests.helpers import load_golden, subsets_of
    arr, prm, merge, subsets, merged = load_golden(fname)
    params = dict(prm, cell_len=(1.0, 1.0, 1.0))
    fp64 = decide == vpm.VPM_DECIDE_FP64
    wl = W.from_cells([arr], params=params, dtype=np.float64 if fp64 else np.float32)
    mm = vpm.VPM_MERGE_CENTROID if merge == "centroid" else vpm.VPM_MERGE_PAIR
    perm, sid, nsub = gpu_partition(wl, params, decide=decide, merge=mm)
    got = subsets_of(perm, sid, wl.cell_off, 0)
    assert [list(map(int, s)) for s in got] == subsets
    out, out_off, tot = gpu_run(wl, params, decide=decide, merge=mm)
    g = np.stack([out[f] for f in ("w", "x", "y", "z", "px", "py", "pz")], axis=1)
    tol = 1e-12 if fp64 else 1e-6
    np.testing.assert_allclose(g, merged, rtol=tol, atol=tol)


def test_exact_ties_on_gpu():
    """Cells whose root holds an exact tie between a position CV and a momentum CV (built from the
    fixed-point codes, so that the tie is exact): the FP64 filter cannot settle them, and the GPU's
    exact 128/256-bit rule must give the oracle's partition (ties to the lowest axis)."""
    from tests.test_oracle_exact_tiny import exact_tie
    r = np.random.Generator(np.random.Philox(99))
    cells = [exact_tie(r) for _ in range(300)]
    params = dict(CLOUD, tol_x=0.01, tol_p=0.01, min_subset=2)
    wl = W.from_cells(cells, params=params, dtype=np.float32)
    full_check(wl, params)
    full_check(wl, params, vpm.VPM_MERGE_CENTROID)


def _gpu_merge(wl, params, perm, sid, nsub, decide=vpm.VPM_DECIDE_FIXED, merge=vpm.VPM_MERGE_PAIR):
    from tests.gpu_common import ctx
    c = ctx(max(wl.n, 1), max(wl.n_cells, 1))
    dt = torch.float32 if decide == vpm.VPM_DECIDE_FIXED else torch.float64
    arrs, off = vpm.upload(wl, dtype=dt)
    n = wl.n
    out = [torch.empty_like(a) for a in arrs]
    out_off = torch.empty(wl.n_cells + 1, dtype=torch.int64, device="cuda")
    tot = torch.empty(1, dtype=torch.int64, device="cuda")
    p = vpm.make_params(merge_mode=merge, decide=decide, **params)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()
    c.merge(arrs, off, n, p, t(perm), t(sid), t(nsub), out, out_off, tot)
    torch.cuda.synchronize()
    k = int(tot.item())
    return {f: out[i][:k].cpu().numpy().astype(np.float64) for i, f in enumerate(FIELDS)}, out_off.cpu().numpy(), k


@pytest.mark.parametrize("decide", [vpm.VPM_DECIDE_FIXED, vpm.VPM_DECIDE_FP64])
@pytest.mark.parametrize("merge", MERGES)
def test_merge_of_partition_equals_run(decide, merge):
    dt = np.float32 if decide == vpm.VPM_DECIDE_FIXED else np.float64
    wl = cloud_cells([300, 57, 1000, 5, 0, 3000, 9000, 2], seed=9, dtype=dt)
    params = dict(CLOUD, min_subset=4 if merge == vpm.VPM_MERGE_PAIR else 2)
    perm, sid, nsub = gpu_partition(wl, params, decide=decide, merge=merge)
    got, got_off, tot = _gpu_merge(wl, params, perm, sid, nsub, decide, merge)
    ref, ref_off, rtot = gpu_run(wl, params, decide=decide, merge=merge)
    assert tot == rtot
    np.testing.assert_array_equal(got_off, ref_off)
    for f in FIELDS:
        np.testing.assert_array_equal(got[f], ref[f])


@pytest.mark.parametrize("merge", MERGES)
def test_merge_of_oracle_partition(merge):
    wl = cloud_cells([400, 64, 7, 2500], seed=10)
    params = dict(CLOUD, min_subset=4 if merge == vpm.VPM_MERGE_PAIR else 2)
    ref = oracle.run_workload(wl, merge_mode=merge, **oracle_params(params))
    got, got_off, tot = _gpu_merge(wl, params, ref.perm, ref.subset_id, ref.n_subsets, merge=merge)
    assert tot == ref.out_total
    check_merged_values(wl, params, merge, got, got_off, ref)


def test_merge_rejects_inconsistent_partition():
    from tests.gpu_common import ctx
    wl = cloud_cells([50, 50], seed=11)
    perm, sid, nsub = gpu_partition(wl, CLOUD)
    perm = perm.copy()
    perm[3] = 70                                  # a member from the other cell
    ctx().device_status(clear=True)
    got, got_off, tot = _gpu_merge(wl, CLOUD, perm, sid, nsub)
    assert ctx().device_status(clear=True) & vpm.VPM_FLAG_BAD_PARTITION
    assert got_off[1] - got_off[0] == 50          # copied unchanged
    np.testing.assert_array_equal(got["x"][:50], wl.x[:50].astype(np.float64))


@pytest.mark.parametrize("decide", [vpm.VPM_DECIDE_FIXED, vpm.VPM_DECIDE_FP64])
def test_merge_rejects_duplicated_member(decide):
    """A perm that lists one member twice (and leaves another out) is not a partition of the cell:
    the cell is copied unchanged and flagged, in both decision modes."""
    from tests.gpu_common import ctx
    dt = np.float32 if decide == vpm.VPM_DECIDE_FIXED else np.float64
    wl = cloud_cells([60, 40], seed=12, dtype=dt)
    perm, sid, nsub = gpu_partition(wl, CLOUD, decide=decide)
    perm = perm.copy()
    perm[5] = perm[17]                            # member perm[17] twice, old perm[5] missing
    assert perm[5] >= 0 and perm[5] < 60
    ctx().device_status(clear=True)
    got, got_off, tot = _gpu_merge(wl, CLOUD, perm, sid, nsub, decide=decide)
    assert ctx().device_status(clear=True) & vpm.VPM_FLAG_BAD_PARTITION
    assert got_off[1] - got_off[0] == 60          # copied unchanged
    for f in FIELDS:
        np.testing.assert_array_equal(got[f][:60], getattr(wl, f)[:60].astype(np.float64))
    # the other cell is merged as usual
    ref = oracle.run_workload(wl.cells([1]), decide=oracle.FIXED if decide == vpm.VPM_DECIDE_FIXED else oracle.PAPER,
                              **oracle_params(CLOUD))
    assert tot - 60 == ref.out_total


@pytest.mark.parametrize("concurrent", [0, 1, 2])
def test_large_cells_across_workgroups(concurrent):
    """Cells above the LDS bins are split by several workgroups at once once no cell is left to claim
    (subsets of >= 8,192 particles go to a device task queue).  Heavy-tailed momenta and lognormal
    weights make the splits lopsided, so tasks spawn tasks along chains.  The result must be the
    oracle's, with the bins in sequence (idle workgroups wait for tasks), concurrent (they leave) and
    with only the two-wavefront bin beside the others (they wait again)."""
    from tests.gpu_common import ctx
    r = np.random.Generator(np.random.Philox(41))
    cells = []
    for k in (60000, 33000, 17000, 9000, 4400, 2100, 300):
        p = np.exp(1.5 * r.standard_normal((k, 3))) * np.array([1.0, 0.3, 0.2])
        cells.append(np.concatenate([r.random((k, 3)), p, np.exp(r.standard_normal((k, 1)))], axis=1))
    params = dict(CLOUD, tol_x=0.2, tol_p=0.5)
    wl = W.from_cells(cells, params=params, dtype=np.float32)
    c = ctx(wl.n, wl.n_cells)
    default = c.get_tuning()
    c.set_tuning(vpm.make_tuning(concurrent_bins=concurrent))
    try:
        ref = full_check(wl, params)
        full_check(wl, params, vpm.VPM_MERGE_CENTROID)
    finally:
        c.set_tuning(default)
    assert ref.stats["max_depth"].max() > 12 and ref.out_total < wl.n


@pytest.mark.parametrize("merge", MERGES)
def test_normalised_axis_rule(merge):
    """Step 4 on each CV over its tolerance (VPM_AXIS_NORMALISED), with tolerances far apart so that
    the rule changes the partitions: the fixed-point path against the FIXED oracle (bit-exact), the
    FP64 form against the PAPER oracle (near-ties certified), and the result differs from the raw
    rule's."""
    wl = cloud_cells([300, 57, 1000, 5, 0, 3000, 9000, 2, 600], seed=15)
    params = dict(CLOUD, tol_x=0.6, tol_p=0.02, axis_rule=1, min_subset=4 if merge == vpm.VPM_MERGE_PAIR else 2)
    ref = full_check(wl, params, merge)
    raw = oracle.run_workload(wl, merge_mode=merge, **oracle_params(dict(params, axis_rule=0)))
    assert not np.array_equal(ref.subset_id, raw.subset_id)
    wl64 = cloud_cells([300, 57, 1000, 5, 0, 3000, 2, 600], seed=16, dtype=np.float64)
    assert _fp64_check(wl64, params, merge) <= 1


def test_normalised_axis_rule_zero_tolerance_and_ties():
    """A zero position tolerance makes every position CV > 0 infinite under the normalised rule (the
    lowest such axis is cut); the exact-tie cells go through the GPU's exact 320-bit comparison."""
    from tests.test_oracle_exact_tiny import exact_tie
    wl = cloud_cells([200, 64, 33], seed=17)
    full_check(wl, dict(CLOUD, tol_x=0.0, tol_p=0.05, axis_rule=1, min_subset=2))
    full_check(wl, dict(CLOUD, tol_x=0.05, tol_p=0.0, axis_rule=1, min_subset=2))
    full_check(wl, dict(CLOUD, tol_x=0.0, tol_p=0.0, axis_rule=1, min_subset=2))
    r = np.random.Generator(np.random.Philox(98))
    cells = [exact_tie(r) for _ in range(200)]
    params = dict(CLOUD, tol_x=0.01, tol_p=0.01, min_subset=2, axis_rule=1)
    full_check(W.from_cells(cells, params=params, dtype=np.float32), params)

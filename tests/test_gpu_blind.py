"""GPU blind method (vpm_blind) against the oracle's: the random pair choices, hence every particle's
output group, bit-exact; output counts exact; copied particles bit-identical; merged centroids
within 1e-6 (weight relative, position against L, momentum against the particle's energy)."""
import math

import numpy as np
import pytest

import oracle
from paper_1504_00636_amd import vpm, workloads as W
from tests.gpu_common import FIELDS, ctx

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _cells(seed, sizes):
    r = np.random.Generator(np.random.Philox(seed))
    cells = []
    for k in sizes:
        cells.append(np.stack([r.random(k), r.random(k), r.random(k), 0.2 * np.sign(r.random(k) - 0.5)
                               + 0.01 * r.standard_normal(k), 0.01 * r.standard_normal(k),
                               0.01 * r.standard_normal(k), 0.5 + r.random(k)], axis=1))
    return W.from_cells(cells, dtype=np.float32)


def gpu_blind(wl, alpha, seed, n_min_cell=0, mass=1.0):
    c = ctx(max(wl.n, 1), max(wl.n_cells, 1))
    arrs, off = vpm.upload(wl)
    out = [torch.full_like(a, -5.0) for a in arrs]
    out_off = torch.empty(wl.n_cells + 1, dtype=torch.int64, device="cuda")
    tot = torch.empty(1, dtype=torch.int64, device="cuda")
    group = torch.full((max(wl.n, 1),), -9, dtype=torch.int32, device="cuda")
    p = vpm.make_params(tol_x=0.1, tol_p=0.1, n_min_cell=n_min_cell, mass=mass)
    c.blind(arrs, off, wl.n, p, alpha, seed, out, out_off, tot, group)
    torch.cuda.synchronize()
    k = int(tot.item())
    return ({f: out[i][:k].cpu().numpy().astype(np.float64) for i, f in enumerate(FIELDS)},
            out_off.cpu().numpy(), group.cpu().numpy()[:wl.n])


def check(wl, alpha, seed, n_min_cell=0, mass=1.0):
    got, got_off, group = gpu_blind(wl, alpha, seed, n_min_cell, mass)
    ref = oracle.blind(wl.arrays(), wl.cell_off, alpha, seed, n_min_cell=n_min_cell, mass=mass)
    np.testing.assert_array_equal(group, ref.group)
    np.testing.assert_array_equal(got_off, ref.out_off)
    sizes = np.zeros(ref.out_total, np.int64)
    for c in range(wl.n_cells):
        lo, hi = int(wl.cell_off[c]), int(wl.cell_off[c + 1])
        np.add.at(sizes, int(ref.out_off[c]) + ref.group[lo:hi], 1)
    single = sizes == 1
    for f in FIELDS:
        np.testing.assert_array_equal(got[f][single], ref.out[f][single], err_msg=f)
    m = ~single
    if m.any():
        ulp = lambda v: np.spacing(np.abs(v).astype(np.float32)).astype(np.float64)   # FP32 storage
        assert np.all(np.abs(got["w"][m] - ref.out["w"][m]) <= 1e-6 * ref.out["w"][m] + ulp(ref.out["w"][m]))
        for f in ("x", "y", "z"):
            assert np.all(np.abs(got[f][m] - ref.out[f][m]) <= 1e-6 + ulp(ref.out[f][m])), f
        eps = np.sqrt(mass ** 2 + sum(ref.out[f][m] ** 2 for f in ("px", "py", "pz")))
        for f in ("px", "py", "pz"):
            assert np.all(np.abs(got[f][m] - ref.out[f][m]) <= 1e-6 * eps + ulp(ref.out[f][m])), f
    return ref


@pytest.mark.parametrize("alpha,seed", [(0.965, 1), (0.88, 2), (0.5, 3), (0.05, 4)])
def test_blind_matches_oracle(alpha, seed):
    wl = _cells(20 + seed, [300, 40, 3, 0, 1, 2, 700, 2100, 64, 5000, 17, 129, 9000])
    ref = check(wl, alpha, seed)
    assert ref.out_total < wl.n


def test_blind_two_stream_grid_counts():
    """64 x 64 two-stream cells at the paper's two-stream fraction 0.965: every cell keeps exactly
    ceil(0.965 N) particles."""
    wl = W.two_stream_grid(nx=64, ny=64, seed=5).astype(np.float32)
    ref = check(wl, 0.965, 11)
    counts = np.diff(wl.cell_off)
    want = np.array([min(math.ceil(0.965 * n), n) for n in counts])
    np.testing.assert_array_equal(np.diff(ref.out_off), want)


def test_blind_untouched_and_photons():
    wl = _cells(30, [10, 30, 0, 2, 400])
    check(wl, 1.0, 3)                                   # nothing to merge
    check(wl, 0.5, 3, n_min_cell=30)                    # only the 400-particle cell merges
    check(wl, 0.7, 4, mass=0.0)


def test_blind_rejects_bad_alpha_and_dtype():
    wl = _cells(31, [10])
    c = ctx(wl.n, 1)
    arrs, off = vpm.upload(wl)
    out = [torch.empty_like(a) for a in arrs]
    oo = torch.empty(2, dtype=torch.int64, device="cuda")
    ot = torch.empty(1, dtype=torch.int64, device="cuda")
    p = vpm.make_params(tol_x=0.1, tol_p=0.1)
    for bad in (-0.1, float("nan"), float("inf")):
        with pytest.raises(vpm.VpmError):
            c.blind(arrs, off, wl.n, p, bad, 1, out, oo, ot)

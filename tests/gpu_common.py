"""Helpers for GPU parity tests: run the HIP library through its C ABI and compare with the oracle."""
from __future__ import annotations

import numpy as np

import oracle
from paper_1504_00636_amd import vpm

FIELDS = ("x", "y", "z", "px", "py", "pz", "w")

_CTX = None


def ctx(np_cap=1 << 22, nc_cap=1 << 18):
    global _CTX
    if _CTX is None:
        _CTX = vpm.Context(0)
    _CTX.reserve(np_cap, nc_cap)
    return _CTX


def gpu_partition(wl, params: dict, decide=vpm.VPM_DECIDE_FIXED, merge=vpm.VPM_MERGE_PAIR):
    import torch
    c = ctx(max(wl.n, 1), max(wl.n_cells, 1))
    dt = torch.float32 if decide == vpm.VPM_DECIDE_FIXED else torch.float64
    arrs, off = vpm.upload(wl, dtype=dt)
    n = wl.n
    perm = torch.full((max(n, 1),), -7, dtype=torch.int32, device="cuda")
    sid = torch.full((max(n, 1),), -7, dtype=torch.int32, device="cuda")
    nsub = torch.full((max(wl.n_cells, 1),), -7, dtype=torch.int32, device="cuda")
    p = vpm.make_params(merge_mode=merge, decide=decide, **params)
    c.partition(arrs, off, n, p, perm, sid, nsub)
    torch.cuda.synchronize()
    return perm.cpu().numpy()[:n], sid.cpu().numpy()[:n], nsub.cpu().numpy()[:wl.n_cells]


def gpu_run(wl, params: dict, decide=vpm.VPM_DECIDE_FIXED, merge=vpm.VPM_MERGE_PAIR):
    import torch
    c = ctx(max(wl.n, 1), max(wl.n_cells, 1))
    dt = torch.float32 if decide == vpm.VPM_DECIDE_FIXED else torch.float64
    arrs, off = vpm.upload(wl, dtype=dt)
    p = vpm.make_params(merge_mode=merge, decide=decide, **params)
    res = vpm.run_population(c, arrs, off, p)
    torch.cuda.synchronize()
    out = {f: res.out[i][:res.out_total].cpu().numpy().astype(np.float64) for i, f in enumerate(FIELDS)}
    return out, res.out_off.cpu().numpy(), res.out_total


def oracle_params(params: dict):
    keys = ("tol_x", "tol_p", "n_min_cell", "min_subset", "cell_len", "mass", "axis_rule")
    return {k: params[k] for k in keys if k in params}


def check_partition_equal(wl, params, decide_gpu=vpm.VPM_DECIDE_FIXED, decide_orc=oracle.FIXED, ref=None,
                          merge=vpm.VPM_MERGE_PAIR):
    perm, sid, nsub = gpu_partition(wl, params, decide_gpu, merge)
    if ref is None:
        ref = oracle.run_workload(wl, decide=decide_orc, **oracle_params(params))
    np.testing.assert_array_equal(nsub, ref.n_subsets)
    np.testing.assert_array_equal(perm, ref.perm)
    np.testing.assert_array_equal(sid, ref.subset_id)
    return ref


def check_merged_values(wl, params, merge, got, got_off, ref, rel=1e-6):
    """Element-wise comparison of the merged populations.

    Copied particles must be bit-identical.  Merged particles: weight to `rel`; position to
    rel * L; momentum: the pair mean to rel * eps and |delta|^2 to rel * eps^2 (eps = energy of the
    merged particle), and the pair direction when |delta| > 1e-3 eps (below that |delta| is
    ill-conditioned).  One FP32 rounding of the stored value is allowed on top when the output is FP32.
    """
    np.testing.assert_array_equal(got_off, ref.out_off)
    L = np.asarray(params["cell_len"], np.float64)
    ulp = (lambda v: np.spacing(np.abs(v).astype(np.float32)).astype(np.float64)) \
        if wl.x.dtype == np.float32 else (lambda v: np.zeros_like(v))
    r = ref.out
    g = got
    mass = params["mass"]
    merged = _merged_mask(wl, ref, params, merge)
    cp = ~merged
    for f in FIELDS:
        np.testing.assert_array_equal(g[f][cp], r[f][cp], err_msg=f"copied {f}")
    if not merged.any():
        return
    w_ok = np.abs(g["w"][merged] - r["w"][merged]) <= rel * np.abs(r["w"][merged]) + ulp(r["w"][merged])
    assert w_ok.all(), "weight"
    for a, f in enumerate(("x", "y", "z")):
        ok = np.abs(g[f][merged] - r[f][merged]) <= rel * L[a] + ulp(r[f][merged])
        assert ok.all(), f"position {f}: max err {np.max(np.abs(g[f][merged] - r[f][merged]))}"
    pr = np.stack([r[f] for f in ("px", "py", "pz")], 1)[merged]
    pg = np.stack([g[f] for f in ("px", "py", "pz")], 1)[merged]
    eps = np.sqrt(mass * mass + (pr * pr).sum(1))
    pul = np.abs(pr).astype(np.float32)
    pul = np.spacing(pul).astype(np.float64) if wl.x.dtype == np.float32 else 0 * pr
    if merge == vpm.VPM_MERGE_CENTROID:
        assert (np.abs(pg - pr) <= rel * eps[:, None] + pul).all(), "centroid momentum"
        return
    # pairs are consecutive merged slots (+delta first)
    idx = np.nonzero(merged)[0]
    assert idx.size % 2 == 0
    a, b = np.arange(0, idx.size, 2), np.arange(1, idx.size, 2)
    assert np.all(idx[b] == idx[a] + 1)
    mr, mg = (pr[a] + pr[b]) / 2, (pg[a] + pg[b]) / 2
    dr, dg = (pr[a] - pr[b]) / 2, (pg[a] - pg[b]) / 2
    e = eps[a]
    tol_m = rel * e[:, None] + pul[a] + pul[b]
    assert (np.abs(mg - mr) <= tol_m).all(), f"pair mean: max {np.max(np.abs(mg - mr) / e[:, None])}"
    nr, ng = (dr * dr).sum(1), (dg * dg).sum(1)
    tol_r = rel * e * e + 4 * np.sqrt(nr) * (pul[a] + pul[b]).max(1)
    assert (np.abs(ng - nr) <= tol_r).all(), f"|delta|^2: max {np.max(np.abs(ng - nr) / (e * e))}"
    big = np.sqrt(nr) > 1e-3 * e
    if big.any():
        ur = dr[big] / np.sqrt(nr[big])[:, None]
        ug = dg[big] / np.sqrt(ng[big])[:, None]
        assert (np.abs(ug - ur) <= 1e-4).all(), "pair direction"


def _merged_mask(wl, ref, params, merge):
    """Boolean mask over the oracle's output slots: True where the slot holds a merged particle."""
    n_out = int(ref.out_off[-1])
    mask = np.zeros(n_out, bool)
    npair = 1 if merge == vpm.VPM_MERGE_CENTROID else 2
    for c in range(wl.n_cells):
        lo, hi = int(wl.cell_off[c]), int(wl.cell_off[c + 1])
        o = int(ref.out_off[c])
        if ref.n_subsets[c] == 0:
            continue
        sid = ref.subset_id[lo:hi]
        sizes = np.bincount(sid, minlength=int(ref.n_subsets[c]))
        for s in sizes:
            if s >= params["min_subset"]:
                mask[o:o + npair] = True
                o += npair
            else:
                o += int(s)
    return mask


def conserved_totals(out, mass):
    w = out["w"]
    px, py, pz = out["px"], out["py"], out["pz"]
    e = np.sqrt(mass * mass + px * px + py * py + pz * pz)
    return np.array([w.sum(), (w * px).sum(), (w * py).sum(), (w * pz).sum(), (w * e).sum()])

"""Seeded synthetic particle populations for the merge hot path.

This module only draws random particles and lays them out cell-sorted with
int64 cell offsets.  It holds none of the merging arithmetic, so both the
GPU library's tests and the CPU oracle's tests may use it.

Shapes follow the paper's workloads (Sec. "Simulation"):

* two counter-drifting electron beams (Sec. "Two-stream instability"),
  here as Maxwellians drifting at +-0.2 m_e c with 0.01 m_e c thermal
  spread per component, uniform inside their cell;
* a magnetic-shower-like population (Sec. "Magnetic Shower"): Lorentz
  factors from dN/dgamma ~ gamma^-2 on [1, 1e4], directions in a narrow
  cone about +x, lognormal weights and lognormal cell occupancy.

The paper's own simulation states are not available; these stand in for
them.  All random numbers come from numpy's Philox bit generator.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, Optional

import numpy as np

FIELDS = ("x", "y", "z", "px", "py", "pz", "w")


@dataclass
class Workload:
    """A cell-sorted structure-of-arrays particle population.

    ``cell_off`` has ``n_cells + 1`` entries; cell ``c`` owns particles
    ``cell_off[c] .. cell_off[c+1]-1``.  ``params`` holds the merge
    parameters the configuration is quoted with (tolerances T_X, T_P,
    N_min, minimum subset size, cell lengths, particle mass).
    """

    name: str
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    px: np.ndarray
    py: np.ndarray
    pz: np.ndarray
    w: np.ndarray
    cell_off: np.ndarray
    cell_id: Optional[np.ndarray] = None
    params: Dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.cell_off[-1])

    @property
    def n_cells(self) -> int:
        return int(self.cell_off.shape[0] - 1)

    @property
    def dtype(self):
        return self.x.dtype

    def arrays(self):
        return [getattr(self, f) for f in FIELDS]

    def astype(self, dtype) -> "Workload":
        """Copy with every particle array converted (FP64 -> FP32 rounds to nearest)."""
        kw = {f: np.ascontiguousarray(getattr(self, f).astype(dtype)) for f in FIELDS}
        return Workload(self.name, cell_off=self.cell_off.copy(),
                        cell_id=None if self.cell_id is None else self.cell_id.copy(),
                        params=dict(self.params), **kw)

    def cells(self, idx) -> "Workload":
        """Sub-population made of the listed cells (kept in the given order)."""
        idx = np.asarray(idx, dtype=np.int64)
        counts = self.cell_off[idx + 1] - self.cell_off[idx]
        off = np.zeros(idx.shape[0] + 1, np.int64)
        np.cumsum(counts, out=off[1:])
        sel = np.concatenate([np.arange(self.cell_off[c], self.cell_off[c + 1]) for c in idx]) \
            if idx.size else np.zeros(0, np.int64)
        kw = {f: np.ascontiguousarray(getattr(self, f)[sel]) for f in FIELDS}
        cid = None if self.cell_id is None else np.ascontiguousarray(self.cell_id[sel])
        return Workload(self.name + "[sub]", cell_off=off, cell_id=cid, params=dict(self.params), **kw)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(seed))


def _offsets(counts: np.ndarray) -> np.ndarray:
    off = np.zeros(counts.shape[0] + 1, np.int64)
    np.cumsum(counts, out=off[1:])
    return off


def from_cells(cells, params=None, name="custom", dtype=np.float64) -> Workload:
    """Build a population from a list of per-cell (n, 7) arrays ordered x,y,z,px,py,pz,w."""
    counts = np.array([np.asarray(c).reshape(-1, 7).shape[0] for c in cells], np.int64)
    data = np.concatenate([np.asarray(c, dtype=np.float64).reshape(-1, 7) for c in cells]) \
        if len(cells) else np.zeros((0, 7))
    kw = {f: np.ascontiguousarray(data[:, i].astype(dtype)) for i, f in enumerate(FIELDS)}
    return Workload(name, cell_off=_offsets(counts), params=dict(params or {}), **kw)


# --------------------------------------------------------------------------------------
# Two counter-drifting Maxwellian beams (two-stream instability shape)
# --------------------------------------------------------------------------------------

TWO_STREAM_PARAMS = dict(tol_x=0.1, tol_p=0.05, n_min_cell=0, min_subset=4,
                         cell_len=(1.0, 1.0, 1.0), mass=1.0)
# The paper's own two-stream tolerances (Table 1): T_X 0.8, T_P 0.15, N_min 200.
TWO_STREAM_PAPER_PARAMS = dict(tol_x=0.8, tol_p=0.15, n_min_cell=200, min_subset=4,
                               cell_len=(1.0, 1.0, 1.0), mass=1.0)


def single_cell_two_beams(n: int = 2000, seed: int = 0) -> Workload:
    """One cell, ``n`` electrons: exactly n/2 per beam, drift +-0.2, spread 0.01, w = 1, FP64."""
    r = _rng(seed)
    half = n // 2
    sign = np.concatenate([np.ones(half), -np.ones(n - half)])
    r.shuffle(sign)
    x = r.random(n)
    y = r.random(n)
    z = r.random(n)
    px = 0.2 * sign + 0.01 * r.standard_normal(n)
    py = 0.01 * r.standard_normal(n)
    pz = 0.01 * r.standard_normal(n)
    w = np.ones(n)
    return Workload("single_cell_2000", x, y, z, px, py, pz, w,
                    cell_off=np.array([0, n], np.int64), cell_id=np.zeros(n, np.int32),
                    params=dict(TWO_STREAM_PARAMS))


def two_stream_grid(nx: int = 256, ny: int = 256, mean: float = 512.0, seed: int = 0,
                    params: Optional[Dict] = None) -> Workload:
    """2-D grid of unit cells, Poisson(mean) electrons per cell, two drifting beams.

    Cell id = i + nx*j.  Positions uniform in [i, i+1) x [j, j+1), z = 0.
    Beam chosen per particle with probability 1/2.  Weights uniform in
    [0.5, 1.5].  FP64 SoA, cell-sorted.
    """
    r = _rng(seed)
    n_cells = nx * ny
    counts = r.poisson(mean, n_cells).astype(np.int64)
    n = int(counts.sum())
    cid = np.repeat(np.arange(n_cells, dtype=np.int64), counts)
    ci = cid % nx
    cj = cid // nx
    x = ci + r.random(n)
    y = cj + r.random(n)
    z = np.zeros(n)
    sign = np.where(r.random(n) < 0.5, 1.0, -1.0)
    px = 0.2 * sign + 0.01 * r.standard_normal(n)
    py = 0.01 * r.standard_normal(n)
    pz = 0.01 * r.standard_normal(n)
    w = 0.5 + r.random(n)
    return Workload(f"two_stream_{nx}x{ny}_mean{int(mean)}", x, y, z, px, py, pz, w,
                    cell_off=_offsets(counts), cell_id=cid.astype(np.int32),
                    params=dict(params or TWO_STREAM_PARAMS))


# --------------------------------------------------------------------------------------
# Magnetic-shower-like population
# --------------------------------------------------------------------------------------

SHOWER_PARAMS = dict(tol_x=1.0, tol_p=0.02, n_min_cell=10, min_subset=4,
                     cell_len=(1.0, 1.0, 1.0), mass=1.0)


def _shower_momenta(r: np.random.Generator, n: int, gamma_max: float = 1e4, cone: float = 0.1):
    u = r.random(n)
    gamma = 1.0 / (1.0 - u * (1.0 - 1.0 / gamma_max))     # inverse CDF of dN/dgamma ~ gamma^-2
    pmag = np.sqrt(np.maximum(gamma * gamma - 1.0, 0.0))
    cos_t = np.cos(cone) + (1.0 - np.cos(cone)) * r.random(n)
    sin_t = np.sqrt(np.maximum(1.0 - cos_t * cos_t, 0.0))
    phi = 2.0 * np.pi * r.random(n)
    return pmag * cos_t, pmag * sin_t * np.cos(phi), pmag * sin_t * np.sin(phi)


def shower_grid(nc: int = 64, seed: int = 0, median: float = 64.0, sigma: float = 1.5,
                cap: int = 32768, dtype=np.float32, params: Optional[Dict] = None) -> Workload:
    """nc^3 unit cells; occupancy min(cap, round(median*exp(sigma*Z))); gamma^-2 momenta in a
    0.1-rad cone about +x; lognormal(0, 1) weights; FP32 storage by default."""
    r = _rng(seed)
    n_cells = nc ** 3
    counts = np.minimum(cap, np.rint(median * np.exp(sigma * r.standard_normal(n_cells)))).astype(np.int64)
    n = int(counts.sum())
    cid = np.repeat(np.arange(n_cells, dtype=np.int64), counts)
    ci = cid % nc
    cj = (cid // nc) % nc
    ck = cid // (nc * nc)
    x = ci + r.random(n)
    y = cj + r.random(n)
    z = ck + r.random(n)
    px, py, pz = _shower_momenta(r, n)
    w = r.lognormal(0.0, 1.0, n)
    wl = Workload(f"shower_{nc}^3", x, y, z, px, py, pz, w, cell_off=_offsets(counts),
                  cell_id=cid.astype(np.int32), params=dict(params or SHOWER_PARAMS))
    return wl.astype(dtype) if dtype != np.float64 else wl


# --------------------------------------------------------------------------------------
# Repeated-merge cascade (pair-splitting growth between merge events)
# --------------------------------------------------------------------------------------

CASCADE_PARAMS = dict(tol_x=1.0, tol_p=0.02, n_min_cell=1024, min_subset=4,
                      cell_len=(1.0, 1.0, 1.0), mass=1.0)


def cascade_initial(nx: int = 512, ny: int = 512, per_cell: int = 256, seed: int = 0,
                    dtype=np.float32) -> Workload:
    """2-D grid, ``per_cell`` particles per cell, shower-like momenta, weights U[0.5, 1.5]."""
    r = _rng(seed)
    n_cells = nx * ny
    counts = np.full(n_cells, per_cell, np.int64)
    n = int(counts.sum())
    cid = np.repeat(np.arange(n_cells, dtype=np.int64), counts)
    x = (cid % nx) + r.random(n)
    y = (cid // nx) + r.random(n)
    z = np.zeros(n)
    px, py, pz = _shower_momenta(r, n)
    w = 0.5 + r.random(n)
    wl = Workload(f"cascade_{nx}x{ny}", x, y, z, px, py, pz, w, cell_off=_offsets(counts),
                  cell_id=cid.astype(np.int32), params=dict(CASCADE_PARAMS))
    return wl.astype(dtype) if dtype != np.float64 else wl


def cascade_split(wl: Workload, step: int, seed: int = 0) -> Workload:
    """One growth step: every particle (w, x, p) becomes (w/2, x, p) followed by
    (w/2, x', p') with x' uniform in its cell and p' drawn like the shower.
    Cell membership is preserved, so the result stays cell-sorted."""
    r = _rng(seed * 1000003 + step + 1)
    n = wl.n
    counts = np.diff(wl.cell_off)
    n_cells = counts.shape[0]
    nx = int(round(np.sqrt(n_cells)))
    cid = np.repeat(np.arange(n_cells, dtype=np.int64), counts)
    nxp = (cid % nx) + r.random(n)
    nyp = (cid // nx) + r.random(n)
    npx, npy, npz = _shower_momenta(r, n)
    dt = wl.x.dtype
    out = {}
    for f, new in zip(FIELDS, (nxp, nyp, np.zeros(n), npx, npy, npz, None)):
        old = getattr(wl, f)
        if f == "w":
            new = old * 0.5
            old = old * 0.5
        pair = np.empty(2 * n, dtype=dt)
        pair[0::2] = old
        pair[1::2] = np.asarray(new, dtype=dt)
        out[f] = pair
    return Workload(wl.name, cell_off=wl.cell_off * 2, cell_id=None, params=dict(wl.params), **out)


def cascade_split_device(arrs, cell_off, n: int, step: int, out_arrs, out_off, nx: int = 512, seed: int = 0):
    """The cascade growth step of `cascade_split` on device tensors (torch's Philox generator, so the
    random numbers differ from the host version; the recipe is the same).  Reads n particles from
    `arrs` (7 tensors) with offsets `cell_off`, writes 2n particles to `out_arrs` and the doubled
    offsets to `out_off`.  Returns 2n."""
    import torch
    dev = arrs[0].device
    g = torch.Generator(device=dev)
    g.manual_seed(seed * 1000003 + step + 1)
    n_cells = cell_off.numel() - 1
    counts = cell_off[1:] - cell_off[:-1]
    cid = torch.repeat_interleave(torch.arange(n_cells, device=dev), counts, output_size=n)
    u = lambda: torch.rand(n, generator=g, device=dev, dtype=torch.float64)
    fresh_x = (cid % nx).double() + u()
    fresh_y = torch.div(cid, nx, rounding_mode="floor").double() + u()
    del cid
    gamma = 1.0 / (1.0 - u() * (1.0 - 1e-4))
    pmag = torch.sqrt(torch.clamp(gamma * gamma - 1.0, min=0.0))
    del gamma
    cos_t = float(np.cos(0.1)) + (1.0 - float(np.cos(0.1))) * u()
    sin_t = torch.sqrt(torch.clamp(1.0 - cos_t * cos_t, min=0.0))
    phi = 2.0 * np.pi * u()
    fresh = [fresh_x, fresh_y, None, pmag * cos_t, pmag * sin_t * torch.cos(phi), pmag * sin_t * torch.sin(phi)]
    for k in range(7):
        dst = out_arrs[k]
        old = arrs[k][:n]
        if k == 6:
            half = old * 0.5
            dst[0:2 * n:2] = half
            dst[1:2 * n:2] = half
        else:
            dst[0:2 * n:2] = old
            dst[1:2 * n:2] = 0.0 if fresh[k] is None else fresh[k].to(dst.dtype)
    out_off.copy_(cell_off * 2)
    return 2 * n


# --------------------------------------------------------------------------------------
# Counter-propagating blocks (Sec. "Counter-propagating Plasma Blocks")
# --------------------------------------------------------------------------------------

BLOCKS_PARAMS = dict(tol_x=0.4, tol_p=0.01, n_min_cell=15, min_subset=4,
                     cell_len=(1.0, 1.0, 1.0), mass=1.0)


def counter_blocks(per_cell: int = 12, nx: int = 100, ny: int = 20, block_cells: int = 25, p0: float = 150.0,
                   seed: int = 0, dtype=np.float32) -> Workload:
    """Two blocks of non-interacting electrons over `block_cells` x `ny` unit cells each of an
    nx x ny grid, `per_cell` particles in every cell of a block (uniform inside the cell, z uniform
    in [0, 1)), with momenta (+p0, 0, 0) and (-p0, 0, 0) in m_e c and unit weights: 12,000
    particles by default, 12 per cell, below the merge threshold N_min = 15 until the blocks
    overlap.  The first block starts a quarter of the row in and moves to +x, the second ends a
    quarter from the far end and moves to -x.  Box and grid are choices made here (the paper gives
    neither)."""
    r = _rng(seed)
    a0 = nx // 4 - block_cells // 2
    b0 = nx - nx // 4 - block_cells // 2
    ix, iy = np.meshgrid(np.arange(block_cells), np.arange(ny), indexing="ij")
    ix = np.repeat(ix.ravel(), per_cell)
    iy = np.repeat(iy.ravel(), per_cell)
    h = ix.size
    x = np.concatenate([a0 + ix + r.random(h), b0 + ix + r.random(h)])
    y = np.concatenate([iy + r.random(h), iy + r.random(h)])
    px = np.concatenate([np.full(h, p0), np.full(h, -p0)])
    n = 2 * h
    wl = _sorted_grid(x, y, r.random(n), px, np.zeros(n), np.zeros(n), np.ones(n), nx, ny, dtype)
    wl.params = dict(BLOCKS_PARAMS)
    wl.name = "counter_blocks"
    return wl


def _sorted_grid(x, y, z, px, py, pz, w, nx, ny, dtype) -> Workload:
    """Particles of an nx x ny grid of unit cells (x wraps around), stably sorted by cell
    c = ix + nx * iy."""
    x = np.mod(np.asarray(x, np.float64), nx)
    y = np.asarray(y, np.float64)
    cid = np.minimum(np.floor(x).astype(np.int64), nx - 1) + nx * np.minimum(np.floor(y).astype(np.int64), ny - 1)
    order = np.argsort(cid, kind="stable")
    cols = [np.asarray(a, np.float64)[order].astype(dtype) for a in (x, y, z, px, py, pz, w)]
    counts = np.bincount(cid, minlength=nx * ny).astype(np.int64)
    return Workload("grid", *cols, cell_off=_offsets(counts), cell_id=None, params={})


def free_stream(wl: Workload, nx: int, ny: int, dt: float, dtype=np.float32) -> Workload:
    """Move every particle by v dt along x (v = p / gamma, c = 1, mass 1), then sort by cell again."""
    px, py, pz = (np.asarray(getattr(wl, f), np.float64) for f in ("px", "py", "pz"))
    gamma = np.sqrt(1.0 + px * px + py * py + pz * pz)
    out = _sorted_grid(np.asarray(wl.x, np.float64) + dt * px / gamma, wl.y, wl.z, px, py, pz, wl.w,
                       nx, ny, dtype)
    out.params = dict(wl.params)
    out.name = wl.name
    return out

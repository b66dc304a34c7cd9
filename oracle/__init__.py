"""CPU oracle for the Voronoi particle-merging hot path -- TEST INFRASTRUCTURE ONLY.

Thin ctypes wrapper over ``vpm_oracle.c`` (a plain C implementation of the
paper's algorithm, Sec. "Algorithm", Steps 1-7).  Only the tests, the smoke
check and the benchmark's CPU-baseline leg import this package; the GPU
library never does.  The shared object is compiled with gcc on first use if
``build()`` has not produced it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vpm_oracle.c")
_LIB = os.path.join(_HERE, "libvpm_oracle.so")

PAIR, CENTROID = 0, 1
FIXED, PAPER = 0, 1
FLAG_BAD_VALUE, FLAG_OUT_OF_CELL, FLAG_TOO_LARGE = 1, 2, 4


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain IEEE arithmetic: no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp",
                               "-ffp-contract=off", "-fno-fast-math", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(C.Structure):
    _fields_ = [("tol_x", C.c_double), ("tol_p", C.c_double),
                ("n_min_cell", C.c_int32), ("min_subset", C.c_int32),
                ("cell_len", C.c_double * 3), ("mass", C.c_double),
                ("merge_mode", C.c_int32), ("decide", C.c_int32), ("axis_rule", C.c_int32)]


class _Stats(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("n_leaves", C.c_int32), ("n_merged", C.c_int32),
                ("max_depth", C.c_int32), ("particle_levels", C.c_int64),
                ("min_margin", C.c_double), ("flags", C.c_uint32), ("n_out", C.c_int32)]


STATS_DTYPE = np.dtype([("n_nodes", np.int32), ("n_leaves", np.int32), ("n_merged", np.int32),
                        ("max_depth", np.int32), ("particle_levels", np.int64),
                        ("min_margin", np.float64), ("flags", np.uint32), ("n_out", np.int32)])
assert STATS_DTYPE.itemsize == C.sizeof(_Stats)

_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = _bind(C.CDLL(_LIB))
    return _lib


def _bind(lib):
    dp = C.POINTER(C.c_double)
    i64p = C.POINTER(C.c_int64)
    i32p = C.POINTER(C.c_int32)
    lib.orc_run.restype = C.c_int
    lib.orc_run.argtypes = ([C.POINTER(_Params), C.c_int64, i64p] + [dp] * 7 +
                            [i32p, i32p, i32p] + [dp] * 7 + [i64p, C.c_void_p, C.c_int])
    return lib


def runner(lib):
    """`run` bound to another build of the oracle's source (the pin tests compile copies with planted
    mistakes and check that the pins catch them)."""
    lib = _bind(lib)
    return lambda *a, **k: run(*a, lib=lib, **k)


@dataclass
class OracleResult:
    perm: np.ndarray        # int32[n] global input index per slot
    subset_id: np.ndarray   # int32[n] final-subset ordinal per slot, -1 untouched
    n_subsets: np.ndarray   # int32[n_cells]
    out: dict               # field -> float64[n_out]
    out_off: np.ndarray     # int64[n_cells+1]
    stats: np.ndarray       # structured, STATS_DTYPE[n_cells]

    @property
    def out_total(self) -> int:
        return int(self.out_off[-1])


def make_params(tol_x, tol_p, n_min_cell=0, min_subset=4, cell_len=(1.0, 1.0, 1.0), mass=1.0,
                merge_mode=PAIR, decide=FIXED, axis_rule=0) -> _Params:
    p = _Params()
    p.tol_x, p.tol_p = float(tol_x), float(tol_p)
    p.n_min_cell, p.min_subset = int(n_min_cell), int(min_subset)
    for a in range(3):
        p.cell_len[a] = float(cell_len[a])
    p.mass = float(mass)
    p.merge_mode, p.decide = int(merge_mode), int(decide)
    p.axis_rule = int(axis_rule)
    return p


def run(arrays, cell_off, tol_x, tol_p, n_min_cell=0, min_subset=4, cell_len=(1.0, 1.0, 1.0),
        mass=1.0, merge_mode=PAIR, decide=FIXED, n_threads: int = 0, lib=None, axis_rule=0) -> OracleResult:
    """Run the oracle.  ``arrays`` = (x, y, z, px, py, pz, w), any float dtype (FIXED mode rounds
    the values to FP32 first, as the GPU's fixed-point path does).  axis_rule 1: Step 4 on each CV
    over its tolerance."""
    lib = lib or _load()
    p = make_params(tol_x, tol_p, n_min_cell, min_subset, cell_len, mass, merge_mode, decide, axis_rule)
    cell_off = np.ascontiguousarray(cell_off, dtype=np.int64)
    n_cells = cell_off.shape[0] - 1
    n = int(cell_off[-1])
    ins = [np.ascontiguousarray(a, dtype=np.float64) for a in arrays]
    for a in ins:
        if a.shape[0] < n:
            raise ValueError("particle arrays shorter than cell_off[-1]")
    perm = np.empty(n, np.int32)
    sid = np.empty(n, np.int32)
    nsub = np.empty(n_cells, np.int32)
    outs = [np.empty(max(n, 1), np.float64) for _ in range(7)]
    out_off = np.empty(n_cells + 1, np.int64)
    stats = np.zeros(n_cells, STATS_DTYPE)
    dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
    rc = lib.orc_run(C.byref(p), n_cells, cell_off.ctypes.data_as(C.POINTER(C.c_int64)),
                     *[dp(a) for a in ins],
                     perm.ctypes.data_as(C.POINTER(C.c_int32)), sid.ctypes.data_as(C.POINTER(C.c_int32)),
                     nsub.ctypes.data_as(C.POINTER(C.c_int32)),
                     *[dp(a) for a in outs], out_off.ctypes.data_as(C.POINTER(C.c_int64)),
                     C.c_void_p(stats.ctypes.data), int(n_threads))
    if rc != 0:
        raise ValueError(f"oracle rejected its arguments (code {rc})")
    nout = int(out_off[-1])
    names = ("x", "y", "z", "px", "py", "pz", "w")
    return OracleResult(perm, sid, nsub, {k: outs[i][:nout] for i, k in enumerate(names)},
                        out_off, stats)


def run_workload(wl, decide=FIXED, merge_mode=PAIR, n_threads: int = 0, **override) -> OracleResult:
    """Convenience: run on a ``workloads.Workload`` with its own parameters (overridable)."""
    prm = dict(wl.params)
    prm.update(override)
    return run(wl.arrays(), wl.cell_off, decide=decide, merge_mode=merge_mode,
               n_threads=n_threads, **prm)


def _bind_blind(lib):
    dp = C.POINTER(C.c_double)
    lib.orc_blind.restype = C.c_int
    lib.orc_blind.argtypes = ([C.c_double, C.c_uint64, C.c_int32, C.c_double, C.c_int, C.c_int64,
                               C.POINTER(C.c_int64)] + [dp] * 7 + [C.POINTER(C.c_int32)] + [dp] * 7 +
                              [C.POINTER(C.c_int64), C.c_int])
    lib.orc_philox4x64_10.restype = None
    lib.orc_philox4x64_10.argtypes = [C.POINTER(C.c_uint64), C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]
    return lib


@dataclass
class BlindResult:
    group: np.ndarray       # int32[n]: cell-local output ordinal of each input particle
    out: dict               # field -> float64[n_out]
    out_off: np.ndarray     # int64[n_cells+1]

    @property
    def out_total(self) -> int:
        return int(self.out_off[-1])


def blind(arrays, cell_off, alpha, seed, n_min_cell=0, mass=1.0, f32=True, n_threads: int = 0,
          lib=None) -> BlindResult:
    """The paper's blind method: random pairs merged per cell until at most ceil(alpha N) remain
    (Philox4x64-10 counter (t, cell, 0, 0), key (seed, 0)).  f32: round the inputs to FP32 first,
    as the GPU's FP32 path works on them."""
    lib = _bind_blind(lib or _load())
    cell_off = np.ascontiguousarray(cell_off, dtype=np.int64)
    n_cells = cell_off.shape[0] - 1
    n = int(cell_off[-1])
    ins = [np.ascontiguousarray(a, dtype=np.float64) for a in arrays]
    group = np.empty(max(n, 1), np.int32)
    outs = [np.empty(max(n, 1), np.float64) for _ in range(7)]
    out_off = np.empty(n_cells + 1, np.int64)
    dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
    rc = lib.orc_blind(float(alpha), int(seed) & (2 ** 64 - 1), int(n_min_cell), float(mass), int(bool(f32)),
                       n_cells, cell_off.ctypes.data_as(C.POINTER(C.c_int64)), *[dp(a) for a in ins],
                       group.ctypes.data_as(C.POINTER(C.c_int32)), *[dp(a) for a in outs],
                       out_off.ctypes.data_as(C.POINTER(C.c_int64)), int(n_threads))
    if rc != 0:
        raise ValueError(f"oracle rejected its arguments (code {rc})")
    nout = int(out_off[-1])
    names = ("x", "y", "z", "px", "py", "pz", "w")
    return BlindResult(group[:n], {k: outs[i][:nout] for i, k in enumerate(names)}, out_off)


def philox4x64_10(counter, key):
    """The oracle's Philox4x64-10 block for a 4-word counter and 2-word key (for its known-answer test)."""
    lib = _bind_blind(_load())
    c = (C.c_uint64 * 4)(*[int(v) for v in counter])
    k = (C.c_uint64 * 2)(*[int(v) for v in key])
    o = (C.c_uint64 * 4)()
    lib.orc_philox4x64_10(c, k, o)
    return [int(v) for v in o]

"""Python binding of libvpm.so (include/vpm.h): argument marshalling only.

Every entry point keeps its C name (vpm_create, vpm_reserve, vpm_run, vpm_partition, vpm_merge,
vpm_check_params, vpm_device_status, ...).  Tensors are passed as raw device pointers; the stream is
torch's current HIP stream unless one is given.  All computation happens in the HIP library; if the
library is missing this module raises instead of computing anything itself.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvpm.so")

VPM_OK, VPM_ERR_INVALID_ARG, VPM_ERR_UNSUPPORTED, VPM_ERR_CAPACITY, VPM_ERR_HIP, VPM_ERR_NO_DEVICE = \
    0, -1, -2, -3, -4, -5
VPM_F32, VPM_F64 = 0, 1
VPM_DECIDE_FIXED, VPM_DECIDE_FP64 = 0, 1
VPM_MERGE_PAIR, VPM_MERGE_CENTROID = 0, 1
VPM_AXIS_RAW, VPM_AXIS_NORMALISED = 0, 1
VPM_FLAG_BAD_VALUE, VPM_FLAG_OUT_OF_CELL, VPM_FLAG_CELL_TOO_LARGE, VPM_FLAG_BAD_OFFSETS = 1, 2, 4, 8
VPM_FLAG_BAD_PARTITION = 16
VPM_FLAG_BAD_SPECIES = 32
VPM_MAX_SPECIES = 8

EXPORTS = ("vpm_create", "vpm_destroy", "vpm_reserve", "vpm_check_params", "vpm_run", "vpm_run_species",
           "vpm_partition",
           "vpm_merge", "vpm_device_status", "vpm_profile_enable", "vpm_profile_read",
           "vpm_check_tuning", "vpm_get_tuning", "vpm_set_tuning", "vpm_autotune",
           "vpm_status_string", "vpm_last_error", "vpm_version", "vpm_run_noalloc", "vpm_blind")
VPM_NOALLOC_MAX_PARTICLES, VPM_NOALLOC_MAX_CELLS = 524288, 32768


class VpmParams(C.Structure):
    _fields_ = [("tol_x", C.c_double), ("tol_p", C.c_double),
                ("n_min_cell", C.c_int32), ("min_subset", C.c_int32),
                ("cell_len", C.c_double * 3), ("mass", C.c_double),
                ("merge_mode", C.c_int32), ("decide", C.c_int32),
                ("dtype", C.c_int32), ("axis_rule", C.c_int32)]


class VpmTuning(C.Structure):
    _fields_ = [("ppl", C.c_int32), ("bin_a_max", C.c_int32), ("bin_b_max", C.c_int32), ("bin_c_max", C.c_int32),
                ("concurrent_bins", C.c_int32), ("bin_s_max", C.c_int32), ("exact_decisions", C.c_int32),
                ("bin_d_max", C.c_int32)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


def make_tuning(ppl=16, bin_a_max=576, bin_b_max=2288, bin_c_max=4592, concurrent_bins=0, bin_s_max=128,
                exact_decisions=0, bin_d_max=None) -> VpmTuning:
    """bin_d_max None: 1144 kept between bin_a_max and bin_b_max."""
    t = VpmTuning()
    t.ppl, t.bin_a_max, t.bin_b_max, t.bin_c_max = int(ppl), int(bin_a_max), int(bin_b_max), int(bin_c_max)
    t.concurrent_bins, t.bin_s_max = int(concurrent_bins), int(bin_s_max)
    t.exact_decisions = int(exact_decisions)
    t.bin_d_max = max(int(bin_a_max), min(1144, int(bin_b_max))) if bin_d_max is None else int(bin_d_max)
    return t


class VpmSoa(C.Structure):
    _fields_ = [(f, C.c_void_p) for f in ("x", "y", "z", "px", "py", "pz", "w")]


class VpmError(RuntimeError):
    def __init__(self, status: int, what: str, detail: str = ""):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} ({status}){' - ' + detail if detail else ''}")


_lib = None


def lib():
    """Load libvpm.so (built by paper_1504_00636_amd.build.build()); raise if it is not there."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1504_00636_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, i64, i32 = C.c_void_p, C.c_int64, C.c_int32
    P = C.POINTER
    L.vpm_create.argtypes = [P(vp), C.c_int]
    L.vpm_destroy.argtypes = [vp]
    L.vpm_reserve.argtypes = [vp, i64, i64]
    L.vpm_check_params.argtypes = [P(VpmParams)]
    L.vpm_run.argtypes = [vp, P(VpmSoa), vp, i64, i64, P(VpmParams), P(VpmSoa), vp, vp, vp]
    L.vpm_run_species.argtypes = [vp, P(VpmSoa), vp, i64, i64, P(VpmParams), vp, P(C.c_double), C.c_int32,
                                  P(VpmSoa), vp, vp, vp]
    L.vpm_run_noalloc.argtypes = [P(VpmSoa), vp, i64, i64, P(VpmParams), P(VpmSoa), vp, vp, vp, vp]
    L.vpm_partition.argtypes = [vp, P(VpmSoa), vp, i64, i64, P(VpmParams), vp, vp, vp, vp]
    L.vpm_blind.argtypes = [vp, P(VpmSoa), vp, i64, i64, P(VpmParams), C.c_double, C.c_uint64, P(VpmSoa), vp, vp,
                            vp, vp]
    L.vpm_merge.argtypes = [vp, P(VpmSoa), vp, i64, i64, P(VpmParams), vp, vp, vp, P(VpmSoa), vp, vp, vp]
    L.vpm_device_status.argtypes = [vp, P(C.c_uint32), C.c_int]
    L.vpm_check_tuning.argtypes = [P(VpmTuning)]
    L.vpm_get_tuning.argtypes = [vp, P(VpmTuning)]
    L.vpm_set_tuning.argtypes = [vp, P(VpmTuning)]
    L.vpm_autotune.argtypes = [vp, P(VpmSoa), vp, i64, i64, P(VpmParams), P(VpmSoa), vp, vp, vp, P(VpmTuning)]
    L.vpm_profile_enable.argtypes = [vp, C.c_int]
    L.vpm_profile_read.argtypes = [vp, C.c_int, vp, P(C.c_int64), P(C.c_double), P(C.c_int), C.c_int]
    L.vpm_status_string.argtypes = [C.c_int]
    L.vpm_status_string.restype = C.c_char_p
    L.vpm_last_error.argtypes = [vp]
    L.vpm_last_error.restype = C.c_char_p
    L.vpm_version.restype = C.c_char_p
    for f in ("vpm_create", "vpm_destroy", "vpm_reserve", "vpm_check_params", "vpm_run", "vpm_run_species",
              "vpm_run_noalloc", "vpm_blind",
              "vpm_partition", "vpm_merge", "vpm_device_status", "vpm_profile_enable", "vpm_profile_read", "vpm_check_tuning",
              "vpm_get_tuning", "vpm_set_tuning", "vpm_autotune"):
        getattr(L, f).restype = C.c_int
    _lib = L
    return L


def status_string(st: int) -> str:
    return lib().vpm_status_string(int(st)).decode()


def vpm_version() -> str:
    return lib().vpm_version().decode()


def make_params(tol_x, tol_p, n_min_cell=0, min_subset=4, cell_len=(1.0, 1.0, 1.0), mass=1.0,
                merge_mode=VPM_MERGE_PAIR, decide=VPM_DECIDE_FIXED, dtype=None, axis_rule=VPM_AXIS_RAW) -> VpmParams:
    p = VpmParams()
    p.tol_x, p.tol_p = float(tol_x), float(tol_p)
    p.n_min_cell, p.min_subset = int(n_min_cell), int(min_subset)
    for a in range(3):
        p.cell_len[a] = float(cell_len[a])
    p.mass = float(mass)
    p.merge_mode, p.decide = int(merge_mode), int(decide)
    if dtype is None:
        dtype = VPM_F32 if decide == VPM_DECIDE_FIXED else VPM_F64
    p.dtype = int(dtype)
    p.axis_rule = int(axis_rule)
    return p


def vpm_check_params(p: VpmParams) -> int:
    """Host-only parameter validation; returns the status code."""
    return int(lib().vpm_check_params(C.byref(p)))


def vpm_check_tuning(t: VpmTuning) -> int:
    """Host-only tuning validation; returns the status code."""
    return int(lib().vpm_check_tuning(C.byref(t)))


# ------------------------------------------------------------------------------------------
# tensor marshalling
# ------------------------------------------------------------------------------------------

def _soa(arrs: Sequence, dtype, n_min: int, what: str) -> VpmSoa:
    import torch
    if len(arrs) != 7:
        raise ValueError(f"{what}: need 7 arrays (x, y, z, px, py, pz, w)")
    s = VpmSoa()
    for f, t in zip(("x", "y", "z", "px", "py", "pz", "w"), arrs):
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError(f"{what}.{f}: expected a device tensor")
        if t.dtype != dtype or not t.is_contiguous() or t.numel() < n_min:
            raise ValueError(f"{what}.{f}: expected contiguous {dtype} with >= {n_min} elements")
        setattr(s, f, t.data_ptr())
    return s


def _dev(t, dtype, n: int, what: str) -> int:
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dtype or not t.is_contiguous() \
            or t.numel() < n:
        raise ValueError(f"{what}: expected a contiguous device {dtype} tensor with >= {n} elements")
    return t.data_ptr()


def _stream(stream) -> int:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(getattr(stream, "cuda_stream", stream) or 0)


def _torch_dtype(p: VpmParams):
    """Element type of the input arrays."""
    import torch
    return torch.float32 if p.dtype == VPM_F32 else torch.float64


def _out_dtype(p: VpmParams):
    """Element type of the output arrays: FP32 for fixed-point decisions (FP64 input is rounded to
    FP32 as it is loaded), else the input's."""
    import torch
    return torch.float32 if p.decide == VPM_DECIDE_FIXED else _torch_dtype(p)


class Context:
    """Owns a vpm_ctx (one device, one stream at a time) and its workspace."""

    def __init__(self, device: int = 0):
        h = C.c_void_p()
        st = lib().vpm_create(C.byref(h), int(device))
        if st != VPM_OK:
            raise VpmError(st, "vpm_create")
        self.h = h
        self.device = device

    def close(self):
        if getattr(self, "h", None):
            lib().vpm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int, what: str):
        if st != VPM_OK:
            detail = lib().vpm_last_error(self.h).decode() if st == VPM_ERR_HIP else ""
            raise VpmError(st, what, detail)

    def reserve(self, max_particles: int, max_cells: int):
        self._check(lib().vpm_reserve(self.h, int(max_particles), int(max_cells)), "vpm_reserve")

    def run(self, inp, cell_off, n_particles: int, p: VpmParams, out, out_off, out_total, stream=None):
        import torch
        n_cells = cell_off.numel() - 1
        dt = _torch_dtype(p)
        si = _soa(inp, dt, n_particles, "in")
        so = _soa(out, _out_dtype(p), n_particles, "out")
        st = lib().vpm_run(self.h, C.byref(si), _dev(cell_off, torch.int64, n_cells + 1, "cell_off"), n_cells,
                           int(n_particles), C.byref(p), C.byref(so),
                           _dev(out_off, torch.int64, n_cells + 1, "out_off"),
                           _dev(out_total, torch.int64, 1, "out_total"), _stream(stream))
        self._check(st, "vpm_run")

    def run_species(self, inp, cell_off, n_particles: int, p: VpmParams, cell_species, species_mass, out, out_off,
                    out_total, stream=None):
        """vpm_run_species: cell_species a device uint8 tensor (one entry per cell), species_mass a host
        sequence of 1 ... VPM_MAX_SPECIES masses."""
        import torch
        n_cells = cell_off.numel() - 1
        dt = _torch_dtype(p)
        si = _soa(inp, dt, n_particles, "in")
        so = _soa(out, _out_dtype(p), n_particles, "out")
        masses = [float(m) for m in species_mass]
        tab = (C.c_double * max(1, len(masses)))(*masses)
        st = lib().vpm_run_species(self.h, C.byref(si), _dev(cell_off, torch.int64, n_cells + 1, "cell_off"),
                                   n_cells, int(n_particles), C.byref(p),
                                   _dev(cell_species, torch.uint8, n_cells, "cell_species") if n_cells else None,
                                   tab, len(masses), C.byref(so),
                                   _dev(out_off, torch.int64, n_cells + 1, "out_off"),
                                   _dev(out_total, torch.int64, 1, "out_total"), _stream(stream))
        self._check(st, "vpm_run_species")

    def partition(self, inp, cell_off, n_particles: int, p: VpmParams, perm, subset_id, n_subsets, stream=None):
        import torch
        n_cells = cell_off.numel() - 1
        si = _soa(inp, _torch_dtype(p), n_particles, "in")
        st = lib().vpm_partition(self.h, C.byref(si), _dev(cell_off, torch.int64, n_cells + 1, "cell_off"),
                                 n_cells, int(n_particles), C.byref(p),
                                 _dev(perm, torch.int32, n_particles, "perm"),
                                 _dev(subset_id, torch.int32, n_particles, "subset_id"),
                                 _dev(n_subsets, torch.int32, n_cells, "n_subsets"), _stream(stream))
        self._check(st, "vpm_partition")

    def merge(self, inp, cell_off, n_particles: int, p: VpmParams, perm, subset_id, n_subsets, out, out_off,
              out_total, stream=None):
        import torch
        n_cells = cell_off.numel() - 1
        dt = _torch_dtype(p)
        si = _soa(inp, dt, n_particles, "in")
        so = _soa(out, _out_dtype(p), n_particles, "out")
        st = lib().vpm_merge(self.h, C.byref(si), _dev(cell_off, torch.int64, n_cells + 1, "cell_off"), n_cells,
                             int(n_particles), C.byref(p), _dev(perm, torch.int32, n_particles, "perm"),
                             _dev(subset_id, torch.int32, n_particles, "subset_id"),
                             _dev(n_subsets, torch.int32, n_cells, "n_subsets"), C.byref(so),
                             _dev(out_off, torch.int64, n_cells + 1, "out_off"),
                             _dev(out_total, torch.int64, 1, "out_total"), _stream(stream))
        self._check(st, "vpm_merge")

    def blind(self, inp, cell_off, n_particles: int, p: VpmParams, alpha: float, seed: int, out, out_off,
              out_total, group=None, stream=None):
        """vpm_blind: random pair merges down to ceil(alpha N) per cell; group: optional device int32
        tensor receiving each input particle's cell-local output ordinal."""
        import torch
        n_cells = cell_off.numel() - 1
        dt = _torch_dtype(p)
        si = _soa(inp, dt, n_particles, "in")
        so = _soa(out, _out_dtype(p), n_particles, "out")
        g = None if group is None else _dev(group, torch.int32, n_particles, "group")
        st = lib().vpm_blind(self.h, C.byref(si), _dev(cell_off, torch.int64, n_cells + 1, "cell_off"), n_cells,
                             int(n_particles), C.byref(p), float(alpha), int(seed) & (2 ** 64 - 1), C.byref(so),
                             _dev(out_off, torch.int64, n_cells + 1, "out_off"),
                             _dev(out_total, torch.int64, 1, "out_total"), g, _stream(stream))
        self._check(st, "vpm_blind")

    def get_tuning(self) -> VpmTuning:
        t = VpmTuning()
        self._check(lib().vpm_get_tuning(self.h, C.byref(t)), "vpm_get_tuning")
        return t

    def set_tuning(self, t: VpmTuning):
        self._check(lib().vpm_set_tuning(self.h, C.byref(t)), "vpm_set_tuning")

    def autotune(self, inp, cell_off, n_particles: int, p: VpmParams, out, out_off, out_total,
                 stream=None) -> VpmTuning:
        import torch
        n_cells = cell_off.numel() - 1
        dt = _torch_dtype(p)
        si = _soa(inp, dt, n_particles, "in")
        so = _soa(out, _out_dtype(p), n_particles, "out")
        best = VpmTuning()
        st = lib().vpm_autotune(self.h, C.byref(si), _dev(cell_off, torch.int64, n_cells + 1, "cell_off"), n_cells,
                                int(n_particles), C.byref(p), C.byref(so),
                                _dev(out_off, torch.int64, n_cells + 1, "out_off"),
                                _dev(out_total, torch.int64, 1, "out_total"), _stream(stream), C.byref(best))
        self._check(st, "vpm_autotune")
        return best

    def device_status(self, clear: bool = False) -> int:
        f = C.c_uint32(0)
        self._check(lib().vpm_device_status(self.h, C.byref(f), int(clear)), "vpm_device_status")
        return int(f.value)

    def profile_enable(self, on: bool = True):
        self._check(lib().vpm_profile_enable(self.h, int(on)), "vpm_profile_enable")

    def profile_read(self, reset: bool = True):
        """{kernel name: (launches, total ms)} since the last reset."""
        nmax = 64
        names = (C.c_char * 48 * nmax)()
        launches = (C.c_int64 * nmax)()
        ms = (C.c_double * nmax)()
        n = C.c_int(0)
        self._check(lib().vpm_profile_read(self.h, nmax, C.cast(names, C.c_void_p), launches, ms, C.byref(n),
                                           int(reset)), "vpm_profile_read")
        return {bytes(names[i]).split(b"\0")[0].decode(): (int(launches[i]), float(ms[i]))
                for i in range(min(n.value, nmax))}


# C-named module-level wrappers -----------------------------------------------------------

def vpm_create(device: int = 0) -> Context:
    return Context(device)


def vpm_reserve(ctx: Context, max_particles: int, max_cells: int):
    ctx.reserve(max_particles, max_cells)


def vpm_run(ctx: Context, *a, **k):
    ctx.run(*a, **k)


def vpm_run_species(ctx: Context, *a, **k):
    ctx.run_species(*a, **k)


def vpm_blind(ctx: Context, *a, **k):
    ctx.blind(*a, **k)


def vpm_partition(ctx: Context, *a, **k):
    ctx.partition(*a, **k)


def vpm_merge(ctx: Context, *a, **k):
    ctx.merge(*a, **k)


def vpm_run_noalloc(inp, cell_off, n_particles: int, p: VpmParams, out, out_off, out_total, flags_out=None,
                    stream=None):
    """vpm_run without a context (no device allocation; limits VPM_NOALLOC_MAX_*), on the current
    device.  flags_out: optional device uint32 tensor that receives the call's device flags."""
    import torch
    n_cells = cell_off.numel() - 1
    dt = _torch_dtype(p)
    si = _soa(inp, dt, n_particles, "in")
    so = _soa(out, _out_dtype(p), n_particles, "out")
    fo = None if flags_out is None else _dev(flags_out, torch.int32, 1, "flags_out")
    st = lib().vpm_run_noalloc(C.byref(si), _dev(cell_off, torch.int64, n_cells + 1, "cell_off"), n_cells,
                               int(n_particles), C.byref(p), C.byref(so),
                               _dev(out_off, torch.int64, n_cells + 1, "out_off"),
                               _dev(out_total, torch.int64, 1, "out_total"), fo, _stream(stream))
    if st != VPM_OK:
        raise VpmError(st, "vpm_run_noalloc")


def vpm_device_status(ctx: Context, clear: bool = False) -> int:
    return ctx.device_status(clear)


def vpm_get_tuning(ctx: Context) -> VpmTuning:
    return ctx.get_tuning()


def vpm_set_tuning(ctx: Context, t: VpmTuning):
    ctx.set_tuning(t)


def vpm_autotune(ctx: Context, *a, **k) -> VpmTuning:
    return ctx.autotune(*a, **k)


def vpm_destroy(ctx: Context):
    ctx.close()


# ------------------------------------------------------------------------------------------
# convenience: a whole population in, merged population out
# ------------------------------------------------------------------------------------------

@dataclass
class RunResult:
    out: list             # 7 device tensors (first out_total entries valid)
    out_off: object       # int64 device tensor [n_cells+1]
    out_total: int


def upload(wl, dtype=None, device="cuda"):
    """Copy a workloads.Workload to the device: (list of 7 tensors, cell_off tensor)."""
    import numpy as np
    import torch
    dt = dtype or (torch.float32 if wl.x.dtype == np.float32 else torch.float64)
    arrs = [torch.from_numpy(np.ascontiguousarray(a)).to(device=device, dtype=dt) for a in wl.arrays()]
    off = torch.from_numpy(np.ascontiguousarray(wl.cell_off)).to(device=device)
    return arrs, off


def run_population(ctx: Context, arrs, cell_off, p: VpmParams, stream=None) -> RunResult:
    import torch
    n = int(arrs[0].numel())
    n_cells = cell_off.numel() - 1
    out = [torch.empty_like(a, dtype=_out_dtype(p)) for a in arrs]
    out_off = torch.empty(n_cells + 1, dtype=torch.int64, device=arrs[0].device)
    out_total = torch.empty(1, dtype=torch.int64, device=arrs[0].device)
    ctx.run(arrs, cell_off, n, p, out, out_off, out_total, stream)
    tot = int(out_total.item())
    return RunResult(out, out_off, tot)

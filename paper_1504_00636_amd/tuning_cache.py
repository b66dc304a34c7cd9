"""A persistent cache of autotuned batching configurations (vpm_autotune results).

The autotuner times a few lane-group sizings and bin limits on the population at hand; its result
depends on the device, the ROCm runtime, the particle dtype, the kernels themselves and the shape of
the population (cell count, the spread of cell sizes, tolerances).  Entries are stored in one JSON
file keyed by all of these, so that a later run on the same kind of population and build reuses the
tuning instead of searching again.  The file is `$VPM_TUNING_CACHE`, else
`~/.cache/paper_1504_00636_amd/tuning.json`.
"""
from __future__ import annotations

import hashlib
import json
import os
import time

import numpy as np

from . import vpm

_HERE = os.path.dirname(os.path.abspath(__file__))
_SOURCES = [os.path.join(_HERE, "csrc", f) for f in sorted(os.listdir(os.path.join(_HERE, "csrc")))
            if f.endswith((".hip", ".h", ".hpp", ".cpp"))]


def default_path() -> str:
    return os.environ.get("VPM_TUNING_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "paper_1504_00636_amd", "tuning.json")


def sources_sha() -> str:
    """SHA-256 over the library's kernel and host sources (a changed kernel retunes)."""
    h = hashlib.sha256()
    for f in _SOURCES:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def population_signature(cell_off: np.ndarray, p: vpm.VpmParams) -> dict:
    """What the tuning depends on in a population: the cell count, the histogram of cell sizes over
    power-of-two classes, and the decision parameters."""
    counts = np.diff(np.asarray(cell_off, np.int64))
    cls = np.zeros(counts.shape, np.int64)
    nz = counts > 0
    cls[nz] = np.floor(np.log2(counts[nz])).astype(np.int64) + 1
    hist = np.bincount(cls, minlength=18)
    return {"n_cells": int(counts.size), "size_classes": hist.tolist(),
            "tol_x": float(p.tol_x), "tol_p": float(p.tol_p), "n_min_cell": int(p.n_min_cell),
            "min_subset": int(p.min_subset), "merge_mode": int(p.merge_mode), "axis_rule": int(p.axis_rule)}


def cache_key(device: str, rocm: str, dtype: int, sig: dict) -> str:
    blob = json.dumps({"device": device, "rocm": rocm, "dtype": int(dtype), "sources": sources_sha(),
                       "population": sig}, sort_keys=True)
    return hashlib.sha256(blob.encode()).hexdigest()


def _load(path: str) -> dict:
    try:
        with open(path) as fh:
            d = json.load(fh)
        return d if isinstance(d, dict) else {}
    except (OSError, ValueError):
        return {}


def lookup(path: str, key: str):
    e = _load(path).get(key)
    if not e:
        return None
    return vpm.make_tuning(**e["tuning"])


def store(path: str, key: str, tuning: vpm.VpmTuning, meta: dict) -> None:
    d = _load(path)
    d[key] = {"tuning": tuning.as_dict(), "meta": meta, "stored": time.strftime("%Y-%m-%dT%H:%M:%S")}
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = f"{path}.tmp{os.getpid()}"
    with open(tmp, "w") as fh:
        json.dump(d, fh, indent=1)
    os.replace(tmp, path)


def autotune_cached(ctx: vpm.Context, inp, cell_off, n_particles: int, p: vpm.VpmParams, out, out_off, out_total,
                    path: str | None = None):
    """The tuning for this population from the cache, else from vpm_autotune (then stored).  The
    context is left set to the returned tuning.  Returns (tuning, hit, key)."""
    import torch
    path = path or default_path()
    props = torch.cuda.get_device_properties(cell_off.device)
    device = getattr(props, "gcnArchName", props.name)
    sig = population_signature(cell_off.cpu().numpy(), p)
    key = cache_key(device, str(torch.version.hip), p.dtype, sig)
    t = lookup(path, key)
    if t is not None:
        ctx.set_tuning(t)
        return t, True, key
    t = ctx.autotune(inp, cell_off, n_particles, p, out, out_off, out_total)
    store(path, key, t, {"device": device, "rocm": str(torch.version.hip), "dtype": int(p.dtype),
                         "n_particles": int(n_particles), "population": sig})
    return t, False, key

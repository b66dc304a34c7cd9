"""Shared test helpers: golden-file loader and result checks (no merging arithmetic)."""
from __future__ import annotations

import os
from fractions import Fraction

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
FIELDS = ("x", "y", "z", "px", "py", "pz", "w")


def load_golden(name):
    """Parse a hand-worked golden cell: inputs, params, expected subsets and merged particles."""
    inputs, subsets, merged, params = [], [], [], {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            tag, *rest = line.split()
            if tag == "input":
                inputs.append([float(v) for v in rest])
            elif tag == "subset":
                subsets.append([int(v) for v in rest])
            elif tag == "merged":
                merged.append([float(v) for v in rest])
            elif tag == "params":
                for kv in rest:
                    k, v = kv.split("=")
                    params[k] = v
    arr = np.array(inputs, dtype=np.float64)
    prm = dict(tol_x=float(params["tol_x"]), tol_p=float(params["tol_p"]),
               min_subset=int(params["min_subset"]), n_min_cell=int(params["n_min_cell"]),
               mass=float(params["mass"]), axis_rule=int(params.get("axis_rule", 0)))
    return arr, prm, params.get("merge", "pair"), subsets, np.array(merged, dtype=np.float64)


def subsets_of(perm, subset_id, cell_off, c):
    """Final subsets of cell c as lists of global input indices, in slot order."""
    lo, hi = int(cell_off[c]), int(cell_off[c + 1])
    sid = subset_id[lo:hi]
    per = perm[lo:hi]
    out = []
    for s in range(int(sid.max()) + 1 if hi > lo and sid.max() >= 0 else 0):
        out.append(list(per[sid == s]))
    return out


def partition_sets(perm, subset_id, cell_off, c):
    return sorted(tuple(sorted(s)) for s in subsets_of(perm, subset_id, cell_off, c))


def energy(px, py, pz, mass):
    return np.sqrt(mass * mass + px * px + py * py + pz * pz)


def exact_sum(v):
    """Exact sum of float64 values (as a Fraction), then rounded."""
    return float(sum((Fraction(float(x)) for x in v), Fraction(0)))


def conserved_totals(arrs, mass):
    """(W, Px, Py, Pz, E) of a population, summed exactly from its float64 values."""
    x, y, z, px, py, pz, w = [np.asarray(a, dtype=np.float64) for a in arrs]
    e = energy(px, py, pz, mass)
    return np.array([exact_sum(w), exact_sum(w * px), exact_sum(w * py), exact_sum(w * pz),
                     exact_sum(w * e)])

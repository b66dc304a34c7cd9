"""Pins for the oracle's blind method (the paper's comparison method, Sec. "Simulation": random pairs
merged per cell until at most ceil(alpha N) particles remain; alpha = 0.965 and 0.88 in Tables 1, 2).

* the random numbers: Philox4x64-10 blocks equal numpy's independent implementation (numpy's
  generator advances its counter before each block, so counter c there gives block c + 1 here);
* the pair choices: a plain re-implementation of the slot process on numpy's Philox gives the same
  group of every particle;
* the output count is exactly ceil(alpha N) in merged cells and N elsewhere;
* each output is a singleton copied bit for bit or the numpy.average centroid of its group;
* weight and momentum are conserved, energy is never gained (Jensen's inequality).
"""
import math

import numpy as np
import pytest

import oracle
from paper_1504_00636_amd import workloads as W
from tests.helpers import FIELDS, conserved_totals


def _numpy_block(counter, key):
    c = int(sum(int(v) << (64 * i) for i, v in enumerate(counter))) - 1
    words = np.array([(c >> (64 * i)) & (2 ** 64 - 1) for i in range(4)], dtype=np.uint64)
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=words)
    return [int(v) for v in bg.random_raw(4)]


@pytest.mark.parametrize("counter,key", [([1, 0, 0, 0], [0, 0]), ([7, 3, 0, 0], [12345, 0]),
                                         ([0, 65535, 0, 0], [2 ** 63 + 5, 0]),
                                         ([2 ** 64 - 1, 2 ** 40, 9, 1], [2 ** 64 - 1, 2 ** 64 - 1])])
def test_philox_matches_numpy(counter, key):
    assert oracle.philox4x64_10(counter, key) == _numpy_block(counter, key)


def _python_groups(n, c, alpha, seed):
    """The slot process, written again from its definition on numpy's Philox."""
    T = math.ceil(alpha * n)
    slot, parent = list(range(n)), list(range(n))
    for t in range(n - T):
        M = n - t
        r = _numpy_block([t, c, 0, 0], [seed, 0])
        i, j = r[0] % M, r[1] % (M - 1)
        j += j >= i
        parent[slot[j]] = slot[i]
        slot[j] = slot[M - 1]

    def root(i):
        while parent[i] != i:
            i = parent[i]
        return i

    ordk = {slot[k]: k for k in range(T)}
    return [ordk[root(i)] for i in range(n)], T


def _cells(seed, sizes):
    r = np.random.Generator(np.random.Philox(seed))
    cells = []
    for k in sizes:
        cells.append(np.stack([r.random(k), r.random(k), r.random(k), 0.2 * np.sign(r.random(k) - 0.5)
                               + 0.01 * r.standard_normal(k), 0.01 * r.standard_normal(k),
                               0.01 * r.standard_normal(k), 0.5 + r.random(k)], axis=1))
    return W.from_cells(cells, dtype=np.float32)


@pytest.mark.parametrize("alpha,seed", [(0.965, 1), (0.88, 2), (0.5, 3), (0.2, 4)])
def test_pair_choices_follow_the_definition(alpha, seed):
    wl = _cells(10 + seed, [40, 3, 0, 1, 29, 64, 17, 100])
    r = oracle.blind(wl.arrays(), wl.cell_off, alpha, seed)
    for c in range(wl.n_cells):
        lo, hi = int(wl.cell_off[c]), int(wl.cell_off[c + 1])
        n = hi - lo
        want, T = _python_groups(n, c, alpha, seed)
        if n == 0:
            continue
        if T >= n:                              # untouched: every particle is its own output
            want = list(range(n))
        assert list(r.group[lo:hi]) == want, c
        assert r.out_off[c + 1] - r.out_off[c] == min(T, n)


@pytest.mark.parametrize("alpha", [0.965, 0.88, 0.6])
def test_counts_values_and_conservation(alpha):
    wl = W.two_stream_grid(nx=6, ny=5, mean=60, seed=4).astype(np.float32)
    r = oracle.blind(wl.arrays(), wl.cell_off, alpha, 77)
    q = {f: np.asarray(getattr(wl, f), np.float64) for f in FIELDS}
    for c in range(wl.n_cells):
        lo, hi = int(wl.cell_off[c]), int(wl.cell_off[c + 1])
        n = hi - lo
        T = min(math.ceil(alpha * n), n)
        o = int(r.out_off[c])
        assert r.out_off[c + 1] - o == T
        g = r.group[lo:hi]
        assert sorted(set(g.tolist())) == list(range(T))
        for k in range(T):
            mem = np.nonzero(g == k)[0] + lo
            if len(mem) == 1:
                for f in FIELDS:
                    assert r.out[f][o + k] == q[f][mem[0]]
            else:
                w = q["w"][mem]
                assert r.out["w"][o + k] == pytest.approx(w.sum(), rel=1e-15)
                for f in FIELDS[:6]:
                    assert r.out[f][o + k] == pytest.approx(np.average(q[f][mem], weights=w), rel=1e-13, abs=1e-15)
    tin = conserved_totals(wl.arrays(), 1.0)
    tout = conserved_totals([r.out[f] for f in FIELDS], 1.0)
    scale = np.array([tin[0], *[np.sum(wl.w * np.abs(getattr(wl, f))) for f in ("px", "py", "pz")], tin[4]])
    err = np.abs(tout - tin) / scale
    assert err[:4].max() < 1e-14
    assert tout[4] < tin[4]                     # pair merges lose energy


def test_untouched_cells():
    wl = _cells(5, [10, 30, 0, 2])
    r = oracle.blind(wl.arrays(), wl.cell_off, 1.0, 3)          # ceil(N) = N: nothing to merge
    assert r.out_total == wl.n
    r = oracle.blind(wl.arrays(), wl.cell_off, 0.5, 3, n_min_cell=30)
    assert list(np.diff(r.out_off)) == [10, 30, 0, 2]
    assert list(r.group[10:40]) == list(range(30))

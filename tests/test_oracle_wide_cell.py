"""The C oracle on a cell above 2^16 particles (a whole box merged as one cell), pinned to the exact
second implementation in tests/exact_tiny.py (Python integers: no width limit).

The method's first subset may be the whole simulation box (the paper's remark after the algorithm
on merging globally), so the oracle's FIXED mode takes cells of up to 2^24 particles.  In the cell
here the weights sit within 10 % of the largest and px near the top of its code range, so the
root's |S1| of px passes 2^53 (beyond what FP64 holds exactly) and the 128-bit products of Steps
3-4 carry values past 2^64.  Partition and merged particles must equal the exact ones.  The PAPER
mode keeps the FP64 GPU form's limit of 2^16 and flags a larger cell.
"""
import numpy as np

import oracle
from tests import exact_tiny as X
from tests.test_oracle_exact_tiny import _c_run, _values_differ


def heavy_cell(n, seed):
    r = np.random.Generator(np.random.Philox(seed))
    return np.stack([r.random(n), r.random(n), r.random(n), 3.0 + r.random(n), 1.0 + 0.1 * r.random(n),
                     -2.1 + 0.1 * r.random(n), 0.9 + 0.1 * r.random(n)], axis=1)


def test_fixed_cell_above_2_16_equals_exact():
    n = 150000
    rows = heavy_cell(n, seed=31).astype(np.float32).astype(np.float64)
    prm = (0.3, 0.05, 4, (1.0, 1.0, 1.0), 1.0, oracle.PAIR, 0)
    cell = X.Cell(rows, 0.3, 0.05, 4, (1.0, 1.0, 1.0), 1.0, X.FIXED)
    s1 = abs(sum(o * c[3] for o, c in zip(cell.omega, cell.codes)))
    assert s1 > 2 ** 53
    subs, per_subset = cell.run(X.PAIR)
    assert len(subs) > 2
    res, off = _c_run(oracle.run, [rows], prm, oracle.FIXED)
    assert int(res.stats["flags"][0]) == 0
    sid, per = res.subset_id, res.perm
    got = [list(per[sid == s]) for s in range(int(res.n_subsets[0]))]
    assert got == subs
    assert _values_differ(res, 0, per_subset, (1.0, 1.0, 1.0), 1.0) is None


def test_paper_mode_keeps_the_2_16_limit():
    rows = heavy_cell(65537, seed=32)
    res, _ = _c_run(oracle.run, [rows, rows[:100]], (0.3, 0.05, 4, (1.0, 1.0, 1.0), 1.0, oracle.PAIR, 0),
                    oracle.PAPER)
    assert int(res.stats["flags"][0]) & oracle.FLAG_TOO_LARGE
    assert res.n_subsets[0] == 0 and res.n_subsets[1] > 0
    res, _ = _c_run(oracle.run, [rows], (0.3, 0.05, 4, (1.0, 1.0, 1.0), 1.0, oracle.PAIR, 0), oracle.FIXED)
    assert int(res.stats["flags"][0]) == 0 and res.n_subsets[0] > 0

"""The C oracle against an exact second implementation on thousands of tiny cells (n <= 12).

tests/exact_tiny.py re-derives the method in exact arithmetic (FIXED decisions in Python integers,
PAPER decisions in Fractions, replacements in Fractions and 50-digit decimals) and shares no code
with oracle/vpm_oracle.c.  On seeded random cells and on adversarial ones (duplicates, exactly zero
mean momenta, equal CVs on two axes, exact ties between a position CV and a momentum CV, weights and
momenta over many octaves, lattices at zero tolerance, photons, one varying axis):

* FIXED partitions are identical, subset by subset and member by member;
* PAPER partitions are identical except in cells the C oracle certifies as holding a near-tie (a
  decision margin below 1e-9, where double rounding may go either way);
* replacement particles agree to 1e-12 (weights relative, positions against L, momenta against the
  particle's energy), which pins the pair direction rule as well;
* a replay of every C partition re-derives each internal node's axis and cut.

The mutation tests plant plausible mistakes in a copy of the C oracle (argmax for the pair axis's
argmin, a dropped carry in the 128x128-bit product, ties to the highest axis, a strict fixed-point
cut, a wrong
sign in the pair direction, a wrong shift in the momentum test) and check that these pins fail.
"""
import ctypes as C
import os
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
from tests import exact_tiny as X

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


# ------------------------------------------------------------------------------------------
# Cell families
# ------------------------------------------------------------------------------------------

def _rng(seed):
    return np.random.Generator(np.random.Philox(seed))


def generic(r):
    n = int(r.integers(2, 13))
    x = r.random((n, 3))
    p = np.array([1.0, 0.5, -0.3]) + 0.2 * r.standard_normal((n, 3))
    w = 0.5 + r.random((n, 1))
    return np.concatenate([x, p, w], 1)


def duplicates(r):
    n = int(r.integers(2, 13))
    pool = generic(r)[: int(r.integers(1, 4))]
    rows = pool[r.integers(0, pool.shape[0], n)].copy()
    rows[:, 6] = r.integers(1, 3, n)
    return rows


def zero_mean(r):
    half = int(r.integers(1, 7))
    p = np.array([1.0, 0.5, -0.3]) + 0.2 * r.standard_normal((half, 3))
    w = 0.5 + r.random(half)
    rows = np.zeros((2 * half, 7))
    rows[:, :3] = r.random((2 * half, 3))
    rows[:half, 3:6] = p
    rows[half:, 3:6] = p
    for a in range(3):
        if r.random() < 0.7:
            rows[half:, 3 + a] = -p[:, a]                     # equal weights: sum w p_a is exactly 0
    rows[:, 6] = np.concatenate([w, w])
    return rows


def equal_cv(r):
    rows = generic(r)
    rows[:, 1] = rows[:, 0]                                   # x and y: identical spreads
    rows[:, 5] = rows[:, 4]                                   # py and pz: identical CVs
    return rows


def scales(r):
    n = int(r.integers(2, 13))
    x = r.random((n, 3))
    p = np.sign(r.standard_normal((n, 3))) * 10.0 ** r.uniform(-3, 4, (n, 3))
    w = 2.0 ** r.uniform(-20, 20, (n, 1))
    return np.concatenate([x, p, w], 1)


def lattice(r):
    n = int(r.integers(2, 13))
    x = r.integers(0, 3, (n, 3)) * 0.25
    p = r.integers(-2, 3, (n, 3)).astype(np.float64)
    w = r.integers(1, 4, (n, 1)).astype(np.float64)
    return np.concatenate([x, p, w], 1)


def one_axis(r):
    n = int(r.integers(2, 13))
    rows = np.zeros((n, 7))
    rows[:, :3] = 0.5
    rows[:, 3] = r.integers(1, 40, n) * 0.125
    rows[:, 6] = r.integers(1, 5, n)
    return rows


def exact_tie(r):
    """Equal weights, a position axis a and a momentum axis b whose fixed-point CVs are exactly
    equal: with codes c_a (positions) and c_b = k c_a + m, m = k (2^16 n - sum c_a) / n, the two
    Delta^2 coincide as fractions (V scales by k^2; S1_b = k 2^16 n).  k = n 2^t puts the largest
    momentum code in [2^21, 2^22), so that the codes come out of the encoding exactly."""
    n = int(r.integers(2, 13))
    a, b = int(r.integers(0, 3)), int(r.integers(3, 6))
    ca = r.integers(-32768, 32768, n)
    ca[int(r.integers(0, n))] = -32768                        # the cell minimum codes to -32768
    base = n * ca + (65536 * n - int(ca.sum()))
    if np.all(base == 0):
        base[0] = 1
    t = 0
    while int(np.abs(base).max()) << t < 1 << 21:
        t += 1
    cb = base << t
    rows = np.zeros((n, 7))
    rows[:, :3] = 0.5                                         # the other axes do not vary: the tie
    rows[:, 3:6] = 0.25                                       # is the root's largest CV
    rows[:, a] = (ca + 32768) / 65536.0                       # exact in FP32; L = 1
    rows[:, b] = cb * 2.0 ** -21                              # largest |p| in [1, 2): codes = cb
    rows[:, 6] = 1.0
    return rows


FAMILIES = {"generic": generic, "duplicates": duplicates, "zero_mean": zero_mean, "equal_cv": equal_cv,
            "scales": scales, "lattice": lattice, "one_axis": one_axis, "exact_tie": exact_tie}

# (tol_x, tol_p, min_subset, L, mass, merge, axis_rule)
PARAM_SETS = [
    (0.3, 0.08, 2, (1.0, 1.0, 1.0), 1.0, oracle.PAIR, 0),
    (0.1, 0.05, 4, (1.0, 1.0, 1.0), 1.0, oracle.PAIR, 0),
    (1.0, 0.3, 2, (0.5, 2.0, 1.0), 0.0, oracle.PAIR, 0),
    (0.0, 0.0, 1, (1.0, 1.0, 1.0), 1.0, oracle.CENTROID, 0),
    (5.0, 5.0, 2, (1.0, 1.0, 1.0), 1.0, oracle.CENTROID, 0),
    (0.05, 0.02, 1, (1.0, 1.0, 1.0), 1.0, oracle.CENTROID, 0),
    (0.8, 0.03, 2, (1.0, 1.0, 1.0), 1.0, oracle.PAIR, 1),        # each CV over its tolerance
    (0.02, 0.4, 1, (1.0, 0.5, 1.0), 1.0, oracle.CENTROID, 1),
]
CELLS_PER_GROUP = {"generic": 70, "duplicates": 40, "zero_mean": 45, "equal_cv": 45, "scales": 45,
                   "lattice": 40, "one_axis": 30, "exact_tie": 50}


def groups():
    """[(name, params, [cell rows])]: every family under every parameter set, seeded."""
    out = []
    for fi, (fname, fn) in enumerate(FAMILIES.items()):
        for pi, prm in enumerate(PARAM_SETS):
            r = _rng(1000 * fi + pi)
            out.append((f"{fname}/{pi}", prm, [fn(r) for _ in range(CELLS_PER_GROUP[fname])]))
    return out


def _c_run(lib_run, cells, prm, decide):
    tol_x, tol_p, ms, L, mass, merge, rule = prm
    counts = [c.shape[0] for c in cells]
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    data = np.concatenate(cells, 0)
    return lib_run([data[:, i] for i in range(7)], off, tol_x=tol_x, tol_p=tol_p, n_min_cell=0,
                   min_subset=ms, cell_len=L, mass=mass, merge_mode=merge, decide=decide, axis_rule=rule), off


def _exact(cells, prm, mode):
    tol_x, tol_p, ms, L, mass, merge, rule = prm
    res = []
    for rows in cells:
        cell = X.Cell(rows, tol_x, tol_p, ms, L, mass, mode, rule)
        res.append((cell, *cell.run(X.PAIR if merge == oracle.PAIR else X.CENTROID)))
    return res


@pytest.fixture(scope="module")
def exact_results():
    """Exact partitions and outputs of every group in both modes (computed once)."""
    out = {}
    for name, prm, cells in groups():
        out[(name, X.FIXED)] = _exact(cells, prm, X.FIXED)
        out[(name, X.PAPER)] = _exact(cells, prm, X.PAPER)
    return out


def _compare(lib_run, exact_results, decide, check_values=True, replay=True):
    """Returns a list of disagreements (empty when the C oracle matches the exact results)."""
    mode = X.FIXED if decide == oracle.FIXED else X.PAPER
    bad = []
    n_cells = 0
    n_near = {}
    for name, prm, cells in groups():
        res, off = _c_run(lib_run, cells, prm, decide)
        L, mass = prm[3], prm[4]
        for ci, (cell, subs, rows) in enumerate(exact_results[(name, mode)]):
            n_cells += 1
            lo = int(off[ci])
            sid = res.subset_id[lo:off[ci + 1]]
            per = res.perm[lo:off[ci + 1]] - lo
            got = [list(per[sid == s]) for s in range(int(res.n_subsets[ci]))]
            near = mode == X.PAPER and res.stats["min_margin"][ci] < 1e-9
            n_near[name] = n_near.get(name, 0) + int(near)
            if got != subs:
                if not near:
                    bad.append((name, ci, "partition", got, subs))
                continue
            if replay and not near:
                err = X.replay(cell, got)
                if err:
                    bad.append((name, ci, "replay", err))
            if not check_values:
                continue
            err = _values_differ(res, ci, rows, L, mass)
            if err:
                bad.append((name, ci, "values", err))
    return bad, n_cells, n_near


def _values_differ(res, ci, per_subset, L, mass):
    """Compare the C outputs of cell ci with the exact ones subset by subset.  Copies: bit for bit.
    Centroids: weight relative, position against L, momentum against the particle's energy, 1e-12.
    Pairs: half weights, the common position, the pair's mean momentum and |delta|^2 (against the
    subset's mean energy and its square), and the direction of delta where |delta| > 1e-3 of the mean
    energy (below that sqrt(r) magnifies the rounding of r; the conserved quantities stay exact)."""
    o = int(res.out_off[ci])
    n_out = int(res.out_off[ci + 1]) - o
    if n_out != sum(len(r) for _, r, _ in per_subset):
        return f"count {n_out}"
    got = np.stack([res.out[f][o:o + n_out] for f in ("w", "x", "y", "z", "px", "py", "pz")], 1)
    k = 0
    for kind, rows, ebar in per_subset:
        e = np.array(rows, dtype=np.float64)
        g = got[k:k + len(rows)]
        k += len(rows)
        if kind == "copy":
            if not np.array_equal(g, e):
                return "copied particle changed"
            continue
        if np.any(np.abs(g[:, 0] - e[:, 0]) > 1e-12 * e[:, 0]):
            return "weight"
        if np.any(np.abs(g[:, 1:4] - e[:, 1:4]) > 1e-12 * np.array(L)):
            return "position"
        if len(rows) == 1:
            eps = np.sqrt(mass ** 2 + (e[0, 4:] ** 2).sum())
            if np.any(np.abs(g[0, 4:] - e[0, 4:]) > 1e-12 * eps):
                return "centroid momentum"
            continue
        sc = max(ebar, np.abs(e[:, 4:]).max())
        if np.any(np.abs((g[0, 4:] + g[1, 4:]) - (e[0, 4:] + e[1, 4:])) / 2 > 1e-12 * sc):
            return "pair mean momentum"
        dg, de = (g[0, 4:] - g[1, 4:]) / 2, (e[0, 4:] - e[1, 4:]) / 2
        if abs((dg ** 2).sum() - (de ** 2).sum()) > 1e-12 * sc * sc:
            return "|delta|^2"
        nd = np.sqrt((de ** 2).sum())
        if nd > 1e-3 * sc and np.any(np.abs(dg / np.sqrt((dg ** 2).sum()) - de / nd) > 1e-9):
            return "pair direction"
    return None


def test_enough_cells():
    n = sum(len(c) for _, _, c in groups())
    assert n >= 2000, n


def test_fixed_partitions_and_values_equal_exact(exact_results):
    bad, n, _ = _compare(oracle.run, exact_results, oracle.FIXED)
    assert not bad, bad[:5]
    assert n >= 2000


def test_paper_partitions_equal_exact_except_certified_near_ties(exact_results):
    bad, n, n_near = _compare(oracle.run, exact_results, oracle.PAPER)
    assert not bad, bad[:5]
    # Adversarial families are near-ties by construction, and at T = 0 every zero CV is one; on the
    # families without built-in ties and with T > 0 almost every cell is compared exactly.
    plain = [g for g in n_near if g.split("/")[0] in ("generic", "duplicates", "scales", "one_axis")
             and PARAM_SETS[int(g.split("/")[1])][0] > 0]
    cells = sum(CELLS_PER_GROUP[g.split("/")[0]] for g in plain)
    assert sum(n_near[g] for g in plain) < 0.05 * cells


def test_exact_ties_really_tie():
    """The exact_tie family holds exact ties between a position CV and a momentum CV at the root."""
    r = _rng(77)
    for _ in range(20):
        rows = exact_tie(r)
        cell = X.Cell(rows, 0.01, 0.01, 2)
        members = list(range(cell.n))
        S0 = sum(cell.omega)
        S1 = [sum(o * c[l] for o, c in zip(cell.omega, cell.codes)) for l in range(6)]
        S2 = [sum(o * c[l] ** 2 for o, c in zip(cell.omega, cell.codes)) for l in range(6)]
        V = [S0 * S2[l] - S1[l] ** 2 for l in range(6)]
        from fractions import Fraction
        d = [Fraction(V[l], 2 ** 32 * S0 ** 2) if l < 3 else (Fraction(V[l], S1[l] ** 2) if V[l] else 0)
             for l in range(6)]
        top = max(d)
        assert top > 0 and sum(v == top for v in d) >= 2
        del members


def test_replay_names_a_wrong_node():
    """The replay verifier rejects a partition whose first cut is moved by one particle."""
    rows = np.zeros((8, 7))
    rows[:, :3] = 0.5
    rows[:, 3] = [1.0, 1.1, 1.2, 3.0, 3.1, 5.0, 5.2, 0.9]
    rows[:, 6] = 1.0
    cell = X.Cell(rows, 0.5, 0.02, 1, mode=X.PAPER)
    subs, _ = cell.run(X.CENTROID)
    assert X.replay(cell, subs) is None
    wrong = [list(s) for s in subs]
    moved = wrong[-1].pop()
    wrong[0].append(moved)
    assert X.replay(cell, wrong) is not None


# ------------------------------------------------------------------------------------------
# Planted mistakes in a copy of the C oracle must fail the pins
# ------------------------------------------------------------------------------------------

MUTATIONS = {
    # the pair-direction axis of FIXED mode taken as the argmax instead of the argmin
    "jdir_argmax": ("if (a == 0 || v < bv) { bv = v; best = a; }", "if (a == 0 || v > bv) { bv = v; best = a; }"),
    # the inner carry of the 128 x 128-bit product dropped
    "u256_carry": ("carry = t >> 64;\n        }\n        int k = i + 2;", "carry = 0;\n        }\n        int k = i + 2;"),
    # Step 4 ties going to the highest axis in FIXED mode
    "ties_high": (": frac_gt(f, best);", ": !frac_gt(best, f);"),
    # Step 5 in FIXED mode with a strict cut (c S0 < S1)
    "strict_cut": ("if ((i128)cc->c[k][i] * S.s0 <= (i128)S.s1[k])", "if ((i128)cc->c[k][i] * S.s0 < (i128)S.s1[k])"),
    # the pair direction's projection with the wrong sign
    "pair_sign": ("u[a] -= P[jdir] * P[a] / P2;", "u[a] += P[jdir] * P[a] / P2;"),
    # the momentum test's scale 2^48 off by one bit
    "mom_shift": ("(u128)1 << (l < 3 ? 16 : 48)", "(u128)1 << (l < 3 ? 16 : 47)"),
    # the normalised axis rule dividing by the wrong tolerance
    "norm_swap": ("frac_gt_norm(f, l < 3 ? tx2 : tp2, best, k < 3 ? tx2 : tp2)",
                  "frac_gt_norm(f, l < 3 ? tp2 : tx2, best, k < 3 ? tp2 : tx2)"),
}


def _mutant_runner(tmpdir, name):
    src = open(os.path.join(ROOT, "oracle", "vpm_oracle.c")).read()
    old, new = MUTATIONS[name]
    assert src.count(old) == 1, name
    path_c = os.path.join(tmpdir, f"mut_{name}.c")
    path_so = os.path.join(tmpdir, f"libmut_{name}.so")
    open(path_c, "w").write(src.replace(old, new))
    subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                           "-fno-fast-math", "-o", path_so, path_c])
    return oracle.runner(C.CDLL(path_so))


@pytest.mark.parametrize("name,decide", [("jdir_argmax", oracle.FIXED), ("u256_carry", oracle.FIXED),
                                         ("ties_high", oracle.FIXED), ("strict_cut", oracle.FIXED),
                                         ("pair_sign", oracle.PAPER), ("mom_shift", oracle.FIXED),
                                         ("norm_swap", oracle.FIXED)])
def test_planted_mistake_is_caught(exact_results, name, decide):
    with tempfile.TemporaryDirectory() as d:
        run = _mutant_runner(d, name)
        bad, _, _ = _compare(run, exact_results, decide)
    assert bad, f"mutation {name} was not detected"

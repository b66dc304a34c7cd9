"""An exact second implementation of the merge method for tiny cells -- test infrastructure.

It exists to pin the C oracle (oracle/vpm_oracle.c) to something other than itself.  It shares no
code with it: the recursion, the decisions and the replacement are written out again here from the
paper (Sec. "Algorithm", Steps 1-7, and the two-particle merge of its remarks), in exact arithmetic:

* PAPER decisions in rational numbers (fractions.Fraction) on the exact binary values of the inputs:
  W = sum w, mean_l = sum w q_l / W, sigma_l^2 = sum w (q_l - mean_l)^2 / W (Steps 1-2); the CVs
  sigma/L and sigma/|P| (Eqs. cv_x, cv_p) compared through their squares, so no square root is
  taken; finished when all six are <= T (Step 3); otherwise the axis of the largest CV, ties to the
  lowest axis (Step 4); V1 = {q <= mean} in stable order (Steps 5-6).
* FIXED decisions in Python integers from the per-cell fixed-point codes (the encoding itself is a
  handful of IEEE single-precision operations, done with numpy float32 scalars):
  omega = rint(w 2^(15 - e_w)), position code rint(fl32(fl32(x - lo) * fl32(65536 / L))) - 32768
  (clamped to 65535 - 32768), momentum code rint(p 2^(22 - e_a)); moments S0, S1, S2; the tests
  V 2^16 <= T^2 S0^2 (positions) and V 2^48 <= T^2 S1^2 (momenta), T^ = rint(T 2^24); the argmax of
  V / D as exact fractions (or, with the tolerance-normalised axis rule, of V 2^48 / (D T^2)); the
  cut c S0 <= S1.
* Replacement with exact sums (Fractions); the pair's square roots in 50-digit decimals.  The pair
  direction: the momentum axis j with the smallest |sum w p_j| (on the codes in FIXED mode), ties
  to the lowest j; u = e_j - (e_j . P) P / |P|^2 (u = e_j when P = 0); delta = sqrt(r) u / |u| with
  r = mean(eps)^2 - m^2 - |P|^2, eps = sqrt(m^2 + |p|^2).

`replay` checks a claimed partition node by node against these decisions and names the first node
where it departs from them.
"""
from __future__ import annotations

import math
from decimal import Decimal, localcontext
from fractions import Fraction

import numpy as np

PAPER, FIXED = "paper", "fixed"
PAIR, CENTROID = "pair", "centroid"
INF = None          # an infinite CV^2 (sigma > 0 with zero mean momentum)


# ------------------------------------------------------------------------------------------
# FIXED-mode codes (single-precision encoding, then integers)
# ------------------------------------------------------------------------------------------

def _f32(v) -> np.float32:
    return np.float32(v)


def _rint32(v: np.float32) -> int:
    return int(np.rint(np.float32(v)))          # round half to even, as rintf


def _frexp_exp(v: float) -> int:
    return math.frexp(float(v))[1] if v > 0 else 0


def fixed_codes(rows, L):
    """rows: list of (x, y, z, px, py, pz, w) already rounded to FP32.  Returns (omega, codes[6]
    per particle, momentum exponents e_a, zero-axis flags)."""
    n = len(rows)
    w = [_f32(r[6]) for r in rows]
    e_w = _frexp_exp(max(w))
    omega = [_rint32(np.ldexp(wi, 15 - e_w).astype(np.float32)) for wi in w]
    codes = [[0] * 6 for _ in range(n)]
    for a in range(3):
        xs = [_f32(r[a]) for r in rows]
        lo = min(xs)
        s = _f32(65536.0 / L[a])
        for i in range(n):
            d = np.float32(xs[i] - lo)               # one FP32 subtraction
            t = np.float32(d * s)                    # one FP32 product
            r = float(np.rint(t))
            codes[i][a] = int(min(r, 65535.0)) - 32768
    e_p, zero = [0, 0, 0], [False, False, False]
    for a in range(3):
        ps = [_f32(r[3 + a]) for r in rows]
        mx = max(abs(v) for v in ps)
        zero[a] = mx == 0
        e_p[a] = _frexp_exp(mx)
        for i in range(n):
            codes[i][3 + a] = 0 if zero[a] else _rint32(np.ldexp(ps[i], 22 - e_p[a]).astype(np.float32))
    return omega, codes, e_p, zero


def _fixed_decide(members, omega, codes, e_p, that_x, that_p, axis_rule=0):
    """(kind, axis, cut, jdir) for a subset in FIXED mode; kind is 'merge' or 'split'."""
    S0 = sum(omega[i] for i in members)
    S1 = [sum(omega[i] * codes[i][l] for i in members) for l in range(6)]
    S2 = [sum(omega[i] * codes[i][l] ** 2 for i in members) for l in range(6)]
    # pair direction: smallest |sum omega c_j| 2^(e_j) over the momentum axes, ties to the lowest
    emin = min(e_p)
    mag = [abs(S1[3 + a]) << (e_p[a] - emin) for a in range(3)]
    jdir = min(range(3), key=lambda a: (mag[a], a))
    if S0 == 0:
        return "merge", 0, 0, jdir
    V = [S0 * S2[l] - S1[l] ** 2 for l in range(6)]
    assert all(v >= 0 for v in V)
    done = True
    for l in range(6):
        if V[l] == 0:
            continue
        if l < 3:
            done &= V[l] * 2 ** 16 <= that_x ** 2 * S0 ** 2
        else:
            done &= S1[l] != 0 and V[l] * 2 ** 48 <= that_p ** 2 * S1[l] ** 2
    if done:
        return "merge", 0, 0, jdir

    def delta2(l):
        if V[l] == 0:
            return Fraction(0)
        D = 2 ** 32 * S0 ** 2 if l < 3 else S1[l] ** 2
        if axis_rule:                       # Delta^2 / T^2, T = T^ / 2^24
            D *= (that_x if l < 3 else that_p) ** 2
            V_l = V[l] * 2 ** 48
        else:
            V_l = V[l]
        return INF if D == 0 else Fraction(V_l, D)

    k, best = 0, delta2(0)
    for l in range(1, 6):
        d = delta2(l)
        if best is INF:
            break
        if d is INF or d > best:
            k, best = l, d
    return "split", k, S1[k], S0, jdir


def _paper_decide(members, q, w, L, tol_x, tol_p, axis_rule=0):
    W = sum(w[i] for i in members)
    mean = [sum(w[i] * q[l][i] for i in members) / W for l in range(6)]
    var = [sum(w[i] * (q[l][i] - mean[l]) ** 2 for i in members) / W for l in range(6)]
    sums = [abs(sum(w[i] * q[3 + a][i] for i in members)) for a in range(3)]
    jdir = min(range(3), key=lambda a: (sums[a], a))

    def delta2(l):
        if l < 3:
            return var[l] / L[l] ** 2
        if var[l] == 0:
            return Fraction(0)
        return INF if mean[l] == 0 else var[l] / mean[l] ** 2

    d2 = [delta2(l) for l in range(6)]
    T2 = [tol_x ** 2] * 3 + [tol_p ** 2] * 3
    if all(d is not INF and d <= T2[l] for l, d in enumerate(d2)):
        return "merge", 0, mean, jdir
    if axis_rule:                           # each CV over its tolerance (> 0 over 0: infinite)
        d2 = [d if d is INF or d == 0 else (d / T2[l] if T2[l] > 0 else INF) for l, d in enumerate(d2)]
    k = 0
    for l in range(1, 6):
        if d2[k] is INF:
            break
        if d2[l] is INF or d2[l] > d2[k]:
            k = l
    return "split", k, mean[k], jdir


# ------------------------------------------------------------------------------------------
# The recursion (Steps 1-6) and the replacement (Step 7)
# ------------------------------------------------------------------------------------------

class Cell:
    """One cell: rows of 7 floats (x, y, z, px, py, pz, w) and the merge parameters."""

    def __init__(self, rows, tol_x, tol_p, min_subset, L=(1.0, 1.0, 1.0), mass=1.0, mode=FIXED, axis_rule=0):
        self.mode = mode
        self.axis_rule = int(axis_rule)
        if mode == FIXED:
            rows = [tuple(float(np.float32(v)) for v in r) for r in rows]
        self.rows = [tuple(float(v) for v in r) for r in rows]
        self.n = len(rows)
        self.tol_x, self.tol_p = float(tol_x), float(tol_p)
        self.min_subset = int(min_subset)
        self.L = [float(v) for v in L]
        self.mass = float(mass)
        self.q = [[Fraction(r[l]) for r in self.rows] for l in range(6)]
        self.w = [Fraction(r[6]) for r in self.rows]
        if mode == FIXED:
            self.omega, self.codes, self.e_p, _ = fixed_codes(self.rows, self.L)
            self.that_x = int(np.rint(self.tol_x * 2 ** 24))
            self.that_p = int(np.rint(self.tol_p * 2 ** 24))

    def decide(self, members):
        """('copy',) | ('merge', jdir) | ('split', axis, V1, V2) for a subset (a list in stable order)."""
        if len(members) < self.min_subset:
            return ("copy",)
        if self.mode == FIXED:
            r = _fixed_decide(members, self.omega, self.codes, self.e_p, self.that_x, self.that_p, self.axis_rule)
            if r[0] == "merge":
                return ("merge", r[3])
            _, k, s1, s0, jdir = r
            v1 = [i for i in members if self.codes[i][k] * s0 <= s1]
        else:
            r = _paper_decide(members, self.q, self.w, self.L, Fraction(self.tol_x), Fraction(self.tol_p),
                              self.axis_rule)
            if r[0] == "merge":
                return ("merge", r[3])
            _, k, cut, jdir = r
            v1 = [i for i in members if self.q[k][i] <= cut]
        in1 = set(v1)
        v2 = [i for i in members if i not in in1]
        assert v1 and v2, "a cut through the exact mean always leaves both sides non-empty"
        return ("split", k, v1, v2)

    def partition(self):
        """Final subsets in depth-first order (V1 first): list of (members, kind, jdir)."""
        out = []

        def rec(members):
            d = self.decide(members)
            if d[0] == "copy":
                out.append((members, "copy", 0))
            elif d[0] == "merge":
                out.append((members, "merge", d[1]))
            else:
                rec(d[2])
                rec(d[3])

        rec(list(range(self.n)))
        return out

    def merged(self, members, jdir, merge):
        """The replacement particles of a finished subset: list of (w, x, y, z, px, py, pz) as
        Fractions (CENTROID) or Decimals (PAIR momenta)."""
        W = sum(self.w[i] for i in members)
        X = [sum(self.w[i] * self.q[a][i] for i in members) / W for a in range(3)]
        P = [sum(self.w[i] * self.q[3 + a][i] for i in members) / W for a in range(3)]
        if merge == CENTROID:
            return [(W, *X, *P)]
        with localcontext() as ctx:
            ctx.prec = 50
            D = lambda f: Decimal(f.numerator) / Decimal(f.denominator)
            m2 = D(Fraction(self.mass) ** 2)
            eps = [(m2 + D(sum(self.q[3 + a][i] ** 2 for a in range(3)))).sqrt() for i in members]
            ebar = sum(D(self.w[i]) * e for i, e in zip(members, eps)) / D(W)
            P2 = sum(p * p for p in P)
            r = ebar * ebar - m2 - D(P2)
            r = max(r, Decimal(0))
            u = [Fraction(1 if a == jdir else 0) for a in range(3)]
            if P2 > 0:
                u = [u[a] - P[jdir] * P[a] / P2 for a in range(3)]
            un = D(sum(v * v for v in u)).sqrt()
            s = r.sqrt() / un
            Pd = [D(p) for p in P]
            ud = [D(v) for v in u]
            a = [Pd[k] + s * ud[k] for k in range(3)]
            b = [Pd[k] - s * ud[k] for k in range(3)]
        return [(W / 2, *X, *a), (W / 2, *X, *b)]

    def run(self, merge):
        """(final subsets as member lists, per subset: (kind, its output rows (w, x, y, z, px, py, pz)
        as floats, its mean energy)); outputs follow the subsets' order."""
        subs, out = [], []
        for members, kind, jdir in self.partition():
            subs.append(members)
            if kind == "copy":
                out.append((kind, [(r[6], *r[:6]) for r in (self.rows[i] for i in members)], 0.0))
            else:
                W = sum(self.w[i] for i in members)
                eps = sum(float(self.w[i]) * math.sqrt(self.mass ** 2 + sum(self.rows[i][3 + a] ** 2
                                                                            for a in range(3)))
                          for i in members) / float(W)
                out.append((kind, [tuple(float(v) for v in p) for p in self.merged(members, jdir, merge)], eps))
        return subs, out


def replay(cell: Cell, claimed):
    """Check a claimed partition (final subsets in order, each a list of cell-local indices in slot
    order) against the decisions, node by node.  Returns None if it is the method's partition, else
    a text naming the first node where the claim departs."""
    pos = [0]

    def rec(members, path):
        d = cell.decide(members)
        if d[0] == "split":
            k, v1, v2 = d[1], d[2], d[3]
            # the claimed leaves under this node must cover exactly V1, then exactly V2
            for side, part in (("V1", v1), ("V2", v2)):
                start = pos[0]
                err = rec(part, path + f"/{side}(axis {k})")
                if err:
                    return err
                got = sorted(i for s in claimed[start:pos[0]] for i in s)
                if got != sorted(part):
                    return f"node {path}: claimed {side} members {got} but the cut gives {sorted(part)}"
            return None
        if pos[0] >= len(claimed):
            return f"node {path}: final subset {members} missing from the claim"
        got = list(claimed[pos[0]])
        pos[0] += 1
        if sorted(got) != sorted(members):
            return f"node {path}: claimed final subset {sorted(got)} but the node is {sorted(members)} ({d[0]})"
        if got != members:
            return f"node {path}: members of {members} not in input order: {got}"
        return None

    err = rec(list(range(cell.n)), "root")
    if err is None and pos[0] != len(claimed):
        err = f"{len(claimed) - pos[0]} claimed subsets left over"
    return err

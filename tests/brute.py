"""Brute-force, exact-rational pins for tiny instances (test helper).

Nothing here uses BDDs or shortest paths: every feasible set is enumerated
explicitly, and min-marginals are minima over the enumerated points (Sec. 3,
Def. "Min-marginals").  All arithmetic is on ``fractions.Fraction`` built from
the exact binary value of each float input, so results are exact.
"""
from __future__ import annotations

import itertools
from fractions import Fraction

import numpy as np


def sense_ok(v, sense, b):
    return v <= b if sense < 0 else v >= b if sense > 0 else v == b


def row_points(coefs, sense, rhs):
    """All 0/1 tuples over the row's variables that satisfy the row."""
    k = len(coefs)
    return [x for x in itertools.product((0, 1), repeat=k)
            if sense_ok(sum(int(a) * xi for a, xi in zip(coefs, x)), sense, rhs)]


def check_rows(ilp, x) -> int:
    """number of original rows violated by x (exact integers)"""
    bad = 0
    for r in range(ilp.n_rows):
        c, a, s, b = ilp.row(r)
        lhs = sum(int(ai) * int(x[ci]) for ci, ai in zip(c, a))
        bad += not sense_ok(lhs, s, b)
    return bad


def ilp_opt(ilp):
    """exact optimum and all optimal points by enumerating {0,1}^n (n <= 20)"""
    n = ilp.n_vars
    assert n <= 20
    best, arg = None, []
    costs = [Fraction(float(c)) for c in ilp.costs]
    for x in itertools.product((0, 1), repeat=n):
        if check_rows(ilp, x):
            continue
        v = sum(c for c, xi in zip(costs, x) if xi)
        if best is None or v < best:
            best, arg = v, [x]
        elif v == best:
            arg.append(x)
    return best, arg


def presolve(ilp):
    """Fix variables that some row allows only one value for, until nothing changes.

    Returns (fixed[n] in {-1,0,1}, kept rows as (row_id, vars, points)) or None if
    the rows cannot all be satisfied.
    """
    n = ilp.n_vars
    fixed = [-1] * n

    def residual(r):
        c, a, s, b = ilp.row(r)
        vs, cs = [], []
        for ci, ai in zip(c, a):
            ci, ai = int(ci), int(ai)
            if ai == 0:
                continue
            if fixed[ci] >= 0:
                b -= ai * fixed[ci]
            else:
                vs.append(ci)
                cs.append(ai)
        order = np.argsort(vs, kind="stable")
        return [vs[i] for i in order], [cs[i] for i in order], s, b

    changed = True
    while changed:
        changed = False
        for r in range(ilp.n_rows):
            vs, cs, s, b = residual(r)
            pts = row_points(cs, s, b)
            if not pts:
                return None
            for h, v in enumerate(vs):
                vals = {p[h] for p in pts}
                if len(vals) == 1:
                    fixed[v] = vals.pop()
                    changed = True
    kept = []
    for r in range(ilp.n_rows):
        vs, cs, s, b = residual(r)
        if vs:
            kept.append((r, vs, row_points(cs, s, b)))
    return fixed, kept


class ExactAlg1:
    """Alg. 1 with enumeration-based min-marginals, in exact rationals."""

    def __init__(self, ilp, omega=Fraction(1, 2)):
        self.ilp = ilp
        self.omega = Fraction(omega)
        res = presolve(ilp)
        assert res is not None
        self.fixed, self.rows = res
        n = ilp.n_vars
        self.c = [Fraction(float(v)) for v in ilp.costs]
        self.deg = [0] * n
        for _, vs, _ in self.rows:
            for v in vs:
                self.deg[v] += 1
        self.lam = [[self.c[v] / self.deg[v] for v in vs] for _, vs, _ in self.rows]
        self.M = [[Fraction(0)] * len(vs) for _, vs, _ in self.rows]
        self.avg = [Fraction(0)] * n
        self.E = [Fraction(0)] * len(self.rows)
        off = Fraction(0)
        for i in range(n):
            if self.fixed[i] >= 0:
                off += self.c[i] * self.fixed[i]
            elif self.deg[i] == 0:
                off += min(self.c[i], Fraction(0))
        self.offset = off

    @staticmethod
    def energy(pts, lam):
        return min(sum(l for l, xi in zip(lam, x) if xi) for x in pts)

    @staticmethod
    def min_marginals(pts, lam, h):
        m = [None, None]
        for x in pts:
            v = sum(l for l, xi in zip(lam, x) if xi)
            b = x[h]
            if m[b] is None or v < m[b]:
                m[b] = v
        return m

    def sweep(self, direction):
        w = self.omega
        for j, (_, vs, pts) in enumerate(self.rows):
            lam = self.lam[j]
            order = range(len(vs)) if direction == 0 else range(len(vs) - 1, -1, -1)
            for h in order:
                m0, m1 = self.min_marginals(pts, lam, h)
                self.M[j][h] = m1 - m0
                lam[h] = lam[h] - w * self.M[j][h] + self.avg[vs[h]]
            self.E[j] = self.energy(pts, lam)

    def average(self):
        acc = [Fraction(0)] * self.ilp.n_vars
        for j, (_, vs, _) in enumerate(self.rows):
            for h, v in enumerate(vs):
                acc[v] += self.M[j][h]
        self.avg = [self.omega / d * a if d else Fraction(0) for a, d in zip(acc, self.deg)]

    def lb_free(self):
        t = sum((min(m, Fraction(0)) for Mj in self.M for m in Mj), Fraction(0))
        return sum(self.E, Fraction(0)) + self.omega * t + self.offset

    def lb_cert(self):
        e = Fraction(0)
        for j, (_, vs, pts) in enumerate(self.rows):
            e += self.energy(pts, [l + self.omega * m for l, m in zip(self.lam[j], self.M[j])])
        return e + self.offset

    def residual(self):
        acc = [Fraction(0)] * self.ilp.n_vars
        for j, (_, vs, _) in enumerate(self.rows):
            for h, v in enumerate(vs):
                acc[v] += self.lam[j][h] + self.omega * self.M[j][h]
        return [acc[i] - self.c[i] if self.deg[i] else Fraction(0) for i in range(self.ilp.n_vars)]

    def flat(self, which):
        src = self.lam if which == "lam" else self.M
        return [v for row in src for v in row]


def completions(ilp, fixed, limit=2):
    """Number (capped at limit) of 0/1 completions of a partial assignment
    (fixed[i] in {-1,0,1}) that satisfy every row: depth-first search with
    interval propagation over the rows, generic in the rows' content."""
    n = ilp.n_vars
    rows = [ilp.row(r) for r in range(ilp.n_rows)]
    rows = [([int(c) for c in cs], [int(a) for a in as_], int(s), int(b)) for cs, as_, s, b in rows]
    by_var = [[] for _ in range(n)]
    for r, (cs, _, _, _) in enumerate(rows):
        for c in cs:
            by_var[c].append(r)

    def propagate(x, queue):
        while queue:
            r = queue.pop()
            cs, as_, s, b = rows[r]
            lo = hi = 0
            for c, a in zip(cs, as_):
                if x[c] >= 0:
                    lo += a * x[c]
                    hi += a * x[c]
                elif a < 0:
                    lo += a
                else:
                    hi += a
            if (s <= 0 and lo > b) or (s >= 0 and hi < b):
                return False
            for c, a in zip(cs, as_):
                if x[c] >= 0:
                    continue
                # the value of x_c that moves the sum to each end
                v = None
                if s <= 0 and lo + abs(a) > b:
                    v = 0 if a > 0 else 1          # the other value would exceed b
                if s >= 0 and hi - abs(a) < b:
                    w = 1 if a > 0 else 0          # the other value would fall short of b
                    if v is not None and v != w:
                        return False
                    v = w
                if v is not None:
                    x[c] = v
                    queue.extend(by_var[c])   # r among them: its interval is recomputed
                    break
        return True

    def dfs(x):
        free = [i for i in range(n) if x[i] < 0]
        if not free:
            return 1
        best = min(free, key=lambda i: min(sum(x[c] < 0 for c in rows[r][0]) for r in by_var[i]) if by_var[i] else n)
        total = 0
        for v in (0, 1):
            y = list(x)
            y[best] = v
            if propagate(y, list(by_var[best])):
                total += dfs(y)
                if total >= limit:
                    return total
        return total

    x = [int(v) for v in fixed]
    if not propagate(x, list(range(len(rows)))):
        return 0
    return dfs(x)

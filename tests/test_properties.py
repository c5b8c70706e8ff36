"""Property tests over generated tiny ILPs (hypothesis; no GPU).

Instances: <= 8 variables, <= 5 rows of 1..5 variables, coefficients in
{-3..3} \\ {0}, any sense, right-hand sides around a hidden 0/1 point (always
feasible) or drawn freely (possibly infeasible).  Every property is checked
against full enumeration (``brute``): feasibility and presolve, min-marginals
at the initial multipliers (Sec. 3, Def. "Min-marginals"), the feasibility
identity of the iterates (Prop. 1), weak duality of both bounds against the
enumerated optimum, and the host-side packing of the C ABI against the
reference implementation's pair lists.
"""
from fractions import Fraction

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import brute
import oracle as O
from paper_2111_10270_amd import binding as B
from paper_2111_10270_amd import instances as I

SETTINGS = settings(max_examples=60, deadline=None, derandomize=True,
                    suppress_health_check=[HealthCheck.too_slow])


@st.composite
def tiny_ilps(draw):
    n = draw(st.integers(1, 8))
    hidden = draw(st.lists(st.integers(0, 1), min_size=n, max_size=n))
    rows = []
    for _ in range(draw(st.integers(0, 5))):
        k = draw(st.integers(1, min(5, n)))
        vs = draw(st.lists(st.integers(0, n - 1), min_size=k, max_size=k, unique=True))
        a = [draw(st.sampled_from([-3, -2, -1, 1, 2, 3])) for _ in vs]
        sense = draw(st.sampled_from([-1, 0, 1]))
        if draw(st.booleans()):
            lhs = sum(ai * hidden[v] for ai, v in zip(a, vs))
            slack = draw(st.integers(0, 2))
            rhs = lhs + (slack if sense < 0 else -slack if sense > 0 else 0)
        else:
            rhs = draw(st.integers(-6, 6))
        rows.append((vs, a, sense, rhs))
    # dyadic costs keep every sum of a few terms exact
    costs = [draw(st.integers(-16, 16)) / 4 for _ in range(n)]
    return I.from_rows(n, costs, rows, name="hyp")


@SETTINGS
@given(tiny_ilps())
def test_feasibility_and_presolve_match_enumeration(ilp):
    o = O.Oracle(ilp)
    opt, _ = brute.ilp_opt(ilp)
    if opt is None:
        # the rows may be jointly infeasible while presolve (single-row
        # implications) does not prove it; a proof must be right, though
        return
    # a feasible ILP is never declared infeasible
    assert o.status == O.OK
    ref = brute.presolve(ilp)
    assert ref is not None
    fixed, _ = ref
    assert list(o.fixed()) == list(fixed)


@SETTINGS
@given(tiny_ilps())
def test_initial_min_marginals_equal_enumeration(ilp):
    o = O.Oracle(ilp)
    if o.status != O.OK:
        return
    ref = brute.presolve(ilp)
    _, rows = ref
    o.init()
    mm = o.full_mm()
    lam, _, _ = o.get()
    at = 0
    for _, vs, pts in rows:
        lf = [Fraction(float(v)) for v in lam[at:at + len(vs)]]
        for q in range(len(vs)):
            m0, m1 = brute.ExactAlg1.min_marginals(pts, lf, q)
            # lambda = c / |J| is not dyadic for |J| = 3, 5, ...: the float sums
            # along a path round, the enumeration does not
            assert abs(mm[at + q] - float(m1 - m0)) <= 1e-12 * max(1.0, abs(float(m1 - m0)))
        at += len(vs)
    assert at == len(mm)


@SETTINGS
@given(tiny_ilps())
def test_iterates_feasible_and_bounds_below_optimum(ilp):
    o = O.Oracle(ilp)
    if o.status != O.OK:
        return
    opt, _ = brute.ilp_opt(ilp)
    o.init()
    pv, _ = o.pairs()
    used = np.bincount(pv, minlength=ilp.n_vars) > 0
    prev = -np.inf
    for s in range(12):
        o.sweep(s % 2)
        o.average()
        lam, mm, _ = o.get()
        acc = np.zeros(ilp.n_vars)
        np.add.at(acc, pv, lam + 0.5 * mm)
        assert np.max(np.abs(acc[used] - ilp.costs[used]), initial=0) <= 1e-12
        lbf = o.lb_free()
        lbc, _ = o.lb_cert()
        assert prev - 1e-12 <= lbf <= lbc + 1e-12
        assert lbc <= float(opt) + 1e-12
        prev = lbf


@SETTINGS
@given(tiny_ilps())
def test_host_packing_matches_reference(ilp):
    o = O.Oracle(ilp)
    if o.status == O.INFEASIBLE:
        with pytest.raises(B.BddmmaError) as e:
            B.Solver(ilp)
        assert e.value.code == B.INFEASIBLE
        return
    for kw in (dict(), dict(small_tiles=0, class_merge_kib=0), dict(fast_path=0)):
        s = B.Solver(ilp, **kw)
        pv, pr = s.pairs()
        opv, opr = o.pairs()
        assert np.array_equal(pv, opv) and np.array_equal(pr, opr)
        assert np.array_equal(s.fixed(), o.fixed())
        assert s.stats.lb_offset == o.lb_offset()
        assert s.stats.n_slots >= s.stats.n_pairs and s.stats.n_slots % 64 == 0

"""Pins of the serial min-marginal averaging in the reference implementation
(the sequential update of Sec. 3 the paper compares its deferred scheme with):
a hand-worked iteration, dual feasibility, monotone bounds below the brute-force
optimum, the agreement of averaged min-marginal differences, and the
decomposable special case where the bound is exact."""
import os

import numpy as np
import pytest

import brute
import oracle as O
from paper_2111_10270_amd import instances as I
from test_oracle import _read, example_a, example_b


def _feasibility_gap(o, ilp):
    lam, _, _ = o.get()
    pv, _ = o.pairs()
    s = np.zeros(ilp.n_vars)
    np.add.at(s, pv, lam)
    used = np.bincount(pv, minlength=ilp.n_vars) > 0
    return float(np.max(np.abs(s - np.asarray(ilp.costs))[used], initial=0.0))


def test_hand_worked_iteration_on_example_b():
    g = _read("serial_example_b.txt")
    o = O.Oracle(example_b())
    o.init()
    lb = o.run_serial(1)
    lam, mm, _ = o.get()
    assert np.array_equal(lam, np.array([float(v) for v in g["lambda"][0]]))
    assert np.array_equal(lb, np.array([float(v) for v in g["bounds"][0]]))
    assert np.all(mm == 0.0)


def test_example_a_bound_stays_at_the_optimum():
    o = O.Oracle(example_a()[0])
    o.init()
    assert np.all(o.run_serial(5) == -5.0)


@pytest.mark.parametrize("seed", range(12))
def test_feasible_monotone_and_below_the_optimum(seed):
    ilp = I.random_ilp(9, 7, max_row_len=5, seed=800 + seed)
    o = O.Oracle(ilp)
    if o.status != O.OK:
        pytest.skip("infeasible draw")
    opt, _ = brute.ilp_opt(ilp)
    o.init()
    o.run_dual(2)                     # start from a deferred state: the run terminates it first
    prev = -np.inf
    for _ in range(6):
        lb = o.run_serial(1)
        assert _feasibility_gap(o, ilp) <= 1e-12 * max(1.0, float(np.max(np.abs(ilp.costs))))
        for v in lb:
            assert v >= prev - 1e-12 * max(1.0, abs(v))
            assert v <= opt + 1e-9 * max(1.0, abs(opt))
            prev = v


def test_last_visited_variable_has_equal_differences():
    """after the backward sweep, variable 0 was averaged last: its min-marginal
    differences agree across all its subproblems (up to rounding of the
    later no-op updates of |J| = 1 variables)"""
    ilp = I.mrf_grid(4, 5, 3, pairwise="potts", seed=2)
    o = O.Oracle(ilp)
    o.init()
    o.run_serial(3)
    mm = o.full_mm()
    pv, _ = o.pairs()
    m0 = mm[pv == 0]
    assert m0.size >= 2
    assert np.max(np.abs(m0 - m0[0])) <= 1e-9 * max(1.0, float(np.max(np.abs(m0))))


def test_variable_disjoint_rows_reach_the_optimum():
    """every variable in at most one row: the decomposition is exact, the
    serial update changes nothing and the bound equals the optimum"""
    rows = [([0, 1, 2], [1, 1, 1], -1, 1), ([3, 4], [2, -1], 1, 0), ([5, 6, 7], [1, 2, 1], 0, 2)]
    ilp = I.from_rows(9, [-1.0, 0.5, -2.0, 1.0, -1.5, -0.25, 0.75, -3.0, 2.0], rows)
    o = O.Oracle(ilp)
    o.init()
    lam0 = o.get()[0].copy()
    lb = o.run_serial(2)
    opt, _ = brute.ilp_opt(ilp)
    assert np.array_equal(o.get()[0], lam0)
    assert np.all(lb == opt)

"""Pins of the averaging form of the termination step in the reference
implementation (the text's description, one more min-marginal averaging,
instead of the algorithm's last loop): exact dual feasibility, certified bounds below the
enumerated optimum, the paper's Example A, and the cases where both forms must
coincide."""
import numpy as np
import pytest

import brute
import oracle as O
from paper_2111_10270_amd import instances as I
from test_oracle import example_a


def _sums(o, ilp):
    lam, _, _ = o.get()
    pv, _ = o.pairs()
    s = np.zeros(ilp.n_vars)
    np.add.at(s, pv, lam)
    used = np.bincount(pv, minlength=ilp.n_vars) > 0
    return s[used], np.asarray(ilp.costs)[used]


@pytest.mark.parametrize("seed", range(10))
def test_averaging_termination_is_feasible_and_certified(seed):
    ilp = I.random_ilp(9, 7, max_row_len=5, seed=1200 + seed)
    o = O.Oracle(ilp)
    if o.status != O.OK:
        pytest.skip("infeasible draw")
    opt, _ = brute.ilp_opt(ilp)
    o.init()
    o.run_dual(4)
    o.set_termination(1)
    cert, res = o.lb_cert()
    assert cert <= opt + 1e-9 * max(1.0, abs(opt))
    assert res <= 1e-12 * max(1.0, float(np.max(np.abs(ilp.costs))))
    o.terminate()
    s, c = _sums(o, ilp)
    assert np.max(np.abs(s - c), initial=0.0) <= 1e-12 * max(1.0, float(np.max(np.abs(c), initial=0.0)))


def test_example_a_certified_bound_is_the_optimum_in_both_forms():
    for mode in (0, 1):
        o = O.Oracle(example_a()[0])
        o.init()
        o.run_dual(3)
        o.set_termination(mode)
        assert o.lb_cert()[0] == -5.0


def test_forms_coincide_for_single_subproblem_variables():
    """|J_i| = 1 everywhere: (omega/1) * M is omega * M, so both forms agree bit for bit"""
    rows = [([0, 1, 2], [1, 1, 1], -1, 1), ([3, 4], [2, -1], 1, 0)]
    ilp = I.from_rows(5, [-1.0, 0.5, -2.0, 1.0, -1.5], rows)
    a, b = O.Oracle(ilp), O.Oracle(ilp)
    for o, mode in ((a, 0), (b, 1)):
        o.init()
        o.run_dual(2)
        o.set_termination(mode)
    assert a.lb_cert() == b.lb_cert()
    a.terminate()
    b.terminate()
    assert np.array_equal(a.get()[0], b.get()[0])


def test_forms_coincide_without_deferred_differences():
    """after serial averaging M-bar = 0, and both forms return lambda itself"""
    ilp = I.mrf_grid(3, 4, 3, pairwise="potts", seed=8)
    a, b = O.Oracle(ilp), O.Oracle(ilp)
    for o, mode in ((a, 0), (b, 1)):
        o.init()
        o.run_serial(2)
        o.set_termination(mode)
        o.terminate()
    assert np.array_equal(a.get()[0], b.get()[0])

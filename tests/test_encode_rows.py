"""Encoding of rows whose BDDs would be too wide (bddmma_encode_rows, host only).

A row sum_i a_i x_i (sense) b is replaced by rows over new variables: the
complement of every variable with a negative coefficient, the bits of the
weighted sum produced column by column by a binary adder, and one comparison
of that binary number with b.  Every new row has small coefficients, so its
BDD stays narrow (Sec. 2 builds one BDD per row; its width is the number of
distinct partial sums, which the adder keeps small).

Pins, none of which uses the encoder's arithmetic: for every assignment of
the original variables, the encoded rows have a completion exactly when the
original row holds, and then exactly one (a generic propagation search over
the encoded rows); rows with few partial sums are copied unchanged; the
optimum of a small encoded ILP equals the enumerated optimum of the original.
"""
import itertools

import numpy as np
import pytest

import brute
from paper_2111_10270_amd import binding as B
from paper_2111_10270_amd import instances as I


def wide_row_ilp(n, seed, sense, lo=-2000, hi=2000):
    rng = np.random.default_rng(seed)
    a = rng.integers(lo, hi, n)
    a[a == 0] = 1
    b = int(a @ rng.integers(0, 2, n))   # a point on the boundary: an rhs off by one fails
    return I.from_rows(n, rng.normal(size=n), [(list(range(n)), [int(v) for v in a], sense, b)], name=f"wide{n}_{seed}")


def same_ilp(a, b):
    return (a.n_vars == b.n_vars and a.n_rows == b.n_rows and np.array_equal(a.costs, b.costs)
            and np.array_equal(a.row_ptr, b.row_ptr) and np.array_equal(a.col, b.col)
            and np.array_equal(a.coef, b.coef) and np.array_equal(a.sense, b.sense) and np.array_equal(a.rhs, b.rhs))


@pytest.mark.parametrize("sense", [-1, 0, 1])
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_each_assignment_has_one_completion_iff_row_holds(sense, seed):
    il = wide_row_ilp(7, 100 * seed + sense + 1, sense)
    enc, ne = B.encode_rows(il, max_states=16)
    assert ne == 1 and enc.meta["n_original_vars"] == il.n_vars
    assert np.array_equal(enc.costs[:il.n_vars], il.costs) and not np.any(enc.costs[il.n_vars:])
    assert B.Solver(enc).stats.max_width <= 64    # every encoded row has a narrow BDD
    holds = 0
    for x in itertools.product((0, 1), repeat=il.n_vars):
        ok = brute.check_rows(il, x) == 0
        holds += ok
        fixed = list(x) + [-1] * (enc.n_vars - il.n_vars)
        assert brute.completions(enc, fixed) == int(ok), (x, ok)
    assert holds > 0


def test_narrow_rows_unchanged():
    il = I.random_ilp(30, 20, max_row_len=6, seed=5)
    enc, ne = B.encode_rows(il)
    assert ne == 0 and same_ilp(enc, il)
    # a long row with small coefficients has few partial sums: kept too
    n = 300
    il = I.from_rows(n, np.ones(n), [(list(range(n)), [1] * n, -1, 40)])
    enc, ne = B.encode_rows(il)
    assert ne == 0 and same_ilp(enc, il)


def test_only_wide_rows_encoded_and_optimum_kept():
    rng = np.random.default_rng(9)
    n = 9
    rows = [([0, 1, 2], [1, 1, 1], -1, 1),
            (list(range(n)), [int(v) for v in rng.integers(100, 3000, n)], -1, 6000),
            ([3, 4, 5, 6], [2, -1, 1, 1], 1, 1),
            ([2, 5, 7, 8], [int(v) for v in rng.integers(-5000, 5000, 4)], 1, -300)]
    il = I.from_rows(n, rng.normal(size=n), rows)
    enc, ne = B.encode_rows(il, max_states=64)
    assert ne == 1                                  # the 4-variable row has only 16 points
    assert enc.n_rows > il.n_rows
    opt, _ = brute.ilp_opt(il)
    # the optimum of the encoded ILP: enumerate the original variables and
    # complete each point (the new variables cost nothing)
    best = None
    for x in itertools.product((0, 1), repeat=n):
        if brute.completions(enc, list(x) + [-1] * (enc.n_vars - n), limit=1):
            v = sum(float(c) for c, xi in zip(il.costs, x) if xi)
            best = v if best is None else min(best, v)
    assert best is not None and abs(best - float(opt)) <= 1e-12 * max(1.0, abs(float(opt)))


def test_encoded_knapsack_loads_where_the_row_does_not():
    rng = np.random.default_rng(1)
    n = 200
    a = rng.integers(-10**6, 10**6, n)
    il = I.from_rows(n, rng.normal(size=n), [(list(range(n)), [int(v) for v in a], -1, int(np.abs(a).sum() // 4))])
    with pytest.raises(B.BddmmaError) as e:
        B.Solver(il)
    assert "wider" in str(e.value)
    enc, ne = B.encode_rows(il)
    assert ne == 1
    st = B.Solver(enc).stats
    assert st.n_vars == enc.n_vars and st.max_width <= 256


def test_encoding_errors():
    il = wide_row_ilp(5, 1, -1)
    with pytest.raises(B.BddmmaError):
        B.encode_rows(il, max_states=1)
    n = 40
    il = I.from_rows(n, np.ones(n), [(list(range(n)), [1 << 25] * n, -1, 1 << 26)])
    with pytest.raises(B.BddmmaError) as e:       # weight sum beyond 2^30
        B.encode_rows(il)
    assert "too large" in str(e.value)

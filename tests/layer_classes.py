"""An ILP whose BDDs cover many register-kernel classes: groups of >= 16 rows
with one topology (shared tiles) for many lengths at widths 2 and 4, and rows
of scattered topologies (mixed tiles) with lengths 1..22.  No method
arithmetic: rows and costs only."""
import numpy as np

from paper_2111_10270_amd import instances as I


def layer_class_ilp(seed: int = 5, n_vars: int = 400) -> I.ILP:
    rng = np.random.default_rng(seed)
    rows = []
    # shared groups, width 2: at most one of K variables
    for k in (2, 3, 5, 8, 9, 12, 13, 16, 17, 21, 24):
        for _ in range(20):
            vs = rng.choice(n_vars, size=k, replace=False)
            rows.append((vs, [1] * k, -1, 1))
    # shared groups, width 4: at most three of K variables
    for k in (4, 6, 10, 16, 18):
        for _ in range(18):
            vs = rng.choice(n_vars, size=k, replace=False)
            rows.append((vs, [1] * k, -1, 3))
    # scattered topologies (width <= 2): sum of K-1 variables <= one more
    # variable, whose position in the variable order varies
    for _ in range(150):
        k = int(rng.integers(1, 23))
        vs = rng.choice(n_vars, size=k, replace=False)
        a = [1] * k
        a[int(rng.integers(0, k))] = -1
        rows.append((vs, a, -1, 0))
    return I.from_rows(n_vars, rng.standard_normal(n_vars), rows, name=f"classes{seed}")

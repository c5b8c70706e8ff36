"""Autotuner of the launch schedule (bddmma_autotune): the options it picks
only choose kernels and layouts, so a solver built with them follows the
default solver's trajectory (FP64 multipliers bit for bit, bounds to 1e-12:
their per-tile partial sums follow the tile order)."""
import sys

import numpy as np
import pytest

from paper_2111_10270_amd import binding as B
from paper_2111_10270_amd import instances as I

pytestmark = pytest.mark.gpu
KEYS = ("fast_path", "small_tiles", "class_merge_kib", "sp_in_lds_max_nodes", "wide_min_width", "wide_lanes",
        "graph_sweeps")


def knapsack_rows(seed=23, n=300, rows=80):
    """rows with coefficients up to 20: layers of tens of nodes, the wide
    kernel's candidates"""
    rng = np.random.default_rng(seed)
    rs = []
    for _ in range(rows):
        k = int(rng.integers(8, 15))
        vs = rng.choice(n, size=k, replace=False)
        a = rng.integers(1, 21, size=k)
        rs.append((vs, a, -1, int(a.sum() // 2)))
    return I.from_rows(n, rng.standard_normal(n), rs, name="knapsack_rows")


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    assert torch.cuda.get_device_properties(0).gcnArchName.startswith("gfx950")


@pytest.mark.parametrize("k", range(4))
def test_autotuned_options_keep_the_trajectory(k):
    ilp = [I.graph_matching(n_left=150, n_right=150, k=10, n_pairs=150, seed=3),
           I.cell_tracking(frames=6, dets=80, seed=4), I.random_ilp(80, 60, max_row_len=8, seed=5),
           knapsack_rows()][k]
    print("autotune", ilp.name, flush=True)
    best, us = B.autotune(ilp, sweeps=16, precision=64)
    assert us > 0 and np.isfinite(us)
    assert best.precision == 64 and best.omega == 0.5
    picked = {key: getattr(best, key) for key in KEYS}
    print("picked", picked, "us/sweep", us, flush=True)
    a = B.Solver(ilp, precision=64).bind()
    b = B.Solver(ilp, precision=64, **picked).bind()
    a.run_dual(12)
    b.run_dual(12)
    la, ma = a.multipliers()
    lb, mb = b.multipliers()
    assert np.array_equal(la, lb) and np.array_equal(ma, mb)
    ha, hb = a.lb_history(), b.lb_history()
    assert np.max(np.abs(ha - hb) / np.maximum(1.0, np.abs(ha))) <= 1e-12

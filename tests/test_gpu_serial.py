"""Serial min-marginal averaging on the GPU (level-scheduled) against the
reference implementation's serial sweeps: FP64 multipliers bit for bit and
bounds to 1e-12, FP32 within the scaled tolerance; the state afterwards (M-bar
= 0) continues with the deferred scheme exactly as the reference does."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2111_10270_amd import binding as B
from paper_2111_10270_amd import instances as I
from test_oracle import example_b

pytestmark = pytest.mark.gpu


def note(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    assert torch.cuda.get_device_properties(0).gcnArchName.startswith("gfx950")


def cases():
    out = [example_b(), I.random_ilp(30, 24, max_row_len=6, seed=901), I.random_ilp(60, 50, max_row_len=9, seed=902),
           I.mrf_grid(6, 7, 3, pairwise="potts", seed=4), I.mrf_grid(5, 5, 8, pairwise="trunc_linear", seed=5),
           I.graph_matching(n_left=40, n_right=40, k=6, n_pairs=40, seed=6),
           I.cell_tracking(frames=4, dets=30, conflicts_per_frame=8, seed=7)]
    return [p for p in out if O.Oracle(p).status == O.OK]


def lam_pairs(s):
    lam, mm, _ = s.get_state()
    return lam, mm


@pytest.mark.parametrize("k", range(7))
def test_serial_matches_reference_fp64(k):
    ps = cases()
    if k >= len(ps):
        pytest.skip("case filtered out")
    ilp = ps[k]
    note("serial fp64", ilp.name, ilp.n_vars)
    s = B.Solver(ilp, precision=64, serial_mma=1).bind()
    o = O.Oracle(ilp)
    o.init()
    s.run_dual(3)
    o.run_dual(3)
    lb = s.run_serial(4)
    lo = o.run_serial(4)
    lam, mm = lam_pairs(s)
    ol, om, _ = o.get()
    assert np.array_equal(lam, ol)
    assert np.all(mm == 0.0) and np.all(om == 0.0)
    assert np.max(np.abs(lb - lo) / np.maximum(1.0, np.abs(lo))) <= 1e-12
    assert np.array_equal(s.lb_history()[-8:], lb)
    f, c, r = s.lower_bound()
    oc, orr = o.lb_cert()
    assert f == lb[-1]
    assert abs(c - oc) <= 1e-12 * max(1.0, abs(oc)) and abs(r - orr) <= 1e-12 * max(1.0, abs(orr))
    # the deferred scheme continues from the serial point (M-bar = 0) identically
    s.run_dual(2)
    o.run_dual(2)
    lam2, mm2 = lam_pairs(s)
    ol2, om2, _ = o.get()
    assert np.array_equal(lam2, ol2) and np.array_equal(mm2, om2)


def test_serial_fp32_within_tolerance():
    for ilp in cases()[1:]:
        s = B.Solver(ilp, precision=32, serial_mma=1).bind()
        o = O.Oracle(ilp)
        o.init()
        lb = s.run_serial(6)
        lo = o.run_serial(6)
        sc = max(1e-12, float(np.mean(np.abs(ilp.costs))))
        assert np.all(np.abs(lb - lo) <= 1e-4 * np.maximum(np.abs(lo), sc * ilp.n_vars)), ilp.name
        lam, _ = lam_pairs(s)
        ol, _, _ = o.get()
        assert np.all(np.abs(lam - ol) <= 1e-4 * np.maximum(np.abs(ol), sc)), ilp.name


def test_serial_needs_its_tables():
    s = B.Solver(I.random_ilp(10, 8, seed=3)).bind()
    with pytest.raises(B.BddmmaError) as e:
        s.run_serial(1)
    assert e.value.code == B.STATE

"""bddmma_bind_static: the solver bound to the library's static device
workspace (no allocation by the caller or the library) gives exactly the
results of the same solver bound to caller memory with bddmma_bind, on two
binds in a row, the second with a smaller problem; the first solver loses the
array to the second."""
import numpy as np
import pytest

import brute
from paper_2111_10270_amd import binding as B
from paper_2111_10270_amd import instances as I

pytestmark = pytest.mark.gpu


def note(*a):
    print(*a, flush=True)


def solve(s, iters):
    s.run_dual(iters)
    lam, mm, avg = s.get_state()
    return dict(lam=lam, mm=mm, avg=avg, hist=s.lb_history(), bounds=np.array(s.lower_bound()),
                round=s.round_primal())


def same(a, b):
    for k in ("lam", "mm", "avg", "hist", "bounds"):
        assert np.array_equal(a[k], b[k]), k
    ra, rb = a["round"], b["round"]
    assert ra["rc"] == rb["rc"] and ra["rounds"] == rb["rounds"]
    if ra["rc"] == 0:
        assert np.array_equal(ra["x"], rb["x"]) and ra["ub"] == rb["ub"]


def test_bind_static_matches_bind():
    cases = [("track20x500", 32, 64, 40), ("mrf10x10L3", 64, 0, 25)]
    held = []
    for name, prec, graph, iters in cases:
        ilp = I.workload(name)
        note("bind_static", name, "precision", prec, "graph_sweeps", graph)
        ref = B.Solver(ilp, precision=prec, graph_sweeps=graph)
        assert ref.workspace_bytes() <= B.STATIC_WORKSPACE_BYTES
        ref.bind("cuda:0")
        want = solve(ref, iters)
        ref = None
        st = B.Solver(ilp, precision=prec, graph_sweeps=graph).bind_static("cuda:0")
        assert st.workspace is None
        got = solve(st, iters)
        same(got, want)
        if want["round"]["rc"] == 0:
            assert brute.check_rows(ilp, got["round"]["x"]) == 0   # exact integer row check
        # a reset and a second solve on the same static workspace repeat it
        st.reset()
        same(solve(st, iters), want)
        held.append(st)
    # the array now belongs to the second solver: the first one is refused
    with pytest.raises(B.BddmmaError) as e:
        held[0].run_dual(1)
    assert e.value.code == B.STATE
    held[1].run_dual(1)

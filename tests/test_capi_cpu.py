"""C ABI checks that need no GPU: exports, options, validation, presolve and
pair bookkeeping against the reference implementation (index work: bit-exact)."""
import os
import re

import numpy as np
import pytest

import oracle as O
from paper_2111_10270_amd import binding as B
from paper_2111_10270_amd import instances as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "bddmma.h")).read()
    declared = set(re.findall(r"\b(bddmma_[a-z_]+)\s*\(", hdr))
    assert declared == set(B.EXPORTS)
    L = B.lib()
    for name in declared:
        assert hasattr(L, name), name


def test_default_options():
    o = B.default_options()
    assert (o.omega, o.precision, o.delta0, o.alpha, o.reopt_iters, o.max_rounds) == (0.5, 32, 1.0, 1.2, 5, 200)
    assert o.lb_every == 1 and o.rel_tol == 0.0 and o.tau < 0
    assert (o.fast_path, o.perturb_scale, o.sp_in_lds_max_nodes, o.graph_sweeps) == (1, 0, 0, 64)
    assert o.class_merge_kib == 32768 and o.small_tiles == 2048 and o.serial_mma == 0 and o.termination == 0
    assert o.wide_min_width == 4 and o.wide_lanes == 32 and o.fused_average == 1 and o.persistent == 0
    assert o.reserved == 0


@pytest.mark.parametrize("bad", [dict(omega=0.0), dict(omega=1.5), dict(precision=16), dict(lb_every=0),
                                 dict(alpha=0.5), dict(delta0=0.0), dict(max_rounds=-1),
                                 dict(sp_in_lds_max_nodes=-2), dict(fast_path=2), dict(perturb_scale=2),
                                 dict(graph_sweeps=-1), dict(class_merge_kib=-1), dict(small_tiles=-1),
                                 dict(serial_mma=2), dict(termination=2), dict(wide_min_width=-1),
                                 dict(wide_min_width=65536), dict(wide_lanes=8), dict(wide_lanes=48),
                                 dict(fused_average=2), dict(persistent=2), dict(reserved=1)])
def test_invalid_options(bad):
    ilp = I.random_ilp(5, 3, seed=1)
    with pytest.raises(B.BddmmaError) as e:
        B.Solver(ilp, **bad)
    assert e.value.code == B.INVALID_ARG


def test_wide_kernel_threshold_moves_tiles():
    """wide_min_width decides which tiles outside the register classes run one
    BDD per wave: 0 none, and a lower threshold takes at least the tiles a
    higher one does"""
    rng = np.random.default_rng(23)
    n = 300
    rows = []
    for _ in range(80):
        k = int(rng.integers(8, 15))
        vs = rng.choice(n, size=k, replace=False)
        a = rng.integers(1, 21, size=k)
        rows.append((vs, a, -1, int(a.sum() // 2)))
    ilp = I.from_rows(n, rng.standard_normal(n), rows)
    counts = {w: B.Solver(ilp, wide_min_width=w).stats.n_wide_tiles for w in (0, 4, 16, 64, 65535)}
    assert counts[0] == 0 and counts[65535] == 0
    assert counts[4] >= counts[16] >= counts[64] and counts[16] > 0


def _raw(ilp, **kw):
    d = dict(n_vars=ilp.n_vars, costs=ilp.costs, row_ptr=ilp.row_ptr, col=ilp.col, coef=ilp.coef,
             sense=ilp.sense, rhs=ilp.rhs)
    d.update(kw)
    return I.ILP(**d)


def test_invalid_ilp_data():
    good = I.from_rows(3, [1.0, 2.0, 3.0], [([0, 1], [1, 1], -1, 1), ([1, 2], [1, -1], 0, 0)])
    for bad in (_raw(good, col=np.array([0, 3, 1, 2], dtype=np.int32)),
                _raw(good, col=np.array([0, 0, 1, 2], dtype=np.int32)),
                _raw(good, sense=np.array([2, 0], dtype=np.int8)),
                _raw(good, costs=np.array([1.0, np.nan, 3.0])),
                _raw(good, costs=np.array([1.0, np.inf, 3.0])),
                _raw(good, row_ptr=np.array([0, 3, 2], dtype=np.int64))):
        with pytest.raises(B.BddmmaError) as e:
            B.Solver(bad)
        assert e.value.code == B.INVALID_ARG


def test_infeasible_rows():
    for rows in ([([0, 1], [1, 1], 1, 3)],                      # x + y >= 3
                 [([0, 1], [2, 2], 0, 1)],                      # 2x + 2y = 1
                 [([0], [1], 0, 1), ([0, 1], [1, 1], -1, 0)]):  # x = 1 and x + y <= 0
        ilp = I.from_rows(2, [1.0, 1.0], rows)
        assert O.Oracle(ilp).status == O.INFEASIBLE
        with pytest.raises(B.BddmmaError) as e:
            B.Solver(ilp)
        assert e.value.code == B.INFEASIBLE


def test_call_order_is_checked():
    s = B.Solver(I.random_ilp(6, 3, seed=2))
    for f in (lambda: s.run_dual(1), lambda: s.lower_bound(), lambda: s.get_state(), lambda: s.reset()):
        with pytest.raises(B.BddmmaError) as e:
            f()
        assert e.value.code == B.STATE
    assert s.workspace_bytes() > 0


def _same_structure(ilp):
    s = B.Solver(ilp)
    o = O.Oracle(ilp)
    assert o.status == O.OK
    pv, pr = s.pairs()
    opv, opr = o.pairs()
    assert np.array_equal(pv, opv) and np.array_equal(pr, opr)
    assert np.array_equal(s.fixed(), o.fixed())
    st = s.stats
    assert (st.n_bdds, st.n_pairs) == (o.n_bdds, o.n_pairs)
    assert st.n_nodes <= o.n_nodes               # reduced BDDs are never larger
    assert st.lb_offset == o.lb_offset()
    assert st.n_slots >= st.n_pairs and st.n_slots % 64 == 0
    return s, o


@pytest.mark.parametrize("seed", range(30))
def test_presolve_and_pairs_match_reference(seed):
    ilp = I.random_ilp(12, 9, max_row_len=6, seed=4000 + seed)
    if O.Oracle(ilp).status == O.INFEASIBLE:
        with pytest.raises(B.BddmmaError):
            B.Solver(ilp)
        return
    _same_structure(ilp)


@pytest.mark.parametrize("name", ["mrf10x10L3", "gm1000k10", "track20x500"])
def test_workload_structure_matches_reference(name):
    s, o = _same_structure(I.workload(name))
    if name == "mrf10x10L3":
        assert (s.stats.n_bdds, s.stats.n_pairs, s.stats.n_nodes) == (1180, 4620, 8060)


def test_reduction_merges_equivalent_nodes():
    # x1 + ... + x6 <= 5: every partial sum <= 1 after 4 variables behaves alike
    ilp = I.from_rows(6, np.ones(6), [(list(range(6)), [1] * 6, -1, 5)])
    s = B.Solver(ilp)
    o = O.Oracle(ilp)
    assert s.stats.n_nodes < o.n_nodes


def test_empty_and_free_variables():
    ilp = I.from_rows(4, [1.0, -2.0, 0.5, -1.0], [])
    s = B.Solver(ilp)
    st = s.stats
    assert (st.n_bdds, st.n_pairs, st.n_free, st.n_tiles) == (0, 0, 4, 0)
    assert st.lb_offset == -3.0


def test_register_path_tile_counts():
    from layer_classes import layer_class_ilp
    st = B.Solver(I.workload("mrf10x10L3"), small_tiles=0).stats
    assert st.n_reg_tiles == st.n_tiles and st.n_reg_mixed_tiles == 0
    st = B.Solver(I.workload("mrf10x10L3")).stats       # small problem: all tiles run as mixed tiles
    assert st.n_reg_mixed_tiles == st.n_tiles and st.n_reg_tiles == 0 and st.n_reg_launches == 1
    merged = B.Solver(layer_class_ilp(), small_tiles=0).stats          # classes merge (padding)
    st = B.Solver(layer_class_ilp(), class_merge_kib=0, small_tiles=0).stats
    assert st.n_reg_tiles > 0 and st.n_reg_mixed_tiles > 0 and st.n_reg_launches >= 12
    assert st.n_reg_tiles + st.n_reg_mixed_tiles < st.n_tiles   # wide or long rows stay general
    assert merged.n_reg_launches < st.n_reg_launches and merged.n_slots > st.n_slots
    assert merged.n_reg_tiles == st.n_reg_tiles and merged.n_reg_mixed_tiles == st.n_reg_mixed_tiles
    st = B.Solver(layer_class_ilp(), fast_path=0).stats
    assert st.n_reg_tiles == st.n_reg_mixed_tiles == st.n_reg_launches == 0


# ---------------------------------------------------------------- batches
def _batch_members():
    return [I.random_ilp(14, 10, max_row_len=6, seed=4100), I.mrf_grid(4, 5, 3, pairwise="potts", seed=3),
            I.random_ilp(30, 24, max_row_len=7, seed=4102), I.from_rows(3, [1.0, -1.0, 0.5], [])]


def test_batch_structure_is_the_union_of_instances():
    ilps = [p for p in _batch_members() if O.Oracle(p).status == O.OK]
    b = B.Solver(ilps)
    alone = [B.Solver(p) for p in ilps]
    assert b.n_inst == len(ilps) and all(a.n_inst == 1 for a in alone)
    st = b.stats
    for f in ("n_bdds", "n_pairs", "n_nodes", "n_fixed", "n_free", "n_tiles"):
        assert getattr(st, f) == sum(getattr(a.stats, f) for a in alone), f
    assert st.lb_offset == sum(a.stats.lb_offset for a in alone)
    pv, pr = b.pairs()
    voff = np.cumsum([0] + [p.n_vars for p in ilps])
    roff = np.cumsum([0] + [p.n_rows for p in ilps])
    ref_v = np.concatenate([a.pairs()[0] + voff[k] for k, a in enumerate(alone)])
    ref_r = np.concatenate([a.pairs()[1] + roff[k] for k, a in enumerate(alone)])
    assert np.array_equal(pv, ref_v) and np.array_equal(pr, ref_r)


def test_batch_rejects_cross_instance_rows_and_bad_counts():
    a = I.from_rows(2, [1.0, 1.0], [([0, 1], [1, 1], -1, 1)])
    u = I.concat([a, a])
    bad = I.ILP(n_vars=u.n_vars, costs=u.costs, row_ptr=u.row_ptr, col=np.array([0, 1, 1, 2], dtype=np.int32),
                coef=u.coef, sense=u.sense, rhs=u.rhs, meta=u.meta)
    L = B.lib()
    import ctypes as C
    for ilp, nv, nr in ((bad, [2, 2], [1, 1]), (u, [2, 1], [1, 1]), (u, [2, 2], [2, 1])):
        h = C.c_void_p()
        assert L.bddmma_create(None, C.byref(h)) == 0
        arrs = [np.ascontiguousarray(x) for x in (ilp.costs, ilp.row_ptr, ilp.col, ilp.coef, ilp.sense, ilp.rhs)]
        nva, nra = np.array(nv, dtype=np.int64), np.array(nr, dtype=np.int64)
        rc = L.bddmma_load_batch(h, len(nv), B._p(nva), B._p(nra), ilp.n_vars, B._p(arrs[0]), ilp.n_rows,
                                 *[B._p(x) for x in arrs[1:]])
        assert rc == B.INVALID_ARG
        L.bddmma_destroy(h)


def test_batch_with_an_infeasible_instance():
    good = I.from_rows(2, [1.0, 1.0], [([0, 1], [1, 1], -1, 1)])
    infeasible = I.from_rows(2, [1.0, 1.0], [([0, 1], [1, 1], 1, 3)])
    with pytest.raises(B.BddmmaError) as e:
        B.Solver([good, infeasible])
    assert e.value.code == B.INFEASIBLE


def test_pool_host_side_states_and_validation():
    """serving pool without a device: option and argument checks, host
    compilation into READY / FAILED, sizes, and which tickets can be released"""
    with pytest.raises(B.BddmmaError) as e:
        B.Pool(max_active=0)
    assert e.value.code == B.INVALID_ARG
    with pytest.raises(B.BddmmaError) as e:
        B.Pool(omega=2.0)
    assert e.value.code == B.INVALID_ARG
    with pytest.raises(B.BddmmaError) as e:
        B._check(B.lib().bddmma_pool_create(None, 2, 1, 4, B.C.byref(B.C.c_void_p())))   # unknown flag
    assert e.value.code == B.INVALID_ARG
    pool = B.Pool(max_active=2, host_threads=2, precision=64)
    good = I.random_ilp(12, 8, seed=3)
    with pytest.raises(B.BddmmaError) as e:
        pool.submit(good, 0)
    assert e.value.code == B.INVALID_ARG
    t_good = pool.submit(good, 10)
    t_inf = pool.submit(I.from_rows(2, [1.0, 1.0], [([0, 1], [1, 1], 0, 3)]), 10)   # x0 + x1 = 3
    bad = I.from_rows(2, [1.0, 1.0], [([0, 1], [1, 1], -1, 1)])
    bad.col = np.array([0, 5], dtype=np.int32)                                      # column out of range
    t_bad = pool.submit(bad, 10)
    t_batch = pool.submit_loaded(B.Solver([good, good], precision=64), 10)           # not a single ILP
    t_prec = pool.submit_loaded(B.Solver(good, precision=32), 10)                    # other precision
    t_own = pool.submit_loaded(B.Solver(good, precision=64), 10)
    pool.wait_compiled()
    g = pool.poll(t_good)
    s = B.Solver(good, precision=64)
    assert g["state"] == B.POOL_READY and g["n_pairs"] == s.n_pairs and g["n_vars"] == good.n_vars
    assert g["workspace_bytes"] == s.workspace_bytes() and g["iters"] == 0 and np.isnan(g["lb_free"])
    assert pool.poll(t_own)["state"] == B.POOL_READY
    assert (pool.poll(t_inf)["state"], pool.poll(t_inf)["error"]) == (B.POOL_FAILED, B.INFEASIBLE)
    for t in (t_bad, t_batch, t_prec):
        assert (pool.poll(t)["state"], pool.poll(t)["error"]) == (B.POOL_FAILED, B.INVALID_ARG), t
    with pytest.raises(B.BddmmaError) as e:
        pool.step(5)                      # no arena bound
    assert e.value.code == B.STATE
    with pytest.raises(B.BddmmaError) as e:
        pool.release(t_good)              # waiting, not retired
    assert e.value.code == B.STATE
    with pytest.raises(B.BddmmaError) as e:
        pool.result(t_good)
    assert e.value.code == B.STATE
    pool.release(t_inf)
    with pytest.raises(B.BddmmaError) as e:
        pool.poll(t_inf)
    assert e.value.code == B.INVALID_ARG
    del pool


def test_serial_tables_cost_workspace_only_when_asked():
    ilp = I.mrf_grid(6, 6, 3, pairwise="potts", seed=1)
    a, b = B.Solver(ilp), B.Solver(ilp, serial_mma=1)
    assert b.workspace_bytes() > a.workspace_bytes()
    st = b.stats
    # node words, two distance arrays, per-pair tables: at least 4 B per node and 16 B per pair more
    assert b.workspace_bytes() - a.workspace_bytes() >= 4 * st.n_nodes + 16 * st.n_pairs


def test_one_topology_tiles_share_their_node_words():
    """grid MRFs repeat a handful of row shapes: the device keeps one copy of
    the node words per shape, orders of magnitude fewer words than nodes"""
    st = B.Solver(I.mrf_grid(48, 48, 8, pairwise="trunc_linear", seed=3), small_tiles=0).stats
    assert st.n_reg_mixed_tiles == 0
    assert st.node_words * 1000 < st.n_nodes
    # per-lane layouts (mixed tiles of a small problem) hold a word per node and lane
    small = B.Solver(I.graph_matching(n_left=100, n_right=100, k=10, n_pairs=100, seed=2)).stats
    assert small.node_words >= small.n_nodes


def test_bind_static_rejects_problems_above_its_size():
    """the static workspace (64 MiB) refuses a larger problem before any
    device call, so this runs without a GPU"""
    s = B.Solver(I.mrf_grid(64, 64, 8, pairwise="trunc_linear", trunc=2, seed=2), precision=64)
    assert s.workspace_bytes() > B.STATIC_WORKSPACE_BYTES
    rc = B.lib().bddmma_bind_static(s._h, None)
    assert rc == B.NO_MEMORY
    msg = B.lib().bddmma_last_error().decode()
    assert "static workspace" in msg and str(B.STATIC_WORKSPACE_BYTES) in msg
    # and a solver with nothing loaded is refused as out of order
    t = B.lib()
    h = __import__("ctypes").c_void_p()
    assert t.bddmma_create(None, __import__("ctypes").byref(h)) == B.OK
    assert t.bddmma_bind_static(h, None) == B.STATE
    t.bddmma_destroy(h)


@pytest.mark.parametrize("name,fused", [("mrf10x10L3", True), ("gm1000k10", False), ("track20x500", False),
                                        ("mrf256x256L8", False)])
def test_fused_averaging_eligibility(name, fused):
    """the sweep averages the variables that span tiles itself when all of
    them lie in mixed register tiles (small problems) in at most five
    subproblems each; the matching and tracking workloads have variables in
    up to 10 and 8 subproblems, the large grid's tiles share one topology: they
    keep the averaging kernel; the option turns it off and the extra device
    tables go with it"""
    ilp = I.workload(name)
    on = B.Solver(ilp)
    off = B.Solver(ilp, fused_average=0)
    assert (on.stats.n_fused_vars > 0) == fused
    assert off.stats.n_fused_vars == 0
    assert (on.workspace_bytes() > off.workspace_bytes()) == fused


def test_stream_probe_rejects_bad_arguments():
    """the bandwidth probe validates its arguments before any device call"""
    t = B.lib()
    assert t.bddmma_stream_probe(None, None, -1, 4, None) == B.INVALID_ARG
    assert t.bddmma_stream_probe(None, None, 10, 2, None) == B.INVALID_ARG
    assert "elem_bytes" in t.bddmma_last_error().decode()
    assert t.bddmma_stream_probe(None, None, 10, 4, None) == B.INVALID_ARG
    assert "NULL" in t.bddmma_last_error().decode()
    assert t.bddmma_stream_probe(None, None, 0, 8, None) == B.OK

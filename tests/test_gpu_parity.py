"""Parity of the HIP path with the FP64 reference implementation (needs a GPU).

FP64 mode performs the same operations in the same order as the reference
(min is exact, the only sums are in fixed order), so multipliers, min-marginal
differences and averaged terms must agree bit for bit; bound sums use a
different association and agree to 1e-12.  FP32 mode is checked with the
scaled tolerance |d| <= 1e-4 * max(|ref|, mean|c|).
"""
import os
import sys

import numpy as np
import pytest

import brute
import oracle as O
from paper_2111_10270_amd import binding as B
from paper_2111_10270_amd import instances as I
from test_oracle import example_a, example_b, tie_example

pytestmark = pytest.mark.gpu


def note(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    assert torch.cuda.get_device_properties(0).gcnArchName.startswith("gfx950")


def solver(ilp, **kw):
    s = B.Solver(ilp, **kw)
    return s.bind()


def scale_of(ilp):
    return max(1e-12, float(np.mean(np.abs(ilp.costs)))) if ilp.n_vars else 1.0


def fp32_close(got, ref, s, tol=1e-4):
    got, ref = np.asarray(got), np.asarray(ref)
    bound = tol * np.maximum(np.abs(ref), s)
    return bool(np.all(np.abs(got - ref) <= bound)), float(np.max(np.abs(got - ref) / np.maximum(np.abs(ref), s), initial=0))


def lockstep(ilp, sweeps, precision=64, **kw):
    """run the GPU and the reference sweep by sweep and compare after each"""
    note("lockstep", ilp.name, sweeps, precision, kw)
    s = solver(ilp, precision=precision, **kw)
    o = O.Oracle(ilp)
    o.init()
    sc = scale_of(ilp)
    worst = 0.0
    for k in range(sweeps):
        s.run_sweeps(1)
        o.sweep(k % 2)
        o.average()
        lam, mm, avg = s.get_state()
        rl, rm, ra = o.get()
        lbf = s.lb_history()[-1]
        if precision == 64:
            assert np.array_equal(lam, rl), k
            assert np.array_equal(mm, rm), k
            assert np.array_equal(avg, ra), k
            assert abs(lbf - o.lb_free()) <= 1e-12 * max(1.0, abs(o.lb_free())), k
        else:
            for g, r in ((lam, rl), (mm, rm), (avg, ra)):
                ok, err = fp32_close(g, r, sc)
                worst = max(worst, err)
                assert ok, (k, err)
            assert abs(lbf - o.lb_free()) <= 1e-4 * max(abs(o.lb_free()), sc * max(1, o.n_bdds)), k
    lf, lc, res = s.lower_bound()
    rc_, rres = o.lb_cert()
    tol = 1e-12 if precision == 64 else 1e-4
    assert abs(lc - rc_) <= tol * max(1.0, abs(rc_)), (lc, rc_)
    return s, o, worst


# ---------------------------------------------------------------- paper examples
def test_paper_examples_fp64_bitexact():
    ilp, _ = example_a()
    s, o, _ = lockstep(ilp, 8)
    # the first sweep of the Fig. 2 example, derived by hand from the update rule
    s2 = solver(ilp, precision=64)
    s2.run_sweeps(1)
    lam, mm, _ = s2.get_state()
    assert list(mm) == [-5, 0.5, 2, 3.5, 5, 1.75] and list(lam) == [-2.5, 0.25, 1, -1.25, -0.5, 2.125]
    assert s2.lb_history()[-1] == -5.0
    lockstep(example_b(), 12)
    lockstep(tie_example(), 4)


def test_fig3_min_marginals():
    ilp = I.from_rows(4, [2.0, 3.0, 1.0, 4.0], [([0, 1, 2, 3], [1, -1, -1, 1], 0, 0)])
    for prec in (32, 64):
        s = solver(ilp, precision=prec)
        assert list(s.min_marginals()) == [3.0, 5.0, 3.0, 5.0]
        assert s.lower_bound()[1] == 0.0


# ---------------------------------------------------------------- random instances
# register kernels (small problems: per-lane topologies only), register kernels
# with one-topology tiles, general kernels with LDS, general kernels with
# device scratch
PATHS = [dict(fast_path=1), dict(fast_path=1, small_tiles=0), dict(fast_path=0),
         dict(fast_path=0, sp_in_lds_max_nodes=-1)]


@pytest.mark.parametrize("path", PATHS)
def test_random_fp64_bitexact(path):
    for seed in range(12):
        ilp = I.random_ilp(14, 10, max_row_len=7, seed=6000 + seed)
        if O.Oracle(ilp).status != O.OK:
            continue
        lockstep(ilp, 10, precision=64, **path)


@pytest.mark.parametrize("path", PATHS)
def test_random_fp32(path):
    for seed in range(12):
        ilp = I.random_ilp(14, 10, max_row_len=7, seed=7000 + seed)
        if O.Oracle(ilp).status != O.OK:
            continue
        lockstep(ilp, 10, precision=32, **path)


@pytest.mark.parametrize("path", PATHS)
def test_workload_paths_agree_fp64(path):
    """the three kernel paths give bit-identical FP64 trajectories"""
    ilp = I.workload("track20x500")
    s = solver(ilp, precision=64, **path)
    ref = solver(ilp, precision=64)
    s.run_dual(6)
    ref.run_dual(6)
    for x, y in zip(s.get_state(), ref.get_state()):
        assert np.array_equal(x, y)


def test_long_and_wide_rows_fp64():
    rng = np.random.default_rng(11)
    # one 150-variable cardinality row (width 4), one knapsack row with large
    # coefficients (wide layers -> shortest paths outside LDS), plus short rows
    n = 160
    rows = [(list(range(150)), [1] * 150, -1, 3)]
    kv = list(range(140, 156))
    rows.append((kv, [int(v) for v in rng.integers(3, 40, size=16)], -1, 150))
    for r in range(40):
        vs = rng.choice(n, size=3, replace=False)
        rows.append((vs, [1, 1, 1], -1, 2))
    ilp = I.from_rows(n, rng.standard_normal(n), rows, name="long_wide")
    s, o, _ = lockstep(ilp, 6, precision=64)
    assert s.stats.max_layers >= 150 and s.stats.max_width > 8


@pytest.mark.parametrize("prec", [64, 32])
def test_encoded_wide_rows(prec):
    """an ILP whose knapsack rows are rewritten into binary adders
    (encode_rows): sweep-by-sweep parity with the reference on the encoded
    rows, certified bound below the enumerated optimum of the original ILP,
    and a rounded point that satisfies the original rows"""
    rng = np.random.default_rng(31)
    n = 12
    rows = [(list(range(n)), [int(v) for v in rng.integers(200, 5000, n)], -1, 12000),
            ([1, 4, 7, 9, 10], [int(v) for v in rng.integers(-3000, 3000, 5)], 1, -500)]
    for r in range(6):
        rows.append((rng.choice(n, size=3, replace=False), [1, 1, 1], -1, 1))
    ilp = I.from_rows(n, rng.standard_normal(n) - 0.5, rows, name="knap12")
    enc, ne = B.encode_rows(ilp, max_states=24)
    assert ne == 2
    note("encoded", enc.n_vars, "vars", enc.n_rows, "rows")
    s, o, _ = lockstep(enc, 8, precision=prec)
    s.run_dual(200)
    opt, _ = brute.ilp_opt(ilp)
    lb = s.lower_bound()[1]
    assert lb <= float(opt) + 1e-9 * max(1.0, abs(float(opt))), (lb, opt)
    r = s.round_primal()
    if r["rc"] == 0:
        assert brute.check_rows(ilp, r["x"][:n]) == 0
        assert brute.check_rows(enc, r["x"]) == 0


@pytest.mark.parametrize("prec", [64, 32])
@pytest.mark.parametrize("merge", [0, 32768])
def test_layer_classes(prec, merge):
    """many register classes (shared at widths 2 and 4, mixed), class merging
    with padding, and general tiles, against the reference sweep by sweep"""
    from layer_classes import layer_class_ilp
    ilp = layer_class_ilp()
    s, o, _ = lockstep(ilp, 6, precision=prec, class_merge_kib=merge, small_tiles=0)
    st = s.stats
    assert st.n_reg_tiles > 0 and st.n_reg_mixed_tiles > 0
    assert st.n_reg_launches >= (12 if merge == 0 else 2)


def wide_ilp(seed=23):
    """knapsack rows with coefficients up to 20 (layers of tens to hundreds of
    nodes): 70 rows sharing one coefficient pattern (a one-topology tile) and
    60 rows with their own patterns (mixed tiles)"""
    rng = np.random.default_rng(seed)
    n = 300
    rows = []
    pat = rng.integers(1, 21, size=12)
    for _ in range(70):
        vs = np.sort(rng.choice(n, size=12, replace=False))
        rows.append((vs, pat, -1, int(pat.sum() // 2)))
    hidden = rng.integers(0, 2, size=n)
    for _ in range(60):
        k = int(rng.integers(8, 15))
        vs = rng.choice(n, size=k, replace=False)
        a = rng.integers(1, 21, size=k) * rng.choice([-1, 1], size=k)
        sense = int(rng.integers(-1, 2))
        lhs = int(np.dot(a, hidden[vs]))
        rows.append((vs, a, sense, lhs + (3 if sense < 0 else -3 if sense > 0 else 0)))
    ilp = I.from_rows(n, rng.standard_normal(n), rows, name="wide")
    return ilp


@pytest.mark.parametrize("prec", [64, 32])
@pytest.mark.parametrize("wmin,lanes", [(16, 16), (4, 16), (4, 32), (4, 64), (0, 16)])
def test_wide_rows_node_parallel_kernel(prec, wmin, lanes):
    """BDDs with wide layers on the node-parallel kernel (LDS scatter minima),
    sweep by sweep against the reference, and the rounding's fixed-multiplier
    sweeps; the width threshold of that kernel (wide_min_width, 0 = lane per
    BDD throughout) and its lanes per BDD (several BDDs of a tile per wave)
    move tiles between schedules, never the results"""
    ilp = wide_ilp()
    if O.Oracle(ilp).status != O.OK:
        pytest.skip("generated instance infeasible")
    s, o, _ = lockstep(ilp, 6, precision=prec, wide_min_width=wmin, wide_lanes=lanes)
    if wmin == 0:
        assert s.stats.n_wide_tiles == 0
    else:
        assert s.stats.n_wide_tiles >= 2 and s.stats.max_width >= 16
    if prec == 64:
        assert np.array_equal(s.min_marginals(), o.full_mm())


@pytest.mark.parametrize("prec", [64, 32])
def test_wide_large_bdds_lane_fallback(prec):
    """BDDs of about 2,100 nodes (LDS regions of ~30 KB in FP32, ~50 KB in
    FP64): 16 lanes per BDD are asked for, four regions do not fit a block,
    so the launch takes 32 (FP32) or 64 (FP64) lanes per BDD; one tile, most
    of its lanes padding BDDs.  Sweep by sweep against the reference."""
    rng = np.random.default_rng(41)
    n = 60
    rows = []
    for _ in range(6):
        vs = rng.choice(n, size=20, replace=False)
        a = rng.integers(50, 300, size=20)
        rows.append((vs, a, -1, int(a.sum() // 2)))
    ilp = I.from_rows(n, rng.standard_normal(n), rows, name="large_wide")
    s, o, _ = lockstep(ilp, 6, precision=prec, wide_lanes=16)
    assert s.stats.n_wide_tiles == 1 and s.stats.n_nodes / s.stats.n_bdds > 1500
    if prec == 64:
        assert np.array_equal(s.min_marginals(), o.full_mm())


@pytest.mark.parametrize("prec", [64, 32])
@pytest.mark.parametrize("kw", [dict(), dict(small_tiles=0)])
def test_long_rows_chunked_kernel(prec, kw):
    """width-2 BDDs longer than every register class (assignment-type rows of a
    QAP-like instance, plus rows of scattered lengths 33..90) on the chunked
    register kernel, sweep by sweep against the reference"""
    rng = np.random.default_rng(17)
    qap = I.graph_matching(n_left=40, n_right=40, k=40, n_pairs=6, seed=7)
    n = 300
    rows = []
    for _ in range(70):
        k = int(rng.integers(33, 91))
        vs = rng.choice(n, size=k, replace=False)
        a = [1] * k
        a[int(rng.integers(0, k))] = -1
        rows.append((vs, a, -1, 0))
    mixed = I.from_rows(n, rng.standard_normal(n), rows, name="long_mixed")
    for ilp in (qap, mixed):
        s, o, _ = lockstep(ilp, 6, precision=prec, **kw)
        st = s.stats
        assert st.max_layers > 32 and st.n_reg_tiles + st.n_reg_mixed_tiles == st.n_tiles


@pytest.mark.parametrize("prec", [64, 32])
def test_very_long_rows(prec):
    """a 6,000-variable at-most-one row (width 2: the chunked register kernel,
    18,000 scratch values per lane) and a 5,000-variable cardinality row
    (width 4, too large for LDS: the general kernel with device scratch),
    linked by short rows; sweep by sweep against the reference"""
    rng = np.random.default_rng(5)
    n = 8000
    rows = [(list(range(6000)), [1] * 6000, -1, 1), (list(range(2000, 7000)), [1] * 5000, -1, 3)]
    for _ in range(300):
        rows.append((rng.choice(n, size=3, replace=False), [1, 1, -1], -1, 1))
    ilp = I.from_rows(n, rng.standard_normal(n), rows, name="very_long")
    s, o, _ = lockstep(ilp, 4, precision=prec)
    assert s.stats.max_layers == 6000 and s.stats.n_tiles > s.stats.n_reg_tiles + s.stats.n_reg_mixed_tiles


@pytest.mark.parametrize("path", PATHS[:3])
@pytest.mark.parametrize("n_rows", [1, 63, 64, 65, 130])
def test_ragged_tile_counts_fp64(n_rows, path):
    rng = np.random.default_rng(n_rows)
    rows = []
    for r in range(n_rows):
        k = int(rng.integers(1, 6))
        vs = rng.choice(40, size=k, replace=False)
        rows.append((vs, [1] * k, -1, 1))
    ilp = I.from_rows(40, rng.standard_normal(40), rows, name=f"ragged{n_rows}")
    lockstep(ilp, 4, precision=64, **path)


def test_empty_and_fixed_problems():
    ilp = I.from_rows(3, [1.0, -2.0, 0.5], [])
    s = solver(ilp, precision=32)
    s.run_dual(3)
    lf, lc, res = s.lower_bound()
    assert lf == lc == -2.0 and res == 0.0
    r = s.round_primal()
    assert r["rc"] == 0 and list(r["x"]) == [0, 1, 0] and r["ub"] == -2.0
    ilp = I.from_rows(3, [1.0, -2.0, 0.5], [([0], [1], 0, 1), ([0, 1], [1, 1], -1, 1)])   # everything fixed
    s = solver(ilp, precision=64)
    s.run_dual(2)
    assert s.lower_bound()[1] == 1.0
    r = s.round_primal()
    assert r["rc"] == 0 and list(r["x"]) == [1, 0, 0]


# ---------------------------------------------------------------- the named workloads
@pytest.mark.parametrize("path", PATHS[:3])
def test_mrf10_fp64_200_iterations(path):
    ilp = I.workload("mrf10x10L3")
    note("mrf10x10L3 fp64 200 iterations", path)
    s = solver(ilp, precision=64, **path)
    o = O.Oracle(ilp)
    o.init()
    s.run_dual(200)
    hist = o.run_dual(200)
    g = s.lb_history()
    assert g.shape == hist.shape
    assert np.max(np.abs(g - hist)) <= 1e-12 * np.max(np.abs(hist))
    lam, mm, avg = s.get_state()
    rl, rm, ra = o.get()
    assert np.array_equal(lam, rl) and np.array_equal(mm, rm) and np.array_equal(avg, ra)
    lf, lc, res = s.lower_bound()
    rc_, rres = o.lb_cert()
    assert abs(lc - rc_) <= 1e-12 * abs(rc_) and res <= 1e-12


@pytest.mark.parametrize("name", ["gm1000k10", "track20x500"])
def test_gm_tracking_fp64_500_iterations(name):
    """the matching and tracking workloads in FP64 (graph replay, the fused
    and kernel averaging as the defaults choose): multipliers, differences
    and averaged terms equal the reference's bit for bit after 500
    iterations; bound history and certified bound within 1e-12"""
    ilp = I.workload(name)
    note(name, "fp64 500 iterations")
    s = solver(ilp, precision=64)
    o = O.Oracle(ilp, threads=oracle_threads())
    o.init()
    s.run_dual(500)
    hist = o.run_dual(500)
    g = s.lb_history()
    assert g.shape == hist.shape
    assert np.max(np.abs(g - hist)) <= 1e-12 * np.max(np.abs(hist))
    lam, mm, avg = s.get_state()
    rl, rm, ra = o.get()
    assert np.array_equal(lam, rl) and np.array_equal(mm, rm) and np.array_equal(avg, ra)
    lf, lc, res = s.lower_bound()
    rc_, rres = o.lb_cert()
    assert abs(lc - rc_) <= 1e-12 * abs(rc_)


@pytest.mark.parametrize("name", ["gm1000k10", "track20x500"])
def test_gm_tracking_fp32(name):
    ilp = I.workload(name)
    note(name, "fp32")
    s = solver(ilp, precision=32, **I.rounding_options(name))
    o = O.Oracle(ilp)
    o.init()
    sc = scale_of(ilp)
    done = 0
    for target in (1, 2, 10):
        while done < target:
            s.run_sweeps(1)
            o.sweep(done % 2)
            o.average()
            done += 1
        lam, mm, avg = s.get_state()
        rl, rm, _ = o.get()
        for g, r in ((lam, rl), (mm, rm)):
            ok, err = fp32_close(g, r, sc)
            assert ok, (target, err)
    # 100 iterations: multipliers and differences at the end, bounds within
    # tolerance, monotone, below the certified bound
    s.run_sweeps(200 - done)
    o_hist = np.concatenate([[0.0] * done, o.run_dual((200 - done) // 2)])
    lam, mm, avg = s.get_state()
    rl, rm, ra = o.get()
    for what, g, r in (("lambda", lam, rl), ("M", mm, rm), ("avg", avg, ra)):
        ok, err = fp32_close(g, r, sc)
        note(f"  {name} after 200 sweeps: {what} max scaled error {err:.2e}")
        assert ok, (what, err)
    g = s.lb_history()
    assert abs(g[-1] - o_hist[-1]) <= 1e-4 * abs(o_hist[-1])
    lf, lc, res = s.lower_bound()
    rc_, _ = o.lb_cert()
    assert abs(lc - rc_) <= 1e-4 * abs(rc_)
    # LB_free <= LB_cert holds exactly; FP32 path sums move LB_free by ~1e-5 relative
    assert lf <= lc + 1e-4 * abs(lc)
    # Alg. 2 with the workload's options terminates with a feasible point
    # (exact row check by the reference) whose cost is above the bound, within
    # the paper's "fewer than 100" rounds; the dual state is left as it was
    before = s.get_state()
    r = s.round_primal()
    note(f"  {name} rounding: rc {r['rc']} rounds {r['rounds']} ub {r['ub']}")
    assert r["rc"] == 0 and r["rounds"] < 100
    assert o.count_violated(r["x"]) == 0
    assert r["ub"] >= lc - 1e-6 * abs(lc)
    assert all(np.array_equal(a, b) for a, b in zip(before, s.get_state()))


def oracle_threads():
    """host threads for the reference's loops over BDDs (results do not
    depend on the count)"""
    env = os.environ.get("OMP_NUM_THREADS")
    n = int(env) if env and env.isdigit() else (os.cpu_count() or 1)
    return max(1, min(n, 16))


def test_mrf256_trajectory_from_init():
    """the benchmark's instance and launch configuration (FP32, eager
    launches), all 2,154,496 BDDs: the GPU and the FP64 reference start from
    lambda = c/|J| and run the same sweeps; multipliers, min-marginal
    differences, LB_free and LB_cert agree within the scaled 1e-4 tolerance
    after sweeps 1 (forward), 2 (backward), 9 (forward) and 10 (backward)"""
    ilp = I.workload("mrf256x256L8")
    note("mrf256x256L8: load")
    s = solver(ilp, precision=32, graph_sweeps=0)
    note("mrf256x256L8: reference")
    o = O.Oracle(ilp, threads=oracle_threads())
    o.init()
    sc = scale_of(ilp)
    done = 0
    worst = {}
    for target in (1, 2, 9, 10):
        while done < target:
            s.run_sweeps(1)
            o.sweep(done % 2)
            o.average()
            done += 1
        lam, mm, avg = s.get_state()
        rl, rm, ra = o.get()
        for name, g, r in (("lambda", lam, rl), ("M", mm, rm), ("avg", avg, ra)):
            ok, err = fp32_close(g, r, sc)
            worst[name] = max(worst.get(name, 0.0), err)
            assert ok, (target, name, err)
        lbf = s.lb_history()[-1]
        lf, lc, res = s.lower_bound()
        rc_, rres = o.lb_cert()
        assert abs(lbf - o.lb_free()) <= 1e-4 * abs(o.lb_free()), (target, lbf, o.lb_free())
        assert abs(lc - rc_) <= 1e-4 * abs(rc_), (target, lc, rc_)
        assert lf <= lc + 1e-4 * abs(lc)
        note(f"  sweep {target}: lambda {worst['lambda']:.2e} M {worst['M']:.2e} "
             f"LB_free {abs(lbf - o.lb_free()) / abs(o.lb_free()):.2e} LB_cert {abs(lc - rc_) / abs(rc_):.2e}")
    o = None
    # bounds stay monotone (up to FP32 path sums) and the residual small
    s.run_dual(20)
    hist = s.lb_history()
    assert np.all(np.diff(hist) >= -1e-5 * np.abs(hist[1:]))
    lf, lc, res = s.lower_bound()
    assert lf <= lc + 1e-4 * abs(lc)
    assert res <= 1e-4 * sc * 8
    # Alg. 2 at full size: every original row holds for the decoded point
    # (checked again by the reference, exactly), and UB >= the certified bound
    note("mrf256x256L8: rounding")
    s.run_dual(200)
    lf, lc, res = s.lower_bound()
    r = s.round_primal()
    assert r["rc"] == 0
    assert O.Oracle(ilp).count_violated(r["x"]) == 0
    assert r["ub"] >= lc


def test_mrf256_fp64_bitexact_50_iterations():
    """the benchmark's instance in FP64 (graph replay, one-topology register
    tiles, the averaging kernel): multipliers, differences and averaged terms
    equal the reference's bit for bit after 50 iterations (100 sweeps); bound
    history and certified bound within 1e-12"""
    ilp = I.workload("mrf256x256L8")
    note("mrf256x256L8 fp64: load")
    s = solver(ilp, precision=64)
    note("mrf256x256L8 fp64: reference")
    o = O.Oracle(ilp, threads=oracle_threads())
    o.init()
    s.run_dual(50)
    hist = o.run_dual(50)
    g = s.lb_history()
    assert g.shape == hist.shape
    assert np.max(np.abs(g - hist)) <= 1e-12 * np.max(np.abs(hist))
    lam, mm, avg = s.get_state()
    rl, rm, ra = o.get()
    assert np.array_equal(lam, rl) and np.array_equal(mm, rm) and np.array_equal(avg, ra)
    lf, lc, res = s.lower_bound()
    rc_, rres = o.lb_cert()
    assert abs(lc - rc_) <= 1e-12 * abs(rc_)


# ---------------------------------------------------------------- Alg. 2
def test_rounding_fp64_matches_reference():
    cases = [example_a()[0], tie_example()]
    for seed in range(10):
        ilp = I.random_ilp(12, 8, max_row_len=5, seed=8000 + seed)
        if O.Oracle(ilp).status == O.OK:
            cases.append(ilp)
    for k, ilp in enumerate(cases):
        scale = k % 2
        note("rounding", ilp.name, "scale", scale)
        s = solver(ilp, precision=64, tau=0.0, seed=3, perturb_scale=scale)
        o = O.Oracle(ilp)
        o.init()
        s.run_dual(15)
        o.run_dual(15)
        r = s.round_primal()
        ro = o.round(tau=0.0, seed=3, scale=scale)
        assert r["rc"] == ro["rc"] and r["rounds"] == ro["rounds"]
        if r["rc"] == 0:
            # the point is integer work (bit-exact); c^T x is an FP64 sum in a
            # different order on the device
            assert np.array_equal(r["x"], ro["x"])
            assert abs(r["ub"] - ro["ub"]) <= 1e-12 * max(1.0, abs(ro["ub"]))
            assert brute.check_rows(ilp, r["x"]) == 0
        # the dual state is untouched by rounding
        assert np.array_equal(s.get_state()[0], o.get()[0])


@pytest.mark.parametrize("reopt,seed,converges", [(5, 0, False), (50, 0, True)])
def test_gm1000_rounding_fp64_matches_reference(reopt, seed, converges):
    """Alg. 2 on the full graph-matching instance in FP64, from the same
    500-iteration dual point: the GPU takes the reference's rounds exactly.
    With 5 re-optimisation iterations per round neither terminates within 60
    rounds (the perturbation runs ahead of the dual and a few dozen variables
    keep disagreeing); with 50 (the workload's setting) both terminate in the
    same round with the same feasible point."""
    ilp = I.workload("gm1000k10")
    cap = 60 if not converges else 150
    note("gm1000k10 rounding fp64 reopt", reopt, "seed", seed)
    s = solver(ilp, precision=64, reopt_iters=reopt, seed=seed, max_rounds=cap, tau=0.0)
    o = O.Oracle(ilp, threads=oracle_threads())
    o.init()
    s.run_dual(500)
    o.run_dual(500)
    r = s.round_primal()
    ro = o.round(reopt_iters=reopt, max_rounds=cap, tau=0.0, seed=seed, scale=0)
    note(f"  GPU rc {r['rc']} rounds {r['rounds']}; reference rc {ro['rc']} rounds {ro['rounds']}, "
         f"conflicts {list(ro['conflicts'][:8])}...{list(ro['conflicts'][-3:])}")
    assert r["rc"] == ro["rc"] and r["rounds"] == ro["rounds"]
    if converges:
        assert r["rc"] == 0
        assert np.array_equal(r["x"], ro["x"]) and o.count_violated(r["x"]) == 0
        assert abs(r["ub"] - ro["ub"]) <= 1e-12 * max(1.0, abs(ro["ub"]))
        assert r["ub"] >= s.lower_bound()[1]
    else:
        assert r["rc"] == B.NOT_CONVERGED and min(ro["conflicts"]) > 0


def test_rounding_not_converged_keeps_state():
    s = solver(example_b(), precision=64, max_rounds=30)
    s.run_dual(10)
    before = s.get_state()
    r = s.round_primal()
    assert r["rc"] == B.NOT_CONVERGED and r["rounds"] == 30
    after = s.get_state()
    assert all(np.array_equal(a, b) for a, b in zip(before, after))


@pytest.mark.parametrize("prec", [32, 64])
def test_rounding_partially_filled_shared_tile(prec):
    """20 independent exactly-one rows share one topology; their tile has 44
    unused lanes whose all-zero point the topology rejects"""
    rng = np.random.default_rng(5)
    rows = [([3 * r, 3 * r + 1, 3 * r + 2], [1, 1, 1], 0, 1) for r in range(20)]
    ilp = I.from_rows(60, rng.standard_normal(60), rows, name="onehot20")
    s = solver(ilp, precision=prec)
    s.run_dual(3)
    r = s.round_primal()
    assert r["rc"] == 0 and r["rounds"] == 0
    x = r["x"].reshape(20, 3)
    assert np.all(x.sum(axis=1) == 1)
    assert np.array_equal(np.argmax(x, axis=1), np.argmin(ilp.costs.reshape(20, 3), axis=1))


def test_rounding_mrf10_fp32_feasible():
    ilp = I.workload("mrf10x10L3")
    s = solver(ilp, precision=32)
    s.run_dual(100)
    lf, lc, _ = s.lower_bound()
    r = s.round_primal()
    assert r["rc"] == 0 and O.Oracle(ilp).count_violated(r["x"]) == 0
    assert r["ub"] >= lc - 1e-6 * abs(lc)


# ---------------------------------------------------------------- state handling
@pytest.mark.parametrize("prec", [32, 64])
def test_checkpoint_resume_is_bitwise(prec):
    ilp = I.workload("gm1000k10")
    a = solver(ilp, precision=prec)
    a.run_dual(10)
    blob = a.save_state()
    a.run_dual(10)
    b = solver(ilp, precision=prec)
    b.load_state(blob)
    b.run_dual(10)
    c = solver(ilp, precision=prec)
    c.run_dual(20)
    for x, y, z in zip(a.get_state(), b.get_state(), c.get_state()):
        assert np.array_equal(x, y) and np.array_equal(x, z)
    assert np.array_equal(a.lb_history(), b.lb_history())
    assert np.array_equal(a.lb_history(), c.lb_history())


def test_reset_and_determinism():
    ilp = I.workload("track20x500")
    s = solver(ilp, precision=32)
    s.run_dual(15)
    h1, st1 = s.lb_history(), s.get_state()
    s.reset()
    s.run_dual(15)
    h2, st2 = s.lb_history(), s.get_state()
    assert np.array_equal(h1, h2)
    assert all(np.array_equal(x, y) for x, y in zip(st1, st2))


def test_multipliers_are_feasible_and_min_marginals_match():
    ilp = I.random_ilp(20, 14, max_row_len=6, seed=9)
    s = solver(ilp, precision=64)
    o = O.Oracle(ilp)
    o.init()
    s.run_dual(7)
    o.run_dual(7)
    lam, mm = s.multipliers()
    pv, _ = s.pairs()
    acc = np.zeros(ilp.n_vars)
    np.add.at(acc, pv, lam)
    used = np.bincount(pv, minlength=ilp.n_vars) > 0
    assert np.max(np.abs(acc[used] - ilp.costs[used]), initial=0) <= 1e-12 * max(1, np.max(np.abs(ilp.costs)))
    assert np.array_equal(s.min_marginals(), o.full_mm())


def test_profiling_counts_launches():
    s = solver(I.workload("mrf10x10L3"), precision=32)
    s.profile(True)
    s.run_dual(5)
    for k in (B.K_SWEEP_FWD, B.K_SWEEP_BWD):
        n, ms = s.kernel_time(k)
        assert n == 5 and ms > 0
    n, _ = s.kernel_time(B.K_AVERAGE)
    assert n == 0   # only sweeps are bracketed
    s.profile(False)


# ---------------------------------------------------------------- graph replay
def _same_run(a, b, what):
    for x, y in zip(a.get_state(), b.get_state()):
        assert np.array_equal(x, y), what
    assert np.array_equal(a.lb_history(), b.lb_history()), what


@pytest.mark.parametrize("name,prec", [("random", 64), ("gm1000k10", 32), ("mrf10x10L3", 64)])
def test_graph_replay_matches_eager(name, prec):
    """sweeps replayed from a captured graph equal eager launches bit for bit,
    over several replays with eager work and synchronisation in between"""
    ilp = I.random_ilp(40, 30, max_row_len=7, seed=21) if name == "random" else I.workload(name)
    note("graph replay", name, prec)
    eager = solver(ilp, precision=prec, graph_sweeps=0)
    graph = solver(ilp, precision=prec, graph_sweeps=8)
    # odd start (eager sweep first), two replays, eager tail
    for s in (eager, graph):
        s.run_sweeps(1)
        s.run_sweeps(20)
    _same_run(eager, graph, "after 21 sweeps")
    for s in (eager, graph):
        s.lower_bound()                 # eager kernels between replays
    for s in (eager, graph):
        s.run_dual(30)                  # seven replays + eager sweeps
    _same_run(eager, graph, "after run_dual(30)")
    assert eager.lower_bound() == graph.lower_bound()
    ra, rb = eager.round_primal(), graph.round_primal()
    assert ra["rc"] == rb["rc"] and ra["rounds"] == rb["rounds"]
    if ra["rc"] == 0:
        assert np.array_equal(ra["x"], rb["x"]) and ra["ub"] == rb["ub"]
    for s in (eager, graph):
        s.reset()
        s.run_dual(12)
    _same_run(eager, graph, "after reset")


# ---------------------------------------------------------------- batches
def _members():
    ms = [I.random_ilp(14, 10, max_row_len=6, seed=4100 + k) for k in range(6)]
    ms += [I.mrf_grid(5, 6, 3, pairwise="potts", seed=3), I.workload("mrf10x10L3"),
           I.random_ilp(40, 30, max_row_len=7, seed=4107), I.from_rows(3, [1.0, -1.0, 0.5], [])]
    return [p for p in ms if O.Oracle(p).status == O.OK]


@pytest.mark.parametrize("prec", [64, 32])
def test_batch_matches_each_instance_alone(prec):
    """every instance of a batch follows its solo trajectory bit for bit"""
    ilps = _members()
    note("batch of", len(ilps), "prec", prec)
    b = solver(ilps, precision=prec)
    alone = [solver(p, precision=prec) for p in ilps]
    b.run_dual(25)
    for a in alone:
        a.run_dual(25)
    lam, mm = b.multipliers()
    pv, _ = b.pairs()
    voff = np.cumsum([0] + [p.n_vars for p in ilps])
    lbf, lbc, res = b.batch_bounds()
    at = 0
    for k, a in enumerate(alone):
        la, ma = a.multipliers()
        n = la.size
        assert np.array_equal(lam[at:at + n], la) and np.array_equal(mm[at:at + n], ma), k
        assert np.array_equal(pv[at:at + n] - voff[k], a.pairs()[0]), k
        at += n
        f, c, r = a.lower_bound()
        tol = 1e-12 if prec == 64 else 1e-6
        assert abs(lbf[k] - a.lb_history()[-1]) <= tol * max(1.0, abs(f)), k
        assert abs(lbc[k] - c) <= tol * max(1.0, abs(c)), k
        assert abs(res[k] - r) <= tol * max(1.0, abs(r)), k
    assert abs(sum(lbf) - b.lb_history()[-1]) <= 1e-9 * max(1.0, abs(sum(lbf)))
    rb = b.batch_round()
    for k, a in enumerate(alone):
        ra = a.round_primal()
        assert rb["status"][k] == ra["rc"], k
        assert rb["rounds"][k] == ra["rounds"], k
        if ra["rc"] == 0:
            assert np.array_equal(rb["x"][voff[k]:voff[k + 1]], ra["x"]), k
            assert rb["ub"][k] == ra["ub"], k
    # the dual state is untouched by the rounding
    l2, m2 = b.multipliers()
    assert np.array_equal(l2, lam) and np.array_equal(m2, mm)


def test_batch_with_graph_replay_and_checkpoint():
    """batches replayed from captured graphs, checkpointed and resumed, stay
    identical to the instances run alone with eager launches"""
    ilps = _members()[:6]
    b = solver(ilps, precision=64)
    with pytest.raises(B.BddmmaError) as e:
        b.batch_bounds()                       # no recorded sweep yet
    assert e.value.code == B.STATE
    b.run_dual(40)                             # 80 sweeps: one 64-sweep replay + 16 eager
    blob = b.save_state()
    b.run_dual(30)
    c = solver(ilps, precision=64)
    c.load_state(blob)
    c.run_dual(30)
    alone = [solver(p, precision=64, graph_sweeps=0) for p in ilps]
    for a in alone:
        a.run_dual(70)
    for s in (b, c):
        lam, mm = s.multipliers()
        at = 0
        for a in alone:
            la, ma = a.multipliers()
            assert np.array_equal(lam[at:at + la.size], la) and np.array_equal(mm[at:at + la.size], ma)
            at += la.size
    assert np.array_equal(b.lb_history(), c.lb_history())
    lbf, _, _ = b.batch_bounds()
    for k, a in enumerate(alone):
        assert abs(lbf[k] - a.lb_history()[-1]) <= 1e-12 * max(1.0, abs(lbf[k]))


# ---------------------------------------------------------------- fused averaging
def small_case(name):
    if name == "random":
        return I.random_ilp(300, 200, max_row_len=4, seed=23)
    if name == "mrf32L8":
        return I.mrf_grid(32, 32, 8, pairwise="trunc_linear", trunc=2, seed=1)
    return I.workload(name)


@pytest.mark.parametrize("name,prec", [("mrf10x10L3", 64), ("mrf10x10L3", 32), ("mrf32L8", 32), ("random", 64)])
def test_fused_averaging_matches_averaging_kernel(name, prec):
    """the sweep averaging the variables that span tiles itself (from the
    per-variable copy of the previous differences) runs the averaging
    kernel's operations in the same order: multipliers, differences, bound
    history and rounding equal those of the separate averaging launch bit for
    bit, eager and replayed from a graph, across a state load and a reset"""
    ilp = small_case(name)
    note("fused averaging", name, prec)
    for graph in (0, 8):
        fused = solver(ilp, precision=prec, graph_sweeps=graph)
        plain = solver(ilp, precision=prec, graph_sweeps=graph, fused_average=0)
        assert fused.stats.n_fused_vars > 0 and plain.stats.n_fused_vars == 0
        for s in (fused, plain):
            s.run_sweeps(3)
            s.run_sweeps(18)
        _same_run(fused, plain, "after 21 sweeps")
        # an external state (the other solver's, perturbed) loaded into both
        lam, mm, avg = plain.get_state()
        lam = lam + (np.arange(lam.size) % 7 - 3) * 1e-3
        for s in (fused, plain):
            s.set_state(lam, mm, avg)
            s.run_sweeps(9)
        _same_run(fused, plain, "after a state load")
        ra, rb = fused.round_primal(), plain.round_primal()
        assert ra["rc"] == rb["rc"] and ra["rounds"] == rb["rounds"]
        if ra["rc"] == 0:
            assert np.array_equal(ra["x"], rb["x"]) and ra["ub"] == rb["ub"]
        for s in (fused, plain):
            s.reset()
            s.run_dual(12)
        _same_run(fused, plain, "after a reset")


# ---------------------------------------------------------------- persistent kernel
@pytest.mark.parametrize("name,prec", [("mrf10x10L3", 64), ("mrf10x10L3", 32), ("mrf32L8", 32), ("random", 64)])
def test_persistent_kernel_matches_per_sweep_launches(name, prec):
    """blocks of sweeps in one cooperative launch (grid barrier between
    sweeps) give bit for bit the multipliers, differences and bound history of
    one launch per sweep, from an even and an odd start, across blocks of the
    bound-history capacity; in FP64 they also equal the reference"""
    ilp = small_case(name)
    note("persistent kernel", name, prec)
    per = solver(ilp, precision=prec, graph_sweeps=0)
    pst = solver(ilp, precision=prec, persistent=1)
    assert pst.stats.persist_tiles == pst.stats.n_tiles > 0
    for s in (per, pst):
        s.run_sweeps(1)      # odd start: the block begins with a backward sweep
        s.run_sweeps(40)
        s.run_dual(600)      # more sweeps than one launch holds
    _same_run(per, pst, "after 1241 sweeps")
    if prec == 64:
        o = O.Oracle(ilp, threads=oracle_threads())
        o.init()
        hist = []
        for k in range(1241):    # sweep k runs direction k mod 2, as on the GPU
            o.sweep(k % 2)
            o.average()
            hist.append(o.lb_free())
        hist = np.asarray(hist[41:])
        lam, mm, avg = pst.get_state()
        rl, rm, ra = o.get()
        assert np.array_equal(lam, rl) and np.array_equal(mm, rm)
        g = pst.lb_history()[-1200:]
        assert np.max(np.abs(g - hist)) <= 1e-12 * np.max(np.abs(hist))
    r1, r2 = per.round_primal(), pst.round_primal()
    assert r1["rc"] == r2["rc"] and r1["rounds"] == r2["rounds"]


# ---------------------------------------------------------------- certified bound off the feasible set
@pytest.mark.parametrize("prec", [64, 32])
def test_lb_cert_at_infeasible_multipliers(prec):
    """the certified bound of multipliers that do not sum to c (the state
    after FP32 rounding): the hand-derived point of Example A gives OPT = -5
    and max residual 1 exactly (dyadic values), and at perturbed multipliers
    of small random ILPs the GPU equals the reference (FP64: 1e-12; FP32
    multipliers are exact copies of the reference's rounded values)"""
    from test_oracle import residual_point
    ilp, _ = example_a()
    t, mbar, g = residual_point()
    s = solver(ilp, precision=prec)
    s.set_state(t - 0.5 * mbar, mbar, np.zeros(4))
    _, lbc, res = s.lower_bound()
    assert lbc == float(g["lb_cert"][0][0]) and res == float(g["max_residual"][0][0])
    rng = np.random.default_rng(5)
    for seed in range(6):
        ilp = I.random_ilp(30, 20, max_row_len=5, seed=700 + seed)
        o = O.Oracle(ilp)
        if o.status != O.OK:
            continue
        s = solver(ilp, precision=prec)
        o.init()
        o.run_dual(10)
        lam, mm, avg = o.get()
        lam = lam + rng.uniform(-0.5, 0.5, size=lam.size)
        if prec == 32:   # the reference sees the values the FP32 state holds
            lam, mm = lam.astype(np.float32).astype(np.float64), mm.astype(np.float32).astype(np.float64)
        o.set(lam=lam, mm=mm, avg=avg)
        s.set_state(lam, mm, avg)
        _, lbc, res = s.lower_bound()
        rc_, rres = o.lb_cert()
        scale = max(1.0, abs(rc_))
        assert abs(lbc - rc_) <= 1e-12 * scale * o.n_pairs, (seed, lbc, rc_)
        assert abs(res - rres) <= 1e-12 * max(1.0, rres)


def test_mrf512_fp64_bitexact_3_iterations():
    """the roofline workload in FP64, eager launches: all 77M multipliers,
    differences and averaged terms equal the reference's bit for bit after 3
    iterations (6 sweeps); bound history and certified bound within 1e-12"""
    ilp = I.workload("mrf512x512L8")
    note("mrf512x512L8 fp64: load")
    s = solver(ilp, precision=64, graph_sweeps=0)
    note("mrf512x512L8 fp64: reference")
    o = O.Oracle(ilp, threads=oracle_threads())
    o.init()
    s.run_dual(3)
    hist = o.run_dual(3)
    g = s.lb_history()
    assert g.shape == hist.shape
    assert np.max(np.abs(g - hist)) <= 1e-12 * np.max(np.abs(hist))
    lam, mm, avg = s.get_state()
    rl, rm, ra = o.get()
    assert np.array_equal(lam, rl) and np.array_equal(mm, rm) and np.array_equal(avg, ra)
    del lam, mm, avg, rl, rm, ra
    lf, lc, res = s.lower_bound()
    rc_, rres = o.lb_cert()
    assert abs(lc - rc_) <= 1e-12 * abs(rc_)


def test_mrf512_first_sweeps_match_reference():
    """the roofline workload of the benchmark (512x512 grid, 8 labels,
    77,447,168 pairs, multipliers beyond the last-level cache) in its launch
    configuration (FP32, eager launches): from lambda = c/|J| the GPU and the
    FP64 reference run a forward and a backward sweep; multipliers,
    min-marginal differences, LB_free and LB_cert agree within the scaled
    1e-4 tolerance after each"""
    ilp = I.workload("mrf512x512L8")
    note("mrf512x512L8: load")
    s = solver(ilp, precision=32, graph_sweeps=0)
    note("mrf512x512L8: reference")
    o = O.Oracle(ilp, threads=oracle_threads())
    o.init()
    sc = scale_of(ilp)
    for k in range(2):
        s.run_sweeps(1)
        o.sweep(k)
        o.average()
        lam, mm, _ = s.get_state()
        rl, rm, _ = o.get()
        for name, g, r in (("lambda", lam, rl), ("M", mm, rm)):
            ok, err = fp32_close(g, r, sc)
            assert ok, (k, name, err)
            note(f"  sweep {k + 1}: {name} max scaled error {err:.2e}")
        del lam, mm, rl, rm
        lbf = s.lb_history()[-1]
        _, lc, _ = s.lower_bound()
        rc_, _ = o.lb_cert()
        assert abs(lbf - o.lb_free()) <= 1e-4 * abs(o.lb_free()), (k, lbf, o.lb_free())
        assert abs(lc - rc_) <= 1e-4 * abs(rc_), (k, lc, rc_)

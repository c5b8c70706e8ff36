"""Serving pool (continuous batching) on the GPU, through the C ABI.

Whatever joins or leaves the resident batch around it, every instance ends
where a solver loaded with it alone ends after the same number of Alg. 1
iterations: multipliers, deferred differences and per-instance bounds are
compared bit for bit (the instance keeps its own tiles, the batch tables are
assembled on the device from the members' images, and a member's state is
copied unchanged when the batch is re-assembled).  Also: admission by
workspace bytes and member count, retirement by tolerance, adopted solvers.
"""
import sys
import threading
import time

import numpy as np
import pytest

import oracle as O
from paper_2111_10270_amd import binding as B
from paper_2111_10270_amd import instances as I

pytestmark = pytest.mark.gpu


def note(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    assert torch.cuda.get_device_properties(0).gcnArchName.startswith("gfx950")


def members():
    ms = [I.random_ilp(14, 10, max_row_len=6, seed=4200 + k) for k in range(4)]
    ms += [I.mrf_grid(5, 6, 3, pairwise="potts", seed=3), I.mrf_grid(6, 5, 8, pairwise="trunc_linear", seed=8),
           I.graph_matching(n_left=60, n_right=60, k=10, n_pairs=60, seed=11),
           I.cell_tracking(frames=5, dets=40, conflicts_per_frame=10, seed=12),
           I.random_ilp(40, 30, max_row_len=7, seed=4207), I.from_rows(3, [1.0, -1.0, 0.5], [])]
    return [p for p in ms if O.Oracle(p).status == O.OK]


def solo(ilp, n_iter, **kw):
    s = B.Solver(ilp, **kw).bind()
    s.run_dual(n_iter)
    return s


def assert_matches_oracle(ilp, n_iter, lam, mm, pv, pr, info, prec):
    """a retired member against the FP64 reference run alone from the start
    for the same iterations: terminated multipliers and differences bitwise
    in FP64 (within the scaled 1e-4 tolerance in FP32), bounds to 1e-12
    (1e-4)"""
    o = O.Oracle(ilp)
    o.init()
    hist = o.run_dual(n_iter)
    lbc, res = o.lb_cert()
    o.terminate()
    rl, rm, _ = o.get()
    opv, opr = o.pairs()
    assert np.array_equal(pv, opv) and np.array_equal(pr, opr), ilp.name
    sc = max(1e-12, float(np.mean(np.abs(ilp.costs)))) if ilp.n_vars else 1.0
    if prec == 64:
        assert np.array_equal(lam, rl) and np.array_equal(mm, rm), ilp.name
        tol_f = tol_c = 1e-12 * max(1.0, abs(lbc))
        tol_r = 1e-12 * max(1.0, float(np.max(np.abs(ilp.costs), initial=0.0)))
    else:
        for g, r in ((lam, rl), (mm, rm)):
            err = np.abs(g - r) / np.maximum(np.abs(r), sc)
            assert np.all(err <= 1e-4), (ilp.name, float(np.max(err, initial=0)))
        tol_f = tol_c = 1e-4 * max(abs(lbc), sc * max(1, o.n_bdds))
        tol_r = 1e-4 * sc * 8
    assert abs(info["lb_free"] - hist[-1]) <= tol_f, (ilp.name, info["lb_free"], hist[-1])
    assert abs(info["lb_cert"] - lbc) <= tol_c, (ilp.name, info["lb_cert"], lbc)
    assert abs(info["max_residual"] - res) <= tol_r, (ilp.name, info["max_residual"], res)


def assert_matches_solo(pool, t, ilp, oracle_check=True, **kw):
    """bitwise equal to the instance solved alone on the GPU, and (FP64
    bitwise, FP32 within tolerance) to the reference run alone"""
    info = pool.poll(t)
    assert info["state"] == B.POOL_DONE, info
    lam, mm, pv, pr = pool.result(t)
    a = solo(ilp, info["iters"], **kw)
    la, ma = a.multipliers()
    pa, ra = a.pairs()
    assert np.array_equal(lam, la) and np.array_equal(mm, ma), ilp.name
    assert np.array_equal(pv, pa) and np.array_equal(pr, ra), ilp.name
    f, c, r = a.batch_bounds()
    assert info["lb_free"] == f[0] and info["lb_cert"] == c[0] and info["max_residual"] == r[0], (ilp.name, info, f, c, r)
    if oracle_check and O.Oracle(ilp).n_bdds > 0:
        assert_matches_oracle(ilp, info["iters"], lam, mm, pv, pr, info, kw.get("precision", 32))


@pytest.mark.parametrize("prec", [64, 32])
def test_pool_members_match_solo(prec):
    """arrivals at different steps, different iteration counts, a member cap
    of 4: each instance ends bitwise as it ends alone"""
    ilps = members()
    iters = [10, 20, 15, 5, 25, 10, 30, 5, 20, 15][:len(ilps)]
    arrive = [0, 0, 0, 1, 1, 2, 3, 3, 5, 6][:len(ilps)]
    note("pool of", len(ilps), "instances, prec", prec)
    pool = B.Pool(max_active=4, precision=prec).bind(256 << 20)
    tickets = {}
    step = 0
    while len(tickets) < len(ilps) or any(pool.poll(t)["state"] != B.POOL_DONE for t in tickets.values()):
        for k, il in enumerate(ilps):
            if arrive[k] == step and k not in tickets:
                tickets[k] = pool.submit(il, iters[k])
        pool.wait_compiled()
        active, retired = pool.step(5)
        states = [pool.poll(t)["state"] for t in tickets.values()]
        assert active == states.count(B.POOL_ACTIVE) <= 4
        for t in tickets.values():   # lb_free after every step, lb_cert at retirement
            info = pool.poll(t)
            if info["state"] == B.POOL_ACTIVE:
                assert np.isfinite(info["lb_free"]) and np.isnan(info["lb_cert"]) and np.isnan(info["max_residual"])
        step += 1
        assert step < 100
    note("pool steps", step)
    for k, il in enumerate(ilps):
        info = pool.poll(tickets[k])
        assert info["iters"] == iters[k] and info["steps"] == iters[k] // 5
        assert_matches_solo(pool, tickets[k], il, precision=prec)
        pool.release(tickets[k])
    assert pool.step(5) == (0, 0)


@pytest.mark.parametrize("prec", [64, 32])
def test_pool_iteration_counts_not_multiple_of_step(prec):
    """n_iter = 7, 3 and 12 with steps of 5: a step stops where a member
    would run past its count, so each member runs exactly its n_iter and
    ends as it ends alone (GPU bitwise, reference)"""
    ilps = members()[:3]
    n_iters = [7, 3, 12]
    pool = B.Pool(max_active=8, precision=prec).bind(128 << 20)
    tickets = [pool.submit(p, n) for p, n in zip(ilps, n_iters)]
    pool.wait_compiled()
    runs = []
    for _ in range(20):
        active, retired = pool.step(5)
        runs.append(pool.poll(tickets[-1])["iters"])
        if active == 0:
            break
    assert runs == [3, 7, 12], runs   # steps of 3 (the second member retires), 4 (the first), 5
    for t, p, n in zip(tickets, ilps, n_iters):
        info = pool.poll(t)
        assert info["iters"] == n
        assert_matches_solo(pool, t, p, precision=prec)
        pool.release(t)


def test_pool_admission_by_workspace():
    """members' solo workspaces never exceed half the arena; an instance that
    can never fit fails with NO_MEMORY; the cap on members holds"""
    ilps = members()[:6]
    sizes = [B.Solver(p, precision=64).workspace_bytes() for p in ilps]
    want = max(sizes) + min(sizes)
    pool = B.Pool(max_active=3, precision=64).bind((8 << 20) + 3 * want + 4096)   # descriptors + 3 thirds
    cnt = pool.counters()
    half = cnt["batch_capacity"]
    assert want <= half < want + 4096 and cnt["image_free"] == cnt["image_capacity"]
    big = I.mrf_grid(40, 40, 8, pairwise="trunc_linear", seed=1)
    tb = pool.submit(big, 5)
    ts = [pool.submit(p, 10) for p in ilps]
    pool.wait_compiled()
    assert pool.poll(tb)["workspace_bytes"] > half
    seen = 0
    for _ in range(40):
        pool.step(5)
        act = [t for t in ts if pool.poll(t)["state"] == B.POOL_ACTIVE]
        assert len(act) <= 3
        assert sum(pool.poll(t)["workspace_bytes"] for t in act) <= half
        seen = max(seen, len(act))
        if all(pool.poll(t)["state"] == B.POOL_DONE for t in ts):
            break
    info = pool.poll(tb)
    assert info["state"] == B.POOL_FAILED and info["error"] == B.NO_MEMORY
    assert seen >= 1
    for p, t in zip(ilps, ts):
        assert_matches_solo(pool, t, p, precision=64)
    cnt = pool.counters()
    assert cnt["image_free"] == cnt["image_capacity"]          # every image released at retirement
    assert cnt["admitted"] == cnt["retired"] == len(ilps) and cnt["assemblies"] >= 2


def test_pool_tolerance_retirement():
    """with rel_tol a member retires once lb_free stops moving over a step,
    still on its solo trajectory"""
    il = I.mrf_grid(8, 8, 3, pairwise="potts", seed=21)
    tol = 1e-4
    pool = B.Pool(max_active=2, precision=64, rel_tol=tol).bind(64 << 20)
    t = pool.submit(il, 2000)
    pool.wait_compiled()
    lbs = []
    while pool.poll(t)["state"] != B.POOL_DONE:
        pool.step(10)
        lbs.append(pool.poll(t)["lb_free"])
        assert len(lbs) < 200
    info = pool.poll(t)
    assert info["iters"] < 2000 and len(lbs) >= 2
    assert abs(lbs[-1] - lbs[-2]) <= tol * max(1.0, abs(lbs[-1]))
    assert all(abs(lbs[k] - lbs[k - 1]) > tol * max(1.0, abs(lbs[k])) for k in range(1, len(lbs) - 1))
    assert_matches_solo(pool, t, il, precision=64)


def test_pool_adopts_loaded_solvers():
    """an instance loaded by the caller joins like a submitted one"""
    ilps = members()[:3]
    pool = B.Pool(max_active=8, precision=32).bind(64 << 20)
    ts = [pool.submit_loaded(B.Solver(p, precision=32), 10) for p in ilps]
    pool.wait_compiled()                      # checked and uploaded by the workers
    assert all(pool.poll(t)["state"] == B.POOL_READY for t in ts)
    assert pool.step(5) == (3, 0)
    assert pool.step(5) == (0, 3)
    for p, t in zip(ilps, ts):
        assert_matches_solo(pool, t, p, precision=32)


def test_pool_bounds_only_and_prefetched_images():
    """keep_multipliers=0 keeps bounds (still equal to the solo ones) and no
    multipliers; images of compiled instances are uploaded by the workers
    before admission"""
    ilps = members()[:4]
    pool = B.Pool(max_active=2, keep_multipliers=False, precision=64).bind(64 << 20)
    ts = [pool.submit(p, 10) for p in ilps]
    pool.wait_compiled()                      # compiled and uploaded
    cnt = pool.counters()
    assert cnt["image_free"] < cnt["image_capacity"]
    while any(pool.poll(t)["state"] != B.POOL_DONE for t in ts):
        pool.step(5)
    assert pool.counters()["image_ms"] >= 0.0
    for p, t in zip(ilps, ts):
        info = pool.poll(t)
        a = solo(p, 10, precision=64)
        f, c, r = a.batch_bounds()
        assert (info["lb_free"], info["lb_cert"], info["max_residual"]) == (f[0], c[0], r[0])
        with pytest.raises(B.BddmmaError) as e:
            pool.result(t)
        assert e.value.code == B.STATE
        _, _, pv, _ = pool.result(t, multipliers=False)
        assert np.array_equal(pv, a.pairs()[0])


@pytest.mark.parametrize("prec", [64, 32])
def test_pool_rounds_members_as_alone(prec):
    """with round=True each member is rounded at retirement in a batch of the
    retiring members: same status, rounds and point as Alg. 2 on the instance
    alone after the same iterations (UB to 1e-12: its sum runs per instance
    chunk either way, in FP64)"""
    ilps = members()[:6]
    iters = [10, 15, 10, 20, 5, 15][:len(ilps)]
    pool = B.Pool(max_active=3, round=True, precision=prec).bind(128 << 20)
    ts = [pool.submit(p, n) for p, n in zip(ilps, iters)]
    pool.wait_compiled()
    while any(pool.poll(t)["state"] != B.POOL_DONE for t in ts):
        pool.step(5)
    assert pool.counters()["round_ms"] > 0.0
    for p, t, n in zip(ilps, ts, iters):
        info = pool.poll(t)
        assert info["rounded"] == 1
        a = solo(p, n, precision=prec)
        r = a.round_primal()
        assert info["round_status"] == r["rc"] and info["rounds"] == r["rounds"], (p.name, info, r["rc"], r["rounds"])
        if r["rc"] == 0:
            assert np.array_equal(pool.primal(t), r["x"])
            assert abs(info["ub"] - r["ub"]) <= 1e-12 * max(1.0, abs(r["ub"]))
        else:
            with pytest.raises(B.BddmmaError) as e:
                pool.primal(t)
            assert e.value.code == B.STATE


def test_pool_submit_and_poll_from_other_threads():
    """a submitter thread and a polling thread run beside the stepping thread
    (the library releases the GIL in every call): each instance still ends
    bitwise as it ends alone"""
    ilps = members()
    iters = [10, 20, 15, 5, 25, 10, 30, 5, 20, 15][:len(ilps)]
    pool = B.Pool(max_active=3, precision=64).bind(256 << 20)
    tickets = [None] * len(ilps)
    submitted = threading.Event()
    errors = []

    def submitter():
        try:
            for k, il in enumerate(ilps):
                tickets[k] = pool.submit(il, iters[k])
                time.sleep(0.002)
        except Exception as e:   # reported by the main thread
            errors.append(e)
        submitted.set()

    def poller():
        try:
            while not submitted.is_set() or any(t is None for t in tickets):
                for t in list(tickets):
                    if t is not None:
                        pool.poll(t)
                pool.counters()
            for _ in range(50):
                for t in tickets:
                    pool.poll(t)
        except Exception as e:
            errors.append(e)

    ts = [threading.Thread(target=submitter), threading.Thread(target=poller)]
    for t in ts:
        t.start()
    steps = 0
    while not submitted.is_set() or any(pool.poll(t)["state"] != B.POOL_DONE for t in tickets if t is not None):
        active, _ = pool.step(5)
        assert active <= 3
        steps += 1
        assert steps < 400
        if not active:
            time.sleep(0.001)
    for t in ts:
        t.join()
    assert not errors, errors
    note("pool steps", steps)
    for k, il in enumerate(ilps):
        info = pool.poll(tickets[k])
        assert info["iters"] == iters[k]
        assert_matches_solo(pool, tickets[k], il, precision=64)


def knapsack_ilp(n, rows, seed, coef=20):
    rng = np.random.default_rng(seed)
    rs = []
    for _ in range(rows):
        k = int(rng.integers(6, 12))
        vs = rng.choice(n, size=k, replace=False)
        a = rng.integers(1, coef, size=k)
        rs.append((vs, a, -1, int(a.sum() // 2)))
    return I.from_rows(n, rng.standard_normal(n), rs, name=f"knap{n}x{rows}")


@pytest.mark.parametrize("prec", [64, 32])
def test_pool_members_with_wide_tiles_match_solo(prec):
    """members whose BDDs run on the node-parallel kernel (wide tiles of
    different sizes, several BDDs per wave) beside register-path members: the
    batch's wide list and LDS regions come from the assembled images, and each
    member still ends bitwise as it ends alone"""
    ilps = [knapsack_ilp(40, 30, 1), knapsack_ilp(60, 50, 2, coef=60), I.mrf_grid(5, 6, 3, pairwise="potts", seed=3),
            knapsack_ilp(30, 12, 3, coef=200)]
    assert all(B.Solver(p, precision=prec).stats.n_wide_tiles > 0 for p in ilps if p.name.startswith("knap"))
    iters = [10, 15, 10, 5]
    pool = B.Pool(max_active=3, precision=prec).bind(256 << 20)
    ts = [pool.submit(p, n) for p, n in zip(ilps, iters)]
    pool.wait_compiled()
    steps = 0
    while any(pool.poll(t)["state"] != B.POOL_DONE for t in ts):
        pool.step(5)
        steps += 1
        assert steps < 50
    for p, t in zip(ilps, ts):
        assert_matches_solo(pool, t, p, precision=prec)

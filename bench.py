"""Benchmark of the BDD Lagrange-decomposition hot path on one MI355X.

One step = one whole solve of the workload with the inputs resident in HBM:
re-initialise the multipliers (Alg. 1 initialisation), run the dual iterations
(forward sweep, averaging, backward sweep, averaging, FP64 bound reduction per
sweep), compute the certified FP64 bound, and run the perturbation rounding
(Alg. 2, including its termination step and exact row check).  Prints one JSON
line.  ``value`` counts every Alg. 1 iteration executed inside the timed steps
(the main ones and those of the rounding's re-optimisation) per second.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E
CSRC = os.path.join(ROOT, "paper_2111_10270_amd", "csrc")
PROFILES = os.path.join(ROOT, "profiles")
# bytes an updating sweep must move per (variable, subproblem) pair in this
# design: lambda and M-bar read, lambda and M written (FP32: 4 B each); the
# shortest paths stay on chip, node words and averaging codes are shared
# between tiles (a few KB per launch)
BYTES_PER_PAIR = {32: 16.0, 64: 32.0}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="mrf256x256L8")
    ap.add_argument("--iters", type=int, default=500)
    ap.add_argument("--precision", type=int, default=32)
    ap.add_argument("--opt", action="append", default=[], metavar="NAME=VALUE",
                    help="extra solver option of the headline solver (integer value), e.g. fused_average=0")
    ap.add_argument("--cpu-iters", type=int, default=10,
                    help="iterations of the single-thread reference sample")
    ap.add_argument("--cpu-all-iters", type=int, default=20,
                    help="iterations of the all-threads reference sample")
    ap.add_argument("--error-iters", default="200,500",
                    help="checkpoints (iterations from the start) at which the GPU state is compared with the FP64 "
                         "reference run on all host threads; the last one is the reported error")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--hbm-workload", default="mrf512x512L8",
                    help="workload of the roofline point whose multipliers exceed the last-level cache ('' = skip)")
    ap.add_argument("--hbm-iters", type=int, default=20)
    ap.add_argument("--roofline-only", action="store_true",
                    help="only the roofline leg on --hbm-workload (for counter runs)")
    ap.add_argument("--no-profile", action="store_true",
                    help="diagnostic: time the steps without per-sweep HIP events (no roofline)")
    ap.add_argument("--graph-sweeps", type=int, default=64, metavar="G",
                    help="replay blocks of G sweeps from a captured HIP graph, the library's default (kernel "
                         "time then comes from a separate profiled pass after the timed steps); 0 = eager "
                         "launches, whose sampled sweeps are timed inside the timed steps")
    ap.add_argument("--serve", type=int, default=512, metavar="N",
                    help="batched serving measurement over N instances of the mixed stream (0 = skip)")
    ap.add_argument("--serve-batch", type=int, default=16)
    ap.add_argument("--serve-iters", type=int, default=200)
    ap.add_argument("--pool-max", type=int, default=16, help="serving pool: most members at once (0 = skip)")
    ap.add_argument("--pool-step", type=int, default=25, help="serving pool: iterations per step")
    ap.add_argument("--pool-arena-gib", type=int, default=16)
    ap.add_argument("--ablation", action="store_true",
                    help="only compare deferred (Alg. 1) with serial min-marginal averaging: iterations to the "
                         "same bound and time per iteration")
    ap.add_argument("--abl-workloads", default="mrf10x10L3,gm1000k10,track20x500,mrf256x256L8")
    ap.add_argument("--abl-serial", type=int, default=100)
    ap.add_argument("--abl-deferred", type=int, default=1500)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB three times (HBM counter calibration)")
    ap.add_argument("--stream-sweep", action="store_true",
                    help="only run the stream probe over a range of array sizes (the sweep's bandwidth ceiling "
                         "with and without last-level-cache residency)")
    return ap.parse_args()


def log(msg):
    print(f"bench: {msg}", file=sys.stderr, flush=True)


# device code of the sweep kernel (the roofline kernel) and the headers it is compiled with
KERNEL_FILES = ("device_common.hpp", "kernels.hpp", "layout.hpp", "sweep_reg.hip", "sweep_tile.hpp")


def kernel_sha() -> str:
    """fingerprint of the kernel sources the counter summary was taken on"""
    h = hashlib.sha256()
    for f in KERNEL_FILES:
        h.update(f.encode())
        h.update(open(os.path.join(CSRC, f), "rb").read())
    return h.hexdigest()[:16]


def read_traffic(workload):
    """HBM bytes per sweep launch from the committed counter summary of the
    workload, if it was taken on the current kernel source."""
    path = os.path.join(PROFILES, f"sweep_{workload}_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_sha") != kernel_sha():
        return None
    try:
        return float(kv["hbm_bytes_per_sweep"])
    except (KeyError, ValueError):
        return None


def host_threads() -> int:
    """host threads this process may use: OMP_NUM_THREADS when set (the box
    sets it to its CPU share), else the CPUs of this process's affinity mask"""
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        return int(env)
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(ilp, a, gpu_states):
    """The FP64 reference on the host: a single-thread sample and an
    all-threads sample (its loops over BDDs and variables on host threads; the
    thread count does not change any result), both timed after BDD
    construction.  The all-threads run then continues to each checkpoint of
    `gpu_states` ({iterations: (lambda, M, lb_free, lb_cert)} of the GPU from
    the same start) and reports the GPU's error against it there."""
    import numpy as np

    import oracle

    nthr = host_threads()
    t = time.perf_counter()
    ref = oracle.Oracle(ilp, threads=nthr)
    build_s = time.perf_counter() - t
    ref.set_threads(1)
    ref.init()
    t = time.perf_counter()
    ref.run_dual(a.cpu_iters)
    dt1 = time.perf_counter() - t
    ref.set_threads(nthr)
    ref.init()
    t = time.perf_counter()
    ref.run_dual(a.cpu_all_iters)
    dtn = time.perf_counter() - t
    base = dict(value=a.cpu_all_iters / dtn, unit="dual iters/s", cores=nthr, kind="oracle",
                sample=f"{a.cpu_all_iters} Alg. 1 iterations of the same instance from the start, FP64, "
                       f"{nthr} host threads ({dtn:.1f} s; BDD construction, {build_s:.1f} s, not timed)",
                nproc=os.cpu_count(), cpu_model=cpu_model(),
                arcs_per_s=None,
                single_thread={"value": a.cpu_iters / dt1, "unit": "dual iters/s", "cores": 1,
                               "sample": f"{a.cpu_iters} Alg. 1 iterations from the start, FP64, one thread "
                                         f"({dt1:.1f} s)"})
    base["arcs_per_s"] = 2.0 * ref.n_nodes * base["value"]
    base["single_thread"]["arcs_per_s"] = 2.0 * ref.n_nodes * base["single_thread"]["value"]
    if not gpu_states:
        return base, None
    sc = max(1e-12, float(np.mean(np.abs(ilp.costs))))

    def scaled(g, r):   # |d| / max(|ref|, mean|c|), the parity tests' measure
        return float(np.max(np.abs(g - r) / np.maximum(np.abs(r), sc), initial=0.0))

    done = a.cpu_all_iters
    at = {}
    t = time.perf_counter()
    for k in sorted(gpu_states):
        if k < done:
            continue
        ref.run_dual(k - done)
        done = k
        lam, mm, lbf, lbc = gpu_states[k]
        rl, rm, _ = ref.get()
        rc, _ = ref.lb_cert()
        at[str(k)] = {"lambda_max_scaled": scaled(lam, rl), "min_marginal_max_scaled": scaled(mm, rm),
                      "lb_free_rel": abs(lbf - ref.lb_free()) / max(1.0, abs(ref.lb_free())),
                      "lb_cert_rel": abs(lbc - rc) / max(1.0, abs(rc)),
                      "lb_free_ref": ref.lb_free(), "lb_cert_ref": rc}
        log(f"error vs reference at {k} iterations done")
    last = str(done)
    err = {"iterations": done, "scale_mean_abs_cost": sc, **{k: v for k, v in at[last].items()},
           "at": at, "reference_threads": nthr, "reference_s": time.perf_counter() - t}
    return base, err


def gen_serving(n, seed=5):
    """the serving stream's instances, generated on host processes (forked
    before any GPU work: the generators are plain NumPy)"""
    import multiprocessing as mp

    from paper_2111_10270_amd import instances as I

    specs = I.serving_specs(n, seed)
    with mp.get_context("fork").Pool(min(host_threads(), 16)) as pool:
        return pool.map(I.serving_instance, specs, chunksize=4)


def compile_all(B, ilps, precision):
    """host compilation of independent solvers on host threads (the library
    releases the interpreter while it compiles); returns the solvers and the
    summed per-instance compile seconds"""
    from concurrent.futures import ThreadPoolExecutor

    def one(p):
        t = time.perf_counter()
        s = B.Solver(p, precision=precision)
        return s, time.perf_counter() - t

    with ThreadPoolExecutor(min(host_threads(), 16)) as ex:
        out = list(ex.map(one, ilps))
    return [s for s, _ in out], sum(t for _, t in out)


def serve(a, B, insts, torch):
    """Batched serving of a seeded stream of small instances (four families,
    sizes drawn per instance).  A solve is serve_iters Alg. 1 iterations plus
    the per-instance bounds (the serving target is the solo lower bound, which
    every batched instance reproduces exactly).  Service times are measured on
    the GPU, instance by instance (sequential) and in batches of consecutive
    arrivals; latencies come from Poisson arrivals at twice the sequential
    solve rate replayed against those service times (FIFO server).  Host
    compilation is untimed and done in chunks just before use."""
    import numpy as np

    n = len(insts)
    groups = [list(range(i, min(i + a.serve_batch, n))) for i in range(0, n, a.serve_batch)]

    def run(s):
        """bind + solve s, then drop it (and its workspace)"""
        torch.cuda.synchronize()
        t = time.perf_counter()
        s.bind("cuda:0")
        s.run_dual(a.serve_iters)
        lbf, _, _ = s.batch_bounds()
        torch.cuda.synchronize()
        return time.perf_counter() - t, lbf

    run(B.Solver(insts[0], precision=a.precision))   # warm-up (allocator, code objects)
    seq_t, seq_lb = [], []
    compile_s = 0.0
    chunk = 64
    for c0 in range(0, n, chunk):
        solvers, cs = compile_all(B, insts[c0:c0 + chunk], a.precision)
        compile_s += cs
        for k in range(len(solvers)):
            dt, lbf = run(solvers[k])
            solvers[k] = None
            seq_t.append(dt)
            seq_lb.append(lbf[0])
    log(f"serving: {n} sequential solves done")
    bat_t, diff = [], 0.0
    for j0 in range(0, len(groups), 8):
        gs = groups[j0:j0 + 8]
        batches, _ = compile_all(B, [[insts[k] for k in g] for g in gs], a.precision)
        for q, g in enumerate(gs):
            dt, lbf = run(batches[q])
            batches[q] = None
            bat_t.append(dt)
            for i, k in enumerate(g):
                diff = max(diff, abs(lbf[i] - seq_lb[k]) / max(1.0, abs(seq_lb[k])))
    log(f"serving: {len(groups)} batches done")
    seq_rate = n / sum(seq_t)
    rate = 2.0 * seq_rate
    rng = np.random.default_rng(7)
    arrive = np.cumsum(rng.exponential(1.0 / rate, size=n))
    # sequential FIFO server
    t, lat_seq = 0.0, []
    for k in range(n):
        t = max(t, arrive[k]) + seq_t[k]
        lat_seq.append(t - arrive[k])
    # batched server: a batch starts once its last member has arrived
    t, lat_b = 0.0, []
    for g, dt in zip(groups, bat_t):
        t = max(t, arrive[g[-1]]) + dt
        lat_b += [t - arrive[k] for k in g]
    pct = lambda v, q: float(np.percentile(np.asarray(v) * 1e3, q))
    pool = serve_pool(a, B, insts, seq_lb, rate, pct) if a.pool_max > 0 else None
    return {"instances": n, "batch": a.serve_batch, "iterations": a.serve_iters,
            "host_compile_ms_per_instance": compile_s / n * 1e3, "pool": pool,
            "vars": int(sum(p.n_vars for p in insts)),
            "seq_solves_per_s": seq_rate, "batched_solves_per_s": n / sum(bat_t),
            "speedup": (n / sum(bat_t)) / seq_rate, "arrival_rate_per_s": rate,
            "p50_ms": pct(lat_b, 50), "p99_ms": pct(lat_b, 99),
            "seq_p50_ms": pct(lat_seq, 50), "seq_p99_ms": pct(lat_seq, 99),
            "lb_max_rel_diff_vs_solo": diff}


def serve_pool(a, B, insts, seq_lb, rate, pct):
    """Continuous batching, live in wall-clock time: the same Poisson arrivals
    (rate, seed 7) as the replayed servers; each instance arrives compiled
    (host compilation is reported separately), joins the pool at a step
    boundary once its table image is on the device, and retires after
    serve_iters iterations.  Latency to target: arrival -> end of the first
    step after which its lb_free is within 1e-3 (relative) of its solo final
    lb_free; latency to done: arrival -> retirement.  Members follow their
    solo trajectories exactly, so every final bound equals the solo one.  The
    pool keeps bounds only (no multiplier copies at retirement).  The
    saturated run submits every instance at time 0 (capacity)."""
    import numpy as np

    n = len(insts)
    rng = np.random.default_rng(7)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=n))
    target = [lb - 1e-3 * max(1.0, abs(lb)) for lb in seq_lb]

    def run(arrive, graph=False):
        """graph: each step's sweeps replay from a HIP graph captured once
        per batch membership (captured again after every re-assembly)"""
        solvers, _ = compile_all(B, insts, a.precision)
        pool = B.Pool(max_active=a.pool_max, keep_multipliers=False, precision=a.precision,
                      graph_sweeps=2 * a.pool_step if graph else 0).bind(a.pool_arena_gib << 30)
        tw = pool.submit_loaded(B.Solver(insts[0], precision=a.precision), a.pool_step)   # warm-up
        pool.wait_compiled()
        pool.step(a.pool_step)
        pool.release(tw)
        c0 = pool.counters()
        tickets, reach, fin, final = [None] * n, [None] * n, [None] * n, [None] * n
        nxt = done = member_steps = 0
        t0 = time.perf_counter()
        while done < n:
            now = time.perf_counter() - t0
            while nxt < n and arrive[nxt] <= now:
                tickets[nxt] = pool.submit_loaded(solvers[nxt], a.serve_iters)
                solvers[nxt] = None
                nxt += 1
            if nxt == done:
                time.sleep(max(0.0, arrive[nxt] - (time.perf_counter() - t0)))
                continue
            active, retired = pool.step(a.pool_step)
            t = time.perf_counter() - t0
            member_steps += active + retired
            for k in range(nxt):
                if fin[k] is not None:
                    continue
                info = pool.poll(tickets[k])
                if info["steps"] and reach[k] is None and info["lb_free"] >= target[k]:
                    reach[k] = t
                if info["state"] == B.POOL_DONE:
                    fin[k] = t
                    final[k] = info["lb_free"]
                    done += 1
                    pool.release(tickets[k])
        wall = time.perf_counter() - t0
        c = pool.counters()
        steps = c["steps"] - c0["steps"]
        lat_t = [reach[k] - arrive[k] for k in range(n)]
        lat_d = [fin[k] - arrive[k] for k in range(n)]
        diff = max(abs(final[k] - seq_lb[k]) / max(1.0, abs(seq_lb[k])) for k in range(n))
        return {"served_per_s": n / (max(fin) - arrive[0]), "steps": steps,
                "mean_members_per_step": member_steps / max(1, steps),
                "p50_ms_to_target": pct(lat_t, 50), "p99_ms_to_target": pct(lat_t, 99),
                "p50_ms_to_done": pct(lat_d, 50), "p99_ms_to_done": pct(lat_d, 99),
                "lb_max_rel_diff_vs_solo": diff, "wall_ms": wall * 1e3, "assemblies": c["assemblies"] - c0["assemblies"],
                "host_ms": {k: round(c[k] - c0[k], 2) for k in ("image_ms", "merge_ms", "bind_ms", "run_ms",
                                                                 "bounds_ms", "retire_ms")}}

    live = run(arrivals)
    sat = run(np.zeros(n))
    sat_g = run(np.zeros(n), graph=True)
    return {"max_active": a.pool_max, "step_iters": a.pool_step, "arrival_rate_per_s": rate,
            "launch_mode": "eager launches per step (graph replay is measured in saturated_graph)",
            "live": live, "saturated": sat, "saturated_graph": sat_g}


def ablation(a, B, I, torch):
    """Deferred parallel averaging (Alg. 1) against the serial averaging it
    replaces (Sec. 3, sequential update), both on the GPU from the same start
    (lambda = c/|J|): at checkpoints k of the serial run, the number of
    deferred iterations whose bound (LB_free after the iteration) first
    reaches the serial bound after k iterations (Sec. 6 reports about three
    times as many for the deferred scheme), and the wall time each needs."""
    import numpy as np

    out = {}
    for wl in a.abl_workloads.split(","):
        ilp = I.workload(wl)
        d = B.Solver(ilp, precision=a.precision, graph_sweeps=64).bind()
        d.run_dual(2)
        d.reset()
        torch.cuda.synchronize()
        t = time.perf_counter()
        d.run_dual(a.abl_deferred)
        torch.cuda.synchronize()
        td = (time.perf_counter() - t) / a.abl_deferred
        ld = d.lb_history()[1::2]
        d = None
        torch.cuda.empty_cache()
        s = B.Solver(ilp, precision=a.precision, serial_mma=1).bind()
        s.run_serial(1)
        s.reset()
        torch.cuda.synchronize()
        t = time.perf_counter()
        ls = s.run_serial(a.abl_serial)[1::2]
        torch.cuda.synchronize()
        ts = (time.perf_counter() - t) / a.abl_serial
        s = None
        torch.cuda.empty_cache()
        at = {}
        for k in (1, 5, 10, 20, 50, 100):
            if k > len(ls):
                continue
            hit = np.nonzero(ld >= ls[k - 1])[0]
            n = int(hit[0]) + 1 if hit.size else None
            at[str(k)] = {"serial_lb": float(ls[k - 1]), "deferred_iters": n,
                          "iter_ratio": n / k if n else None,
                          "time_ratio": (n * td) / (k * ts) if n else None}
        out[wl] = {"deferred_ms_per_iter": td * 1e3, "serial_ms_per_iter": ts * 1e3,
                   "deferred_final_lb": float(ld[-1]), "serial_final_lb": float(ls[-1]),
                   "deferred_iters": a.abl_deferred, "serial_iters": a.abl_serial, "at_serial_iter": at}
        log(f"ablation {wl} done")
    return {"ablation": "deferred vs serial min-marginal averaging", "dtype": "f64" if a.precision == 64 else "f32",
            "data": "synthetic", "workloads": out, "node_word_sharing": compression(a, B, I, torch)}


def compression(a, B, I, torch):
    """BDD compression by shared node words: the default layout (tiles of one
    topology share one copy of their node words) against per-lane words for
    every width-2 tile (small_tiles = 2^30) on mrf256x256L8, when it is among
    the ablation workloads; us per sweep (sweep + averaging) from HIP events."""
    wl = "mrf256x256L8"
    if wl not in a.abl_workloads.split(","):
        return None   # small problems keep per-lane words anyway (one launch per layer class)
    ilp = I.workload(wl)
    res = {"workload": wl}
    for name, kw in (("shared", {}), ("per_lane", {"small_tiles": 1 << 30})):
        s = B.Solver(ilp, precision=a.precision, graph_sweeps=0, **kw).bind()
        s.run_sweeps(20)
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(3):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(s.stream)
            s.run_sweeps(100)
            e1.record(s.stream)
            torch.cuda.synchronize()
            best = min(best, 1e3 * e0.elapsed_time(e1) / 100)
        res[name] = {"node_words": s.stats.node_words, "nodes": s.stats.n_nodes,
                     "workspace_bytes": s.workspace_bytes(), "us_per_sweep": best}
        s = None
        torch.cuda.empty_cache()
    log("node-word sharing done")
    return res


def roofline_of(P, precision, sweep_ms, workload, traffic, note, stream=None):
    """roofline object of the sweep kernel: algorithmic bytes of one sweep
    launch (BYTES_PER_PAIR per pair) over its average launch time; `stream`
    is the stream probe at the sweep's array size (stream_ceiling)"""
    alg = BYTES_PER_PAIR[precision] * P
    achieved = alg / (sweep_ms * 1e-3) / 1e9 if sweep_ms > 0 else None
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS if achieved else None, "traffic": traffic,
            "kernel": "k_sweep_reg (updating sweep)", "workload": workload,
            "alg_bytes_per_launch": alg, "kernel_ms": sweep_ms,
            "traffic_GBs": traffic / (sweep_ms * 1e-3) / 1e9 if traffic and sweep_ms > 0 else None,
            "stream_probe": stream,
            "frac_of_stream": achieved / stream["GBs"] if achieved and stream else None,
            "note": note}


def model_effective(N, P, V, iters_per_s, precision):
    """bytes per iteration of the node-array cost model (FP32: every node's
    two child indices and shortest paths, every pair's multiplier, difference,
    variable index and gathered term, and the averaging's index and value per
    pair, moved through HBM: 32 N + 56 P + 8 V) at the measured iteration
    rate; null in FP64, for which the model fixes no byte count"""
    if precision != 32 or not iters_per_s:
        return None
    b = 32 * N + 56 * P + 8 * V
    return {"bytes_per_iteration": b, "GBs": b * iters_per_s / 1e9, "iters_per_s": iters_per_s,
            "model": "32 N + 56 P + 8 V bytes per iteration",
            "note": "the design keeps shortest paths in registers or LDS and shares node words, so it does not "
                    "move these bytes; above the HBM peak by construction, not a roofline fraction"}


def stream_ceiling(B, torch, n, precision, reps=10, placements=3):
    """bddmma_stream_probe over two arrays of n elements (the size of the
    sweep's multipliers and differences), both halves of one buffer as in the
    solver's workspace: mean time of `reps` calls after two warm-up calls, HIP
    events on the probe's stream; the arrays stay resident between calls, as
    the sweep's do between sweeps.  The rate depends on where the buffer lands
    in memory, so `placements` buffers are held at once and the fastest is
    reported (with every one's time)"""
    dt = torch.float32 if precision == 32 else torch.float64
    st = torch.cuda.current_stream(torch.device("cuda:0"))
    bufs, times = [], []
    for _ in range(placements):
        buf = torch.zeros(2 * n, dtype=dt, device="cuda:0")
        bufs.append(buf)
        x, y = buf[:n], buf[n:]
        y.fill_(1.0)
        for _ in range(2):
            B.stream_probe(x, y, st)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            B.stream_probe(x, y, st)
        e1.record(st)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1) * 1e3 / reps)
    nbytes = 4 * n * bufs[0].element_size()
    del bufs
    torch.cuda.empty_cache()
    us = min(times)
    return {"GBs": nbytes / (us * 1e-6) / 1e9, "us_per_call": us, "us_per_placement": times,
            "bytes_per_call": nbytes, "elements_per_array": n, "kernel": "k_stream_probe"}


def sweep_event_ms(s, B):
    n_f, t_f = s.kernel_time(B.K_SWEEP_FWD)
    n_b, t_b = s.kernel_time(B.K_SWEEP_BWD)
    return (t_f + t_b) / max(1, n_f + n_b), n_f + n_b


def hbm_leg(a, B, I, torch):
    """the sweep kernel on a workload whose multipliers and differences do not
    fit the 256 MB last-level cache: eager launches, HIP events around every
    sweep launch on the library's stream, iterations from the start"""
    ilp = I.workload(a.hbm_workload)
    extra = {k: int(v) for k, v in (o.split("=", 1) for o in a.opt)}
    s = B.Solver(ilp, precision=a.precision, graph_sweeps=0, **extra).bind("cuda:0")
    P, n_slots, st_n, st_v = s.stats.n_pairs, s.stats.n_slots, s.stats.n_nodes, s.stats.n_vars
    s.run_dual(3)   # warm-up
    s.reset()
    torch.cuda.synchronize()
    s.profile(True, stride=1)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s.stream)
    s.run_dual(a.hbm_iters)
    e1.record(s.stream)
    torch.cuda.synchronize()
    sweep_ms, launches = sweep_event_ms(s, B)
    s.profile(False)
    ws = s.workspace_bytes()
    lbf, lbc, _ = s.lower_bound()
    s = None
    torch.cuda.empty_cache()
    slot_bytes = BYTES_PER_PAIR[a.precision] / 2 * P
    r = roofline_of(P, a.precision, sweep_ms, a.hbm_workload, read_traffic(a.hbm_workload),
                    f"multipliers + differences {slot_bytes / 1e6:.0f} MB > 256 MB last-level cache",
                    stream_ceiling(B, torch, n_slots, a.precision))
    r.update({"sweep_launches_timed": launches, "pairs": P,
              "dual_iters_per_s": a.hbm_iters / (e0.elapsed_time(e1) * 1e-3), "workspace_bytes": ws,
              "lb_free": lbf, "lb_cert": lbc})
    r["model_effective"] = model_effective(st_n, P, st_v, r["dual_iters_per_s"], a.precision)
    log(f"roofline leg on {a.hbm_workload} done")
    return r


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); the multi-GPU path is not built",
              file=sys.stderr)
        sys.exit(2)
    # the serving stream is generated on forked host processes before any GPU work
    serve_insts = gen_serving(a.serve) if a.serve > 0 and not (a.ablation or a.calibrate_copy or a.roofline_only
                                                                  or a.stream_sweep) else None
    if serve_insts:
        log(f"serving: {len(serve_insts)} instances generated")
    import torch

    if a.calibrate_copy:
        n = a.calibrate_copy << 20
        src = torch.ones(n // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        dst.copy_(src)
        e0.record()
        for _ in range(3):
            dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 3
        print(json.dumps({"copy_bytes_per_launch": n, "copy_ms": ms, "copy_read_plus_write_GBs": 2 * n / ms / 1e6}),
              flush=True)
        return

    from paper_2111_10270_amd import binding as B
    from paper_2111_10270_amd import instances as I

    if a.ablation:
        print(json.dumps(ablation(a, B, I, torch)), flush=True)
        return
    if a.stream_sweep:
        # elements per array: 2-8 Mi, then the slot counts of the 256x256 and
        # 512x512 grids (8 labels), twice the latter
        for prec, sizes in ((32, (2 << 20, 4 << 20, 8 << 20, 19390464, 38780928, 77709312, 155418624)),
                            (64, (19390464, 77709312))):
            for n in sizes:
                r = stream_ceiling(B, torch, n, prec)
                r.update({"precision": prec, "working_set_MB": r["bytes_per_call"] / 2e6})
                print(json.dumps(r), flush=True)
        return
    if a.roofline_only:
        print(json.dumps({"roofline": hbm_leg(a, B, I, torch), "kernel_sha": kernel_sha()}), flush=True)
        return

    ilp = I.workload(a.workload)
    extra = {k: int(v) for k, v in (o.split("=", 1) for o in a.opt)}
    s = B.Solver(ilp, precision=a.precision, graph_sweeps=a.graph_sweeps,
                 **{**I.rounding_options(a.workload), **extra})
    s.bind("cuda:0")
    st = s.stats
    N, P, V = st.n_nodes, st.n_pairs, st.n_vars
    stream = s.stream

    def step():
        s.reset()
        s.run_dual(a.iters)
        lf, lc, res = s.lower_bound()
        r = s.round_primal()
        return lf, lc, res, r

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    # HIP events around the sweeps of every 10th iteration of the timed steps
    # (graph replay records no per-sweep events: profiled separately below)
    s.profile(not a.no_profile and not a.graph_sweeps, stride=10)
    t0 = time.perf_counter()
    iters = 0
    results = []
    dual_ms = 0.0
    for k in range(a.steps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        s.reset()
        s.run_dual(a.iters)
        e1.record(stream)
        lf, lc, res = s.lower_bound()
        r = s.round_primal()
        torch.cuda.synchronize()
        dual_ms += e0.elapsed_time(e1)
        iters += a.iters + r["rounds"] * s.options.reopt_iters
        results.append((lf, lc, res, r))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    log(f"{a.steps} timed steps done")
    ms_step = wall * 1e3 / a.steps

    if a.graph_sweeps and not a.no_profile:
        s.profile(True, stride=1)
        s.reset()
        s.run_dual(50)
        torch.cuda.synchronize()
    sweep_ms, _ = sweep_event_ms(s, B)
    s.profile(False)
    lf, lc, res, r = results[-1]
    rl_main = roofline_of(P, a.precision, sweep_ms, a.workload, read_traffic(a.workload),
                          f"multipliers + differences {BYTES_PER_PAIR[a.precision] / 2 * P / 1e6:.0f} MB: resident "
                          f"in the 256 MB last-level cache between sweeps, so this point is not an HBM measurement",
                          stream_ceiling(B, torch, st.n_slots, a.precision))
    out = {
        "metric": "dual iters/s & BDD arcs/s vs HBM roofline; batched solves/s, p50/p99 latency",
        "value": iters / wall,
        "unit": "dual iters/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if a.precision == 32 else "f64",
        "data": "synthetic",
        "config": {"workload": a.workload, "iterations_per_solve": a.iters, "vars": V, "bdds": st.n_bdds,
                   "pairs": P, "nodes": N, "precision_bound_sums": "f64", "graph_sweeps": a.graph_sweeps,
                   "fused_average_vars": st.n_fused_vars, **({"options": extra} if extra else {})},
        "arcs_per_s": 2.0 * N * iters / wall,
        "dual_phase_iters_per_s": a.iters * a.steps / (dual_ms * 1e-3),
        "model_effective": model_effective(N, P, V, a.iters * a.steps / (dual_ms * 1e-3), a.precision),
        "dual_phase_arcs_per_s": 2.0 * N * a.iters * a.steps / (dual_ms * 1e-3),
        "solves_per_s": a.steps / wall,
        "kernel_ms": {"sweep": sweep_ms},
        "roofline": None,
        "roofline_headline_workload": rl_main,
        "result": {"lb_free": lf, "lb_cert": lc, "max_residual": res, "ub": r["ub"] if r["rc"] == 0 else None,
                   "rounding_rc": r["rc"], "rounding_rounds": r["rounds"]},
    }
    gpu_states = {}
    if not a.no_cpu_baseline:
        # the GPU's state at the error checkpoints, from the start (untimed)
        s.reset()
        done = 0
        for k in sorted(int(v) for v in a.error_iters.split(",") if v):
            s.run_dual(k - done)
            done = k
            lam_g, mm_g, _ = s.get_state()
            lbf_g, lbc_g, _ = s.lower_bound()
            gpu_states[k] = (lam_g.astype("float64"), mm_g.astype("float64"), lbf_g, lbc_g)
    s = None
    torch.cuda.empty_cache()
    if a.hbm_workload:
        out["roofline"] = hbm_leg(a, B, I, torch)
    else:
        out["roofline"] = rl_main
    if serve_insts:
        out["batched"] = serve(a, B, serve_insts, torch)
        serve_insts = None
    if not a.no_cpu_baseline:
        out["cpu_baseline"], out["error_vs_oracle"] = cpu_baseline(ilp, a, gpu_states)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

"""ctypes binding of the solver's C ABI (include/bddmma.h).

Argument marshalling only: every step of the method runs in the HIP/C++
library.  PyTorch provides the device workspace and the stream.  There is no
fallback: without ``libbddmma.so`` every call raises.
"""
from __future__ import annotations

import ctypes as C
import os
import sys

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libbddmma.so")

OK, INVALID_ARG, INFEASIBLE, NO_MEMORY, NOT_CONVERGED, HIP_ERROR, STATE = 0, -1, -2, -3, -4, -5, -6
K_SWEEP_FWD, K_SWEEP_BWD, K_AVERAGE, K_LB_REDUCE = 0, 1, 2, 3
KERNEL_NAMES = {K_SWEEP_FWD: "sweep_fwd", K_SWEEP_BWD: "sweep_bwd", K_AVERAGE: "average", K_LB_REDUCE: "lb_reduce"}

# every entry point the header declares (checked by the tests)
EXPORTS = ("bddmma_options_default", "bddmma_create", "bddmma_destroy", "bddmma_load_ilp", "bddmma_get_stats",
           "bddmma_workspace_bytes", "bddmma_bind", "bddmma_reset", "bddmma_run_dual", "bddmma_run_sweeps", "bddmma_lower_bound",
           "bddmma_lb_history", "bddmma_num_pairs", "bddmma_get_pairs", "bddmma_get_fixed",
           "bddmma_get_multipliers", "bddmma_get_state", "bddmma_set_state", "bddmma_min_marginals",
           "bddmma_round_primal", "bddmma_save_state", "bddmma_load_state", "bddmma_profile",
           "bddmma_kernel_time", "bddmma_last_error", "bddmma_load_batch", "bddmma_num_instances",
           "bddmma_batch_bounds", "bddmma_batch_round", "bddmma_pool_create", "bddmma_pool_bind",
           "bddmma_pool_submit", "bddmma_pool_submit_loaded", "bddmma_pool_step", "bddmma_pool_wait_compiled",
           "bddmma_pool_poll", "bddmma_pool_result", "bddmma_pool_release", "bddmma_pool_destroy",
           "bddmma_pool_get_counters", "bddmma_run_serial", "bddmma_autotune", "bddmma_pool_primal",
           "bddmma_encode_rows", "bddmma_bind_static", "bddmma_stream_probe")
STATIC_WORKSPACE_BYTES = 64 << 20

POOL_QUEUED, POOL_READY, POOL_ACTIVE, POOL_DONE, POOL_FAILED = 0, 1, 2, 3, 4
POOL_KEEP_MULTIPLIERS, POOL_ROUND = 1, 2


class BddmmaError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"bddmma error {code}: {msg}")
        self.code = code


class Options(C.Structure):
    _fields_ = [("omega", C.c_double), ("rel_tol", C.c_double), ("lb_every", C.c_int32),
                ("precision", C.c_int32), ("delta0", C.c_double), ("alpha", C.c_double),
                ("reopt_iters", C.c_int32), ("max_rounds", C.c_int32), ("tau", C.c_double),
                ("seed", C.c_uint64), ("sp_in_lds_max_nodes", C.c_int32), ("fast_path", C.c_int32),
                ("perturb_scale", C.c_int32), ("graph_sweeps", C.c_int32),
                ("class_merge_kib", C.c_int32), ("small_tiles", C.c_int32), ("serial_mma", C.c_int32),
                ("termination", C.c_int32), ("wide_min_width", C.c_int32), ("wide_lanes", C.c_int32),
                ("fused_average", C.c_int32), ("persistent", C.c_int32), ("reserved", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("n_vars", C.c_int64), ("n_rows", C.c_int64), ("n_bdds", C.c_int64), ("n_pairs", C.c_int64),
                ("n_nodes", C.c_int64), ("n_fixed", C.c_int64), ("n_free", C.c_int64), ("n_tiles", C.c_int64),
                ("n_slots", C.c_int64), ("max_layers", C.c_int64), ("max_width", C.c_int64),
                ("lb_offset", C.c_double), ("n_reg_tiles", C.c_int64), ("n_reg_mixed_tiles", C.c_int64),
                ("n_reg_launches", C.c_int64), ("n_wide_tiles", C.c_int64), ("node_words", C.c_int64),
                ("n_fused_vars", C.c_int64), ("persist_tiles", C.c_int64)]


class PoolInfo(C.Structure):
    _fields_ = [("state", C.c_int32), ("error", C.c_int32), ("iters", C.c_int32), ("n_iter", C.c_int32),
                ("n_vars", C.c_int64), ("n_pairs", C.c_int64), ("steps", C.c_int64), ("lb_free", C.c_double),
                ("lb_cert", C.c_double), ("max_residual", C.c_double), ("workspace_bytes", C.c_uint64),
                ("rounded", C.c_int32), ("round_status", C.c_int32), ("rounds", C.c_int32), ("reserved_", C.c_int32),
                ("ub", C.c_double)]


_lib = None


def lib():
    """Load libbddmma.so (built by ``paper_2111_10270_amd.build``); raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2111_10270_amd.build.build()")
        # torch first: the library then binds to the HIP runtime torch has
        # loaded (same soname), so both work on one runtime instance; loaded
        # the other way round, torch's device allocations are invisible to
        # the library's runtime
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        P, i32, i64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        sig = {
            "bddmma_options_default": [P], "bddmma_create": [P, P], "bddmma_destroy": [P],
            "bddmma_load_ilp": [P, i64, P, i64, P, P, P, P, P], "bddmma_get_stats": [P, P],
            "bddmma_workspace_bytes": [P, P], "bddmma_bind": [P, P, C.c_size_t, P], "bddmma_bind_static": [P, P],
            "bddmma_reset": [P],
            "bddmma_run_dual": [P, i32, P], "bddmma_run_sweeps": [P, i32], "bddmma_lower_bound": [P, P, P, P],
            "bddmma_lb_history": [P, P, i64, P], "bddmma_num_pairs": [P, P], "bddmma_get_pairs": [P, P, P],
            "bddmma_get_fixed": [P, P], "bddmma_get_multipliers": [P, P, P], "bddmma_get_state": [P, P, P, P],
            "bddmma_set_state": [P, P, P, P], "bddmma_min_marginals": [P, P], "bddmma_round_primal": [P, P, P, P],
            "bddmma_save_state": [P, P, P], "bddmma_load_state": [P, P, C.c_size_t],
            "bddmma_profile": [P, C.c_int], "bddmma_kernel_time": [P, C.c_int, P, P], "bddmma_last_error": [],
            "bddmma_load_batch": [P, i64, P, P, i64, P, i64, P, P, P, P, P], "bddmma_num_instances": [P, P],
            "bddmma_batch_bounds": [P, P, P, P], "bddmma_batch_round": [P, P, P, P, P],
            "bddmma_pool_create": [P, i32, i32, i32, P], "bddmma_pool_bind": [P, P, C.c_size_t, P],
            "bddmma_pool_submit": [P, i64, P, i64, P, P, P, P, P, i32, P],
            "bddmma_pool_submit_loaded": [P, P, i32, P], "bddmma_pool_step": [P, i32, P, P],
            "bddmma_pool_wait_compiled": [P], "bddmma_pool_poll": [P, i64, P],
            "bddmma_pool_result": [P, i64, P, P, P, P], "bddmma_pool_release": [P, i64], "bddmma_pool_destroy": [P],
            "bddmma_pool_get_counters": [P, P], "bddmma_run_serial": [P, i32, P], "bddmma_pool_primal": [P, i64, P],
            "bddmma_autotune": [P, i64, P, i64, P, P, P, P, P, P, C.c_size_t, P, i32, P, P],
            "bddmma_encode_rows": [i64, P, i64, P, P, P, P, P, i64, P, P, P, P, P, P, P, P, P, P],
            "bddmma_stream_probe": [P, P, i64, i32, P],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.bddmma_destroy.restype = None
        L.bddmma_pool_destroy.restype = None
        L.bddmma_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _check(rc):
    if rc != OK:
        raise BddmmaError(rc, lib().bddmma_last_error().decode())
    return rc


def stream_probe(a, b, stream=None):
    """bddmma_stream_probe on two contiguous device tensors of one floating
    dtype and size, asynchronous on `stream` (default: the current stream)"""
    import torch
    if a.dtype != b.dtype or a.dtype not in (torch.float32, torch.float64) or a.numel() != b.numel():
        raise ValueError("stream_probe: two float32 or two float64 tensors of one size")
    if not (a.is_cuda and b.is_cuda and a.is_contiguous() and b.is_contiguous()):
        raise ValueError("stream_probe: contiguous device tensors")
    st = stream if stream is not None else torch.cuda.current_stream(a.device)
    _check(lib().bddmma_stream_probe(C.c_void_p(a.data_ptr()), C.c_void_p(b.data_ptr()), a.numel(),
                                     a.element_size(), C.c_void_p(st.cuda_stream)))


def default_options(**kw) -> Options:
    o = Options()
    _check(lib().bddmma_options_default(C.byref(o)))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def encode_rows(ilp, max_states: int = 4096):
    """ILP with every row of more than max_states partial-sum values replaced by
    a binary adder network (bddmma_encode_rows); -> (ILP, rows replaced).  The
    first ilp.n_vars variables are the original ones."""
    from . import instances
    arrs = [np.ascontiguousarray(ilp.costs, dtype=np.float64), np.ascontiguousarray(ilp.row_ptr, dtype=np.int64),
            np.ascontiguousarray(ilp.col, dtype=np.int32), np.ascontiguousarray(ilp.coef, dtype=np.int32),
            np.ascontiguousarray(ilp.sense, dtype=np.int8), np.ascontiguousarray(ilp.rhs, dtype=np.int64)]
    nv, nr, nnz, ne = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64()
    args = [ilp.n_vars, _p(arrs[0]), ilp.n_rows] + [_p(a) for a in arrs[1:]] + [int(max_states)]
    _check(lib().bddmma_encode_rows(*args, C.byref(nv), C.byref(nr), C.byref(nnz), C.byref(ne),
                                    None, None, None, None, None, None))
    out = [np.zeros(nv.value), np.zeros(nr.value + 1, dtype=np.int64), np.zeros(nnz.value, dtype=np.int32),
           np.zeros(nnz.value, dtype=np.int32), np.zeros(nr.value, dtype=np.int8), np.zeros(nr.value, dtype=np.int64)]
    _check(lib().bddmma_encode_rows(*args, C.byref(nv), C.byref(nr), C.byref(nnz), C.byref(ne),
                                    *[_p(a) for a in out]))
    enc = instances.ILP(nv.value, out[0], out[1], out[2], out[3], out[4], out[5], name=ilp.name + "_enc",
                        meta={"n_original_vars": ilp.n_vars})
    return enc, ne.value


def autotune(ilp, sweeps: int = 64, slack: float = 2.0, device="cuda", stream=None, **options):
    """fastest launch-schedule options for this ILP (bddmma_autotune), timed in
    a device buffer of slack x the default workspace; -> (Options, us per sweep)"""
    import torch
    base = default_options(**options)
    nbytes = int(Solver(ilp, **options).workspace_bytes() * slack) + (1 << 20)
    buf = torch.empty(nbytes, dtype=torch.uint8, device=device)
    st = stream if stream is not None else torch.cuda.current_stream(buf.device)
    arrs = [np.ascontiguousarray(ilp.costs, dtype=np.float64), np.ascontiguousarray(ilp.row_ptr, dtype=np.int64),
            np.ascontiguousarray(ilp.col, dtype=np.int32), np.ascontiguousarray(ilp.coef, dtype=np.int32),
            np.ascontiguousarray(ilp.sense, dtype=np.int8), np.ascontiguousarray(ilp.rhs, dtype=np.int64)]
    best, us = Options(), C.c_double()
    _check(lib().bddmma_autotune(C.byref(base), ilp.n_vars, _p(arrs[0]), ilp.n_rows, *[_p(a) for a in arrs[1:]],
                                 C.c_void_p(buf.data_ptr()), buf.numel(), C.c_void_p(st.cuda_stream), int(sweeps),
                                 C.byref(best), C.byref(us)))
    return best, us.value


class Solver:
    """One ILP (or a batch of independent ILPs, given as a list) on one
    device: load (host) -> bind (device workspace) -> solve."""

    def __init__(self, ilp, **options):
        L = lib()
        self._destroy = L.bddmma_destroy   # kept for __del__, which may run after module teardown
        self._h = C.c_void_p()
        self.options = default_options(**options)
        _check(L.bddmma_create(C.byref(self.options), C.byref(self._h)))
        batch = isinstance(ilp, (list, tuple))
        if batch:
            from . import instances
            ilp = instances.concat(ilp)
        self.ilp = ilp
        arrs = [np.ascontiguousarray(ilp.costs, dtype=np.float64), np.ascontiguousarray(ilp.row_ptr, dtype=np.int64),
                np.ascontiguousarray(ilp.col, dtype=np.int32), np.ascontiguousarray(ilp.coef, dtype=np.int32),
                np.ascontiguousarray(ilp.sense, dtype=np.int8), np.ascontiguousarray(ilp.rhs, dtype=np.int64)]
        if batch:
            nv = np.ascontiguousarray(ilp.meta["inst_vars"], dtype=np.int64)
            nr = np.ascontiguousarray(ilp.meta["inst_rows"], dtype=np.int64)
            _check(L.bddmma_load_batch(self._h, len(nv), _p(nv), _p(nr), ilp.n_vars, _p(arrs[0]), ilp.n_rows,
                                       *[_p(a) for a in arrs[1:]]))
        else:
            _check(L.bddmma_load_ilp(self._h, ilp.n_vars, _p(arrs[0]), ilp.n_rows, *[_p(a) for a in arrs[1:]]))
        n = C.c_int64()
        _check(L.bddmma_num_instances(self._h, C.byref(n)))
        self.n_inst = n.value
        st = Stats()
        _check(L.bddmma_get_stats(self._h, C.byref(st)))
        self.stats = st
        self.workspace = None
        self.stream = None

    def __del__(self, _finalizing=sys.is_finalizing):
        h = getattr(self, "_h", None)
        if h is None or not h.value or _finalizing():
            return   # at interpreter exit the process releases everything
        self._destroy(h)
        self._h = None

    # ---- device binding ----
    def workspace_bytes(self) -> int:
        n = C.c_size_t()
        _check(lib().bddmma_workspace_bytes(self._h, C.byref(n)))
        return n.value

    def bind(self, device="cuda", stream=None):
        import torch
        nbytes = self.workspace_bytes()
        self.workspace = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.workspace.device)
        _check(lib().bddmma_bind(self._h, C.c_void_p(self.workspace.data_ptr()), self.workspace.numel(),
                                 C.c_void_p(self.stream.cuda_stream)))
        return self

    def bind_static(self, device="cuda", stream=None):
        """bind to the library's static device workspace (no allocation);
        the current device of `device` is the one whose copy is bound"""
        import torch
        dev = torch.device(device)
        torch.cuda.set_device(dev)
        self.workspace = None
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        _check(lib().bddmma_bind_static(self._h, C.c_void_p(self.stream.cuda_stream)))
        return self

    # ---- Alg. 1 ----
    def reset(self):
        _check(lib().bddmma_reset(self._h))

    def run_dual(self, n_iter: int) -> int:
        done = C.c_int32()
        _check(lib().bddmma_run_dual(self._h, int(n_iter), C.byref(done)))
        return done.value

    def run_serial(self, n_iter: int) -> np.ndarray:
        """serial min-marginal averaging (ablation); bound after every sweep"""
        out = np.zeros(2 * max(int(n_iter), 0))
        _check(lib().bddmma_run_serial(self._h, int(n_iter), _p(out) if n_iter > 0 else None))
        return out

    def run_sweeps(self, n: int):
        _check(lib().bddmma_run_sweeps(self._h, int(n)))

    def lower_bound(self):
        a, b, c = C.c_double(), C.c_double(), C.c_double()
        _check(lib().bddmma_lower_bound(self._h, C.byref(a), C.byref(b), C.byref(c)))
        return a.value, b.value, c.value

    def lb_history(self) -> np.ndarray:
        n = C.c_int64()
        _check(lib().bddmma_lb_history(self._h, None, 0, C.byref(n)))
        out = np.zeros(n.value)
        _check(lib().bddmma_lb_history(self._h, _p(out), n.value, C.byref(n)))
        return out

    # ---- structure and state ----
    @property
    def n_pairs(self) -> int:
        return int(self.stats.n_pairs)

    def pairs(self):
        pv = np.zeros(self.n_pairs, dtype=np.int32)
        pr = np.zeros(self.n_pairs, dtype=np.int32)
        _check(lib().bddmma_get_pairs(self._h, _p(pv), _p(pr)))
        return pv, pr

    def fixed(self):
        f = np.zeros(self.ilp.n_vars, dtype=np.int8)
        _check(lib().bddmma_get_fixed(self._h, _p(f)))
        return f

    def multipliers(self):
        lam = np.zeros(self.n_pairs)
        mm = np.zeros(self.n_pairs)
        _check(lib().bddmma_get_multipliers(self._h, _p(lam), _p(mm)))
        return lam, mm

    def get_state(self):
        lam = np.zeros(self.n_pairs)
        mm = np.zeros(self.n_pairs)
        avg = np.zeros(self.ilp.n_vars)
        _check(lib().bddmma_get_state(self._h, _p(lam), _p(mm), _p(avg)))
        return lam, mm, avg

    def set_state(self, lam=None, mm=None, avg=None):
        conv = [None if a is None else np.ascontiguousarray(a, dtype=np.float64) for a in (lam, mm, avg)]
        _check(lib().bddmma_set_state(self._h, *[_p(a) for a in conv]))

    def min_marginals(self):
        out = np.zeros(self.n_pairs)
        _check(lib().bddmma_min_marginals(self._h, _p(out)))
        return out

    # ---- Alg. 2 ----
    def round_primal(self):
        x = np.zeros(self.ilp.n_vars, dtype=np.uint8)
        ub, rounds = C.c_double(), C.c_int32()
        rc = lib().bddmma_round_primal(self._h, _p(x), C.byref(ub), C.byref(rounds))
        if rc not in (OK, NOT_CONVERGED):
            _check(rc)
        return dict(rc=rc, x=x, ub=ub.value, rounds=rounds.value)

    # ---- batches ----
    def batch_bounds(self):
        """per-instance (lb_free, lb_cert, max_residual) arrays"""
        out = [np.zeros(self.n_inst) for _ in range(3)]
        _check(lib().bddmma_batch_bounds(self._h, *[_p(a) for a in out]))
        return tuple(out)

    def batch_round(self):
        """per-instance Alg. 2: dict(status, rounds, ub, x)"""
        x = np.zeros(self.ilp.n_vars, dtype=np.uint8)
        ub = np.full(self.n_inst, np.nan)
        rounds = np.zeros(self.n_inst, dtype=np.int32)
        status = np.zeros(self.n_inst, dtype=np.int32)
        _check(lib().bddmma_batch_round(self._h, _p(x), _p(ub), _p(rounds), _p(status)))
        return dict(status=status, rounds=rounds, ub=ub, x=x)

    # ---- checkpoint ----
    def save_state(self) -> bytes:
        n = C.c_size_t()
        _check(lib().bddmma_save_state(self._h, None, C.byref(n)))
        buf = (C.c_char * n.value)()
        _check(lib().bddmma_save_state(self._h, buf, C.byref(n)))
        return bytes(buf)

    def load_state(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        _check(lib().bddmma_load_state(self._h, buf, len(blob)))

    # ---- profiling ----
    def profile(self, enable=True, stride: int = 1):
        _check(lib().bddmma_profile(self._h, int(stride) if enable else 0))

    def kernel_time(self, kernel: int):
        n, ms = C.c_int64(), C.c_double()
        _check(lib().bddmma_kernel_time(self._h, int(kernel), C.byref(n), C.byref(ms)))
        return n.value, ms.value


class PoolCounters(C.Structure):
    _fields_ = [("steps", C.c_int64), ("assemblies", C.c_int64), ("admitted", C.c_int64), ("retired", C.c_int64),
                ("image_ms", C.c_double), ("merge_ms", C.c_double), ("bind_ms", C.c_double), ("run_ms", C.c_double),
                ("bounds_ms", C.c_double), ("retire_ms", C.c_double), ("round_ms", C.c_double),
                ("batch_capacity", C.c_uint64),
                ("image_capacity", C.c_uint64), ("image_free", C.c_uint64)]


class Pool:
    """Serving pool (continuous batching): submit ILPs at any time, step the
    resident batch, poll each ticket; see bddmma_pool_* in the header."""

    def __init__(self, max_active: int = 16, host_threads: int = 0, keep_multipliers: bool = True,
                 round: bool = False, **options):
        self._destroy = lib().bddmma_pool_destroy   # kept for __del__
        self._h = C.c_void_p()
        self.options = default_options(**options)
        flags = (POOL_KEEP_MULTIPLIERS if keep_multipliers else 0) | (POOL_ROUND if round else 0)
        _check(lib().bddmma_pool_create(C.byref(self.options), int(max_active), int(host_threads), flags,
                                        C.byref(self._h)))
        self.arena = None
        self.stream = None

    def __del__(self, _finalizing=sys.is_finalizing):
        h = getattr(self, "_h", None)
        if h is None or not h.value or _finalizing():
            return   # at interpreter exit the process releases everything
        self._destroy(h)
        self._h = None

    def bind(self, nbytes: int, device="cuda", stream=None):
        import torch
        self.arena = torch.empty(int(nbytes), dtype=torch.uint8, device=device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.arena.device)
        _check(lib().bddmma_pool_bind(self._h, C.c_void_p(self.arena.data_ptr()), self.arena.numel(),
                                      C.c_void_p(self.stream.cuda_stream)))
        return self

    def submit(self, ilp, n_iter: int) -> int:
        arrs = [np.ascontiguousarray(ilp.costs, dtype=np.float64), np.ascontiguousarray(ilp.row_ptr, dtype=np.int64),
                np.ascontiguousarray(ilp.col, dtype=np.int32), np.ascontiguousarray(ilp.coef, dtype=np.int32),
                np.ascontiguousarray(ilp.sense, dtype=np.int8), np.ascontiguousarray(ilp.rhs, dtype=np.int64)]
        t = C.c_int64()
        _check(lib().bddmma_pool_submit(self._h, ilp.n_vars, _p(arrs[0]), ilp.n_rows, *[_p(a) for a in arrs[1:]],
                                        int(n_iter), C.byref(t)))
        return t.value

    def submit_loaded(self, solver: "Solver", n_iter: int) -> int:
        """hand over a loaded, unbound Solver (it is emptied: the pool owns it now)"""
        h, solver._h = solver._h, None
        t = C.c_int64()
        _check(lib().bddmma_pool_submit_loaded(self._h, h, int(n_iter), C.byref(t)))
        return t.value

    def step(self, iters: int):
        """-> (members after retirement, retired by this step)"""
        a, r = C.c_int32(), C.c_int32()
        _check(lib().bddmma_pool_step(self._h, int(iters), C.byref(a), C.byref(r)))
        return a.value, r.value

    def wait_compiled(self):
        _check(lib().bddmma_pool_wait_compiled(self._h))

    def poll(self, ticket: int) -> dict:
        i = PoolInfo()
        _check(lib().bddmma_pool_poll(self._h, int(ticket), C.byref(i)))
        return {k: getattr(i, k) for k, _ in PoolInfo._fields_}

    def result(self, ticket: int, multipliers: bool = True):
        """-> (lambda + omega M, M, pair_var, pair_row) of a retired instance
        (lambda and M are None with multipliers=False)"""
        n = self.poll(ticket)["n_pairs"]
        lam, mm = (np.zeros(n), np.zeros(n)) if multipliers else (None, None)
        pv, pr = np.zeros(n, dtype=np.int32), np.zeros(n, dtype=np.int32)
        _check(lib().bddmma_pool_result(self._h, int(ticket), _p(lam), _p(mm), _p(pv), _p(pr)))
        return lam, mm, pv, pr

    def primal(self, ticket: int) -> np.ndarray:
        """rounded point of a retired instance (pool created with round=True)"""
        x = np.zeros(self.poll(ticket)["n_vars"], dtype=np.uint8)
        _check(lib().bddmma_pool_primal(self._h, int(ticket), _p(x)))
        return x

    def release(self, ticket: int):
        _check(lib().bddmma_pool_release(self._h, int(ticket)))

    def counters(self) -> dict:
        c = PoolCounters()
        _check(lib().bddmma_pool_get_counters(self._h, C.byref(c)))
        return {k: getattr(c, k) for k, _ in PoolCounters._fields_}

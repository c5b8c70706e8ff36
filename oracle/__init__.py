"""ctypes front end of the FP64 CPU reference implementation in ``oracle.c``.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg.  The solver product never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

OK, INVALID, INFEASIBLE, NOMEM, NOT_CONVERGED = 0, -1, -2, -3, -4


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` with gcc (FP64, no contraction)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-ffp-contract=off", "-fPIC", "-fopenmp",
                               "-shared", SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = C.CDLL(LIB)
        P = C.c_void_p
        d, i, ll, ull = C.c_double, C.c_int, C.c_longlong, C.c_ulonglong
        L.or_create.restype = P
        L.or_create.argtypes = [ll, P, ll, P, P, P, P, P, d]
        L.or_destroy.argtypes = [P]
        L.or_status.argtypes = [P]
        L.or_lb_offset.restype = d
        L.or_lb_offset.argtypes = [P]
        L.or_sizes.argtypes = [P, P, P, P]
        L.or_pairs.argtypes = [P, P, P]
        L.or_fixed.argtypes = [P, P]
        L.or_get.argtypes = [P, P, P, P]
        L.or_set.argtypes = [P, P, P, P]
        L.or_energies.argtypes = [P, P]
        L.or_bdd_nodes.argtypes = [P, i, P, P, P, P]
        L.or_bdd_sp.argtypes = [P, i, P, P, P, P]
        L.or_init.argtypes = [P]
        L.or_set_threads.argtypes = [P, i]
        L.or_sweep.argtypes = [P, i, i]
        L.or_sweep_subset.argtypes = [P, i, i, ll, P]
        L.or_average.argtypes = [P]
        L.or_lb_free.restype = d
        L.or_lb_free.argtypes = [P]
        L.or_lb_cert.restype = d
        L.or_lb_cert.argtypes = [P, P]
        L.or_terminate.argtypes = [P]
        L.or_run_dual.argtypes = [P, i, P]
        L.or_run_serial.argtypes = [P, i, P]
        L.or_set_termination.argtypes = [P, i]
        L.or_rng_u01.restype = d
        L.or_rng_u01.argtypes = [ull, ull, ull]
        L.or_perturb.argtypes = [P, i, d, d, ull, P, i]
        L.or_round.argtypes = [P, d, d, i, i, d, ull, i, P, P, P, P]
        L.or_count_violated.restype = ll
        L.or_count_violated.argtypes = [P, P]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


class Oracle:
    """One ILP loaded into the reference implementation (presolve + BDDs)."""

    def __init__(self, ilp, omega: float = 0.5, threads: int = 1):
        L = lib()
        self.ilp = ilp
        self.omega = float(omega)
        self._keep = [np.ascontiguousarray(ilp.costs, dtype=np.float64),
                      np.ascontiguousarray(ilp.row_ptr, dtype=np.int64),
                      np.ascontiguousarray(ilp.col, dtype=np.int32),
                      np.ascontiguousarray(ilp.coef, dtype=np.int32),
                      np.ascontiguousarray(ilp.sense, dtype=np.int8),
                      np.ascontiguousarray(ilp.rhs, dtype=np.int64)]
        c, rp, col, coef, sense, rhs = self._keep
        self._destroy = L.or_destroy
        self.h = L.or_create(ilp.n_vars, _p(c), ilp.n_rows, _p(rp), _p(col), _p(coef), _p(sense),
                             _p(rhs), self.omega)
        self.status = L.or_status(self.h)
        self.set_threads(threads)
        nb, np_, nn = C.c_longlong(), C.c_longlong(), C.c_longlong()
        if self.status == OK:
            L.or_sizes(self.h, C.byref(nb), C.byref(np_), C.byref(nn))
        self.n_bdds, self.n_pairs, self.n_nodes = nb.value, np_.value, nn.value

    def __del__(self):
        # the destroy function is kept on the object: at interpreter exit the
        # module globals may already be gone
        if getattr(self, "h", None) and getattr(self, "_destroy", None):
            self._destroy(self.h)
            self.h = None

    def set_threads(self, n: int):
        """host threads of the loops over BDDs and variables (results do not
        depend on it)"""
        self.threads = max(1, int(n))
        lib().or_set_threads(self.h, self.threads)

    # ---- structure ----
    def pairs(self):
        pv = np.zeros(self.n_pairs, dtype=np.int32)
        pr = np.zeros(self.n_pairs, dtype=np.int32)
        lib().or_pairs(self.h, _p(pv), _p(pr))
        return pv, pr

    def fixed(self):
        f = np.zeros(self.ilp.n_vars, dtype=np.int8)
        lib().or_fixed(self.h, _p(f))
        return f

    def lb_offset(self) -> float:
        return lib().or_lb_offset(self.h)

    def bdd_nodes(self, j: int):
        n = lib().or_bdd_nodes(self.h, j, None, None, None, None)
        layer = np.zeros(n, dtype=np.int32)
        state = np.zeros(n, dtype=np.int64)
        lo = np.zeros(n, dtype=np.int32)
        hi = np.zeros(n, dtype=np.int32)
        lib().or_bdd_nodes(self.h, j, _p(layer), _p(state), _p(lo), _p(hi))
        return dict(layer=layer, state=state, lo=lo, hi=hi)

    def bdd_sp(self, j: int):
        n = lib().or_bdd_nodes(self.h, j, None, None, None, None)
        F = np.zeros(n)
        B = np.zeros(n)
        tf, tb = C.c_double(), C.c_double()
        lib().or_bdd_sp(self.h, j, _p(F), _p(B), C.byref(tf), C.byref(tb))
        return F, B, tf.value, tb.value

    # ---- state ----
    def get(self):
        lam = np.zeros(self.n_pairs)
        mm = np.zeros(self.n_pairs)
        avg = np.zeros(self.ilp.n_vars)
        lib().or_get(self.h, _p(lam), _p(mm), _p(avg))
        return lam, mm, avg

    def set(self, lam=None, mm=None, avg=None):
        conv = [None if a is None else np.ascontiguousarray(a, dtype=np.float64) for a in (lam, mm, avg)]
        lib().or_set(self.h, *[None if a is None else _p(a) for a in conv])

    def energies(self):
        E = np.zeros(self.n_bdds)
        lib().or_energies(self.h, _p(E))
        return E

    # ---- Alg. 1 ----
    def init(self):
        lib().or_init(self.h)

    def sweep(self, direction: int, update: bool = True):
        lib().or_sweep(self.h, int(direction), int(bool(update)))

    def sweep_subset(self, direction: int, bdds, update: bool = True):
        sel = np.ascontiguousarray(bdds, dtype=np.int64)
        lib().or_sweep_subset(self.h, int(direction), int(bool(update)), sel.size, _p(sel))

    def average(self):
        lib().or_average(self.h)

    def lb_free(self) -> float:
        return lib().or_lb_free(self.h)

    def lb_cert(self):
        r = C.c_double()
        v = lib().or_lb_cert(self.h, C.byref(r))
        return v, r.value

    def terminate(self):
        lib().or_terminate(self.h)

    def set_termination(self, mode: int):
        """0: lambda + omega M-bar (default), 1: lambda + (omega/|J_i|) sum_k M-bar_ik"""
        lib().or_set_termination(self.h, int(mode))

    def run_dual(self, n_iter: int):
        hist = np.zeros(2 * max(n_iter, 0))
        lib().or_run_dual(self.h, int(n_iter), _p(hist) if n_iter > 0 else None)
        return hist

    def run_serial(self, n_iter: int):
        """serial min-marginal averaging from the terminated multipliers; sum_j E^j
        + offset after every sweep"""
        hist = np.zeros(2 * max(n_iter, 0))
        lib().or_run_serial(self.h, int(n_iter), _p(hist) if n_iter > 0 else None)
        return hist

    def full_mm(self):
        """min-marginal differences at fixed multipliers (no update)"""
        self.sweep(0, update=False)
        return self.get()[1]

    # ---- Alg. 2 ----
    def perturb(self, rnd: int, delta: float, tau: float = 0.0, seed: int = 0, flag=None, scale: int = 0):
        f = None if flag is None else np.ascontiguousarray(flag, dtype=np.uint8)
        lib().or_perturb(self.h, int(rnd), float(delta), float(tau), C.c_ulonglong(seed),
                         None if f is None else _p(f), int(scale))

    def round(self, delta0=1.0, alpha=1.2, reopt_iters=5, max_rounds=200, tau=0.0, seed=0, scale=0):
        x = np.zeros(self.ilp.n_vars, dtype=np.uint8)
        ub, rounds = C.c_double(), C.c_int()
        hist = np.zeros(max_rounds + 1, dtype=np.int64)
        rc = lib().or_round(self.h, float(delta0), float(alpha), int(reopt_iters), int(max_rounds),
                            float(tau), C.c_ulonglong(seed), int(scale), _p(x), C.byref(ub), C.byref(rounds),
                            _p(hist))
        return dict(rc=rc, x=x, ub=ub.value, rounds=rounds.value,
                    conflicts=hist[:rounds.value + 1].copy())

    def count_violated(self, x) -> int:
        x = np.ascontiguousarray(x, dtype=np.uint8)
        return int(lib().or_count_violated(self.h, _p(x)))


def rng_u01(seed: int, rnd: int, i: int) -> float:
    return lib().or_rng_u01(seed, rnd, i)

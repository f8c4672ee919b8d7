"""QIEO oracle -- TEST INFRASTRUCTURE ONLY.

A plain CPU implementation of the QIEO generation (QIP -> Evaluation ->
DetermineElite -> CIP, Sec. III-B and Fig. 1 of the paper) plus exact knapsack
references (brute force, dynamic programming, Dantzig bound).  The arithmetic
lives in ``qieo_oracle.c`` and ``knapsack_exact.c``; this module compiles them
with gcc (FP contraction off, no fast-math) and wraps them with ctypes.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the GPU library
and never calls it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = [os.path.join(_HERE, "qieo_oracle.c"), os.path.join(_HERE, "knapsack_exact.c")]
_LIB = os.path.join(_HERE, "liboracle.so")

# -ffp-contract=off: every a*b+c stays two rounded operations (the GPU side is
# built the same way); x86-64 does binary32 in SSE registers, so there is no
# excess precision.
CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
          "-fno-fast-math", "-fno-unsafe-math-optimizations", "-fopenmp"]


def build(force: bool = True) -> str:
    """Compile liboracle.so next to the sources (always, when force)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", *CFLAGS, "-o", tmp, *_SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, i64, u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
        L.oracle_new.restype = P
        L.oracle_new.argtypes = [i32, i32, P, P, i64, u64, i64]
        L.oracle_new_f64.restype = P
        L.oracle_new_f64.argtypes = [i32, i32, P, P, i64, u64, i64]
        L.oracle_cip_gene_f64.restype = ctypes.c_int
        L.oracle_cip_gene_f64.argtypes = [P, P, ctypes.c_int]
        L.oracle_get_amplitudes_f64.argtypes = [P, P, P]
        L.oracle_set_amplitudes_f64.argtypes = [P, P, P]
        L.oracle_free.argtypes = [P]
        L.oracle_set_threads.argtypes = [P, ctypes.c_int]
        for name in ("oracle_qip", "oracle_fe", "oracle_de", "oracle_cip", "oracle_generation"):
            getattr(L, name).argtypes = [P]
        L.oracle_run.argtypes = [P, i64]
        L.oracle_converged.restype = ctypes.c_int
        L.oracle_converged.argtypes = [P, ctypes.c_int]
        L.oracle_run_until_converged.restype = i64
        L.oracle_run_until_converged.argtypes = [P, i64, ctypes.c_int]
        L.oracle_philox4x32_10.argtypes = [P, P, P]
        L.oracle_uniform.restype = ctypes.c_float
        L.oracle_uniform.argtypes = [u64, i64, i64, i64]
        L.oracle_cip_gene.restype = ctypes.c_int
        L.oracle_cip_gene.argtypes = [P, P, ctypes.c_int]
        L.oracle_row_generation.argtypes = [u64, i64, i64, i64, P, P, i64, P, P, P, P,
                                            ctypes.c_int, P, P]
        L.oracle_row_generation_f64.argtypes = L.oracle_row_generation.argtypes
        L.oracle_get_amplitudes.argtypes = [P, P, P]
        L.oracle_set_amplitudes.argtypes = [P, P, P]
        L.oracle_get_alleles.argtypes = [P, P]
        L.oracle_get_rows.argtypes = [P, i64, i64, P, P, P]
        L.oracle_set_alleles.argtypes = [P, P]
        L.oracle_get_fitness.argtypes = [P, P, P, P]
        L.oracle_set_fitness.argtypes = [P, P]
        L.oracle_generation_index.restype = i64
        L.oracle_generation_index.argtypes = [P]
        L.oracle_elite.restype = i64
        L.oracle_elite.argtypes = [P]
        L.oracle_get_best.argtypes = [P, P, P]
        L.knap_bruteforce.restype = i64
        L.knap_bruteforce.argtypes = [ctypes.c_int, P, P, i64, i64, P]
        L.knap_all_fitness.restype = ctypes.c_int
        L.knap_all_fitness.argtypes = [ctypes.c_int, P, P, i64, i64, P]
        L.knap_dp.restype = i64
        L.knap_dp.argtypes = [ctypes.c_int, P, P, i64]
        L.knap_lp_bound.restype = ctypes.c_double
        L.knap_lp_bound.argtypes = [ctypes.c_int, P, P, i64]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def philox4x32_10(ctr, key) -> np.ndarray:
    """Philox4x32-10 of one 128-bit counter under one 64-bit key."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().oracle_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def uniform(seed: int, t: int, c: int, i: int) -> float:
    """The 24-bit uniform draw of gene i of chromosome c at generation t."""
    return float(lib().oracle_uniform(seed, t, c, i))


def cip_gene(alpha: float, beta: float, tgt: int):
    """CIP on one gene; returns (alpha', beta', rotated)."""
    a = np.array([alpha], dtype=np.float32)
    b = np.array([beta], dtype=np.float32)
    r = lib().oracle_cip_gene(_ptr(a), _ptr(b), int(tgt))
    return np.float32(a[0]), np.float32(b[0]), bool(r)


def cip_gene_f64(alpha: float, beta: float, tgt: int):
    """CIP on one gene in binary64; returns (alpha', beta', rotated)."""
    a = np.array([alpha], dtype=np.float64)
    b = np.array([beta], dtype=np.float64)
    r = lib().oracle_cip_gene_f64(_ptr(a), _ptr(b), int(tgt))
    return float(a[0]), float(b[0]), bool(r)


def row_generation(seed: int, t: int, c: int, v, w, capacity: int, alpha, beta,
                   x_prev=None, elite_prev=None, below_elite: bool = False,
                   precision: int = 32):
    """Chromosome c's part of generation t: CIP of t-1 toward the elite's
    alleles when the chromosome scored below the elite, then QIP and
    Evaluation of t.  alpha, beta: its amplitudes as t-1 observed them
    (binary32, or binary64 with precision=64).  Returns (alpha', beta',
    alleles of t, fitness, profit, weight)."""
    v = np.ascontiguousarray(v, dtype=np.int32)
    w = np.ascontiguousarray(w, dtype=np.int32)
    ng = v.size
    dt = np.float64 if precision == 64 else np.float32
    a = np.array(alpha, dtype=dt, copy=True).reshape(ng)
    b = np.array(beta, dtype=dt, copy=True).reshape(ng)
    xp = np.zeros(ng, np.uint8) if x_prev is None else np.ascontiguousarray(x_prev, np.uint8)
    ep = np.zeros(ng, np.uint8) if elite_prev is None else np.ascontiguousarray(elite_prev,
                                                                                 np.uint8)
    x = np.zeros(ng, np.uint8)
    out = np.zeros(3, np.int64)
    fn = lib().oracle_row_generation_f64 if precision == 64 else lib().oracle_row_generation
    fn(seed & (2**64 - 1), int(t), int(c), ng, _ptr(v), _ptr(w), int(capacity), _ptr(a),
       _ptr(b), _ptr(xp), _ptr(ep), int(bool(below_elite)), _ptr(x), _ptr(out))
    return a, b, x, int(out[0]), int(out[1]), int(out[2])


def row_generation_inplace(seed: int, t: int, c: int, v, w, capacity: int, alpha, beta,
                           x_prev, elite_prev, below_elite: bool, x_out):
    """row_generation on caller-owned contiguous arrays (int32 v, w; float32
    or float64 alpha, beta updated in place; uint8 x_prev, elite_prev, x_out),
    without copies; returns (fitness, profit, weight).  Thread-safe."""
    out = np.zeros(3, np.int64)
    fn = (lib().oracle_row_generation_f64 if alpha.dtype == np.float64
          else lib().oracle_row_generation)
    fn(seed & (2**64 - 1), int(t), int(c), v.size, _ptr(v), _ptr(w), int(capacity),
       _ptr(alpha), _ptr(beta), _ptr(x_prev), _ptr(elite_prev), int(bool(below_elite)),
       _ptr(x_out), _ptr(out))
    return int(out[0]), int(out[1]), int(out[2])


@dataclass
class Best:
    has_best: bool
    fitness: int
    profit: int
    weight: int
    generation: int
    chromosome: int
    bits: np.ndarray


class Oracle:
    """One QIEO population on the CPU (see qieo_oracle.c for the readings)."""

    def __init__(self, v, w, capacity: int, n_pop: int, seed: int,
                 lam: int = 1, threads: int = 1, precision: int = 32):
        self.v = np.ascontiguousarray(v, dtype=np.int32)
        self.w = np.ascontiguousarray(w, dtype=np.int32)
        self.ng = int(self.v.size)
        self.np_ = int(n_pop)
        self.capacity = int(capacity)
        self.seed = int(seed)
        self.precision = int(precision)
        new = lib().oracle_new_f64 if self.precision == 64 else lib().oracle_new
        h = new(self.ng, self.np_, _ptr(self.v), _ptr(self.w),
                self.capacity, self.seed & (2**64 - 1), int(lam))
        if not h:
            raise ValueError("oracle_new rejected the instance")
        self._h = ctypes.c_void_p(h)
        lib().oracle_set_threads(self._h, int(threads))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().oracle_free(h)
            self._h = None

    # steps (Fig. 1 order)
    def qip(self):
        lib().oracle_qip(self._h)

    def fe(self):
        lib().oracle_fe(self._h)

    def de(self):
        lib().oracle_de(self._h)

    def cip(self):
        lib().oracle_cip(self._h)

    def generation(self):
        lib().oracle_generation(self._h)

    def run(self, n: int):
        lib().oracle_run(self._h, int(n))

    def converged(self, window: int) -> bool:
        return bool(lib().oracle_converged(self._h, int(window)))

    def run_until_converged(self, n: int, window: int) -> int:
        """At most n generations, stopping once converged; returns how many ran."""
        return int(lib().oracle_run_until_converged(self._h, int(n), int(window)))

    # state
    @property
    def t(self) -> int:
        return int(lib().oracle_generation_index(self._h))

    @property
    def elite(self) -> int:
        return int(lib().oracle_elite(self._h))

    def amplitudes(self):
        dt = np.float64 if self.precision == 64 else np.float32
        a = np.empty((self.np_, self.ng), dtype=dt)
        b = np.empty((self.np_, self.ng), dtype=dt)
        get = lib().oracle_get_amplitudes_f64 if self.precision == 64 else lib().oracle_get_amplitudes
        get(self._h, _ptr(a), _ptr(b))
        return a, b

    def set_amplitudes(self, alpha, beta):
        dt = np.float64 if self.precision == 64 else np.float32
        a = np.ascontiguousarray(alpha, dtype=dt).reshape(self.np_, self.ng)
        b = np.ascontiguousarray(beta, dtype=dt).reshape(self.np_, self.ng)
        put = lib().oracle_set_amplitudes_f64 if self.precision == 64 else lib().oracle_set_amplitudes
        put(self._h, _ptr(a), _ptr(b))

    def rows(self, row0: int, n_rows: int):
        """Amplitudes (alpha, beta) and alleles of rows [row0, row0 + n_rows)."""
        if row0 < 0 or n_rows < 0 or row0 + n_rows > self.np_:
            raise ValueError("rows outside the population")
        dt = np.float64 if self.precision == 64 else np.float32
        a = np.empty((n_rows, self.ng), dtype=dt)
        b = np.empty((n_rows, self.ng), dtype=dt)
        x = np.empty((n_rows, self.ng), dtype=np.uint8)
        lib().oracle_get_rows(self._h, int(row0), int(n_rows), _ptr(a), _ptr(b), _ptr(x))
        return a, b, x

    def alleles(self) -> np.ndarray:
        x = np.empty((self.np_, self.ng), dtype=np.uint8)
        lib().oracle_get_alleles(self._h, _ptr(x))
        return x

    def set_alleles(self, x):
        a = np.ascontiguousarray(x, dtype=np.uint8).reshape(self.np_, self.ng)
        lib().oracle_set_alleles(self._h, _ptr(a))

    def fitness(self):
        f = np.empty(self.np_, dtype=np.int64)
        P = np.empty(self.np_, dtype=np.int64)
        W = np.empty(self.np_, dtype=np.int64)
        lib().oracle_get_fitness(self._h, _ptr(f), _ptr(P), _ptr(W))
        return f, P, W

    def set_fitness(self, fit):
        f = np.ascontiguousarray(fit, dtype=np.int64)
        lib().oracle_set_fitness(self._h, _ptr(f))

    def best(self) -> Best:
        out = np.zeros(6, dtype=np.int64)
        bits = np.zeros(self.ng, dtype=np.uint8)
        lib().oracle_get_best(self._h, _ptr(out), _ptr(bits))
        return Best(bool(out[0]), int(out[1]), int(out[2]), int(out[3]),
                    int(out[4]), int(out[5]), bits)


# exact knapsack references -------------------------------------------------

def knap_bruteforce(v, w, capacity: int, lam: int = 1):
    v = np.ascontiguousarray(v, dtype=np.int32)
    w = np.ascontiguousarray(w, dtype=np.int32)
    m = ctypes.c_uint64(0)
    f = lib().knap_bruteforce(int(v.size), _ptr(v), _ptr(w), int(capacity), int(lam),
                              ctypes.byref(m))
    return int(f), int(m.value)


def knap_all_fitness(v, w, capacity: int, lam: int = 1) -> np.ndarray:
    v = np.ascontiguousarray(v, dtype=np.int32)
    w = np.ascontiguousarray(w, dtype=np.int32)
    out = np.empty(1 << v.size, dtype=np.int64)
    if lib().knap_all_fitness(int(v.size), _ptr(v), _ptr(w), int(capacity), int(lam), _ptr(out)):
        raise ValueError("too many items for enumeration")
    return out


def knap_dp(v, w, capacity: int) -> int:
    v = np.ascontiguousarray(v, dtype=np.int32)
    w = np.ascontiguousarray(w, dtype=np.int32)
    return int(lib().knap_dp(int(v.size), _ptr(v), _ptr(w), int(capacity)))


def knap_lp_bound(v, w, capacity: int) -> float:
    v = np.ascontiguousarray(v, dtype=np.int32)
    w = np.ascontiguousarray(w, dtype=np.int32)
    return float(lib().knap_lp_bound(int(v.size), _ptr(v), _ptr(w), int(capacity)))

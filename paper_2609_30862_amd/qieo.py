"""ctypes binding of libqieo (include/qieo.h).

Argument marshalling only: every step of the QIEO generation runs in the HIP
kernels of libqieo.so.  The functions keep the C names; ``Instance`` is a
small owner object around a handle.  There is no CPU fallback: if the shared
library is missing or fails to load, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libqieo.so")

QIEO_OK = 0
QIEO_EINVAL = -1
QIEO_EOVERFLOW = -2
QIEO_ENOMEM = -3
QIEO_EDEVICE = -4
QIEO_EAGAIN = -5
QIEO_ESTATE = -6

# qieo_best_noalloc: largest instance (items) its static staging holds
QIEO_BEST_NOALLOC_MAX_ITEMS = 1 << 23

PATH_LAUNCHES = 0
PATH_LDS = 1
PATH_GLOBAL = 2
PATH_ONCHIP = 3

PIPELINE_FUSED = 0
PIPELINE_UNFUSED = 1
PIPELINE_UNFUSED_FE_DE = 2
PIPELINE_UNFUSED_HOST_DE = 3
PIPELINE_CHROMOSOME = 4
STAGES = ("fused", "cip", "qip", "fe", "de")


class QieoError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str):
        super().__init__("%s failed (%d, %s): %s" % (where, code, _strerror(code), detail))
        self.code = code


class qieo_item(ctypes.Structure):
    _fields_ = [("profit", ctypes.c_int32), ("weight", ctypes.c_int32)]


class qieo_result(ctypes.Structure):
    _fields_ = [("fitness", ctypes.c_int32), ("profit", ctypes.c_int32),
                ("weight", ctypes.c_int32), ("feasible", ctypes.c_int32),
                ("generation", ctypes.c_int64), ("chromosome", ctypes.c_int64)]


class qieo_problem(ctypes.Structure):
    _fields_ = [("items", ctypes.c_void_p), ("n_items", ctypes.c_int32),
                ("capacity", ctypes.c_int32), ("n_pop", ctypes.c_int32),
                ("seed", ctypes.c_uint64)]


class qieo_server_cfg(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("max_resident", ctypes.c_int32),
                ("gens_per_iter", ctypes.c_int32), ("convergence_window", ctypes.c_int32)]


class qieo_server_stats(ctypes.Structure):
    _fields_ = [("queued", ctypes.c_int64), ("resident", ctypes.c_int64),
                ("admitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("failed", ctypes.c_int64), ("iterations", ctypes.c_int64),
                ("gene_updates", ctypes.c_double), ("pool_bytes", ctypes.c_size_t),
                ("pool_used", ctypes.c_size_t), ("peak_resident", ctypes.c_int64),
                ("peak_pool_used", ctypes.c_size_t), ("error", ctypes.c_int32)]


class qieo_tune_result(ctypes.Structure):
    _fields_ = [("rows_per_block", ctypes.c_int32), ("waves_per_block", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("candidates", ctypes.c_int32),
                ("ms_per_generation", ctypes.c_double),
                ("worst_ms_per_generation", ctypes.c_double)]


class qieo_class_tune(ctypes.Structure):
    _fields_ = [("shape_class", ctypes.c_int32), ("rows", ctypes.c_int32),
                ("max_chunks", ctypes.c_int32), ("rows_per_block", ctypes.c_int32),
                ("waves_per_block", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("default_rows_per_block", ctypes.c_int32),
                ("default_waves_per_block", ctypes.c_int32), ("default_flags", ctypes.c_int32),
                ("candidates", ctypes.c_int32), ("ms_per_generation", ctypes.c_double),
                ("default_ms_per_generation", ctypes.c_double)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class qieo_dev_ctx(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", ctypes.c_void_p),
                ("stream", ctypes.c_void_p)]


class DeviceContext:
    """A caller's device allocator and stream for a handle (qieo_dev_ctx).

    alloc(nbytes) -> device pointer as an int (0 when it cannot allocate) and
    free(ptr) replace hipMalloc / hipFree for the handle's device memory
    (both or neither); stream is a hipStream_t (int) on which the handle
    orders all its work, or None.  The object keeps the C callbacks alive
    and must outlive every handle created with it."""

    def __init__(self, alloc=None, free=None, stream: int | None = None):
        if (alloc is None) != (free is None):
            raise ValueError("alloc and free go together")
        self._alloc = ALLOC_FN(lambda n, user: alloc(int(n)) or None) if alloc else ALLOC_FN(0)
        self._free = FREE_FN(lambda p, user: free(int(p))) if free else FREE_FN(0)
        self.struct = qieo_dev_ctx(self._alloc, self._free, None,
                                   ctypes.c_void_p(stream) if stream else None)


def _ctx_ref(ctx: DeviceContext | None, stream: int | None):
    """(reference to a qieo_dev_ctx or None, object to keep alive)."""
    if ctx is None and stream is not None:
        ctx = DeviceContext(stream=stream)
    return (ctypes.byref(ctx.struct) if ctx is not None else None), ctx


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libqieo.so is not built (expected at %s); run "
                          "__graft_entry__.build()" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    P, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    H = ctypes.c_void_p
    L.qieo_create.restype = ctypes.c_int
    L.qieo_create.argtypes = [P, i32, i32, i32, u64, ctypes.POINTER(H)]
    L.qieo_create_f64.restype = ctypes.c_int
    L.qieo_create_f64.argtypes = [P, i32, i32, i32, u64, ctypes.POINTER(qieo_dev_ctx),
                                  ctypes.POINTER(H)]
    L.qieo_get_kernel_flags.restype = ctypes.c_int
    L.qieo_get_kernel_flags.argtypes = [H, ctypes.POINTER(i32)]
    L.qieo_state_size.restype = ctypes.c_int
    L.qieo_state_size.argtypes = [H, ctypes.POINTER(ctypes.c_size_t)]
    L.qieo_export_state.restype = ctypes.c_int
    L.qieo_export_state.argtypes = [H, P, ctypes.c_size_t]
    L.qieo_import_state.restype = ctypes.c_int
    L.qieo_import_state.argtypes = [H, P, ctypes.c_size_t]
    L.qieo_export_rows_f64.restype = ctypes.c_int
    L.qieo_export_rows_f64.argtypes = [H, i32, i32, P, P, P, P, P, P, ctypes.POINTER(i32)]
    L.qieo_create_ex.restype = ctypes.c_int
    L.qieo_create_ex.argtypes = [P, i32, i32, i32, u64, ctypes.POINTER(qieo_dev_ctx),
                                 ctypes.POINTER(H)]
    for n in ("qieo_step", "qieo_step_async"):
        getattr(L, n).restype = ctypes.c_int
        getattr(L, n).argtypes = [H, i32]
    L.qieo_sync.restype = ctypes.c_int
    L.qieo_sync.argtypes = [H]
    L.qieo_best.restype = ctypes.c_int
    L.qieo_best.argtypes = [H, ctypes.POINTER(qieo_result), P, ctypes.c_size_t]
    L.qieo_best_noalloc.restype = ctypes.c_int
    L.qieo_best_noalloc.argtypes = [H, ctypes.POINTER(qieo_result), P, ctypes.c_size_t]
    L.qieo_generations.restype = ctypes.c_int
    L.qieo_generations.argtypes = [H, ctypes.POINTER(i64)]
    L.qieo_autotune.restype = ctypes.c_int
    L.qieo_autotune.argtypes = [i32, i32, P, i32, i32, ctypes.POINTER(qieo_tune_result)]
    L.qieo_tune_db_save.restype = ctypes.c_int
    L.qieo_tune_db_save.argtypes = [ctypes.c_char_p]
    L.qieo_tune_db_load.restype = ctypes.c_int
    L.qieo_tune_db_load.argtypes = [ctypes.c_char_p]
    L.qieo_tune_db_clear.restype = None
    L.qieo_tune_db_clear.argtypes = []
    L.qieo_set_graph.restype = ctypes.c_int
    L.qieo_set_graph.argtypes = [H, i32]
    L.qieo_set_persistent.restype = ctypes.c_int
    L.qieo_set_persistent.argtypes = [H, i32]
    L.qieo_get_call_path.restype = ctypes.c_int
    L.qieo_get_call_path.argtypes = [H, ctypes.POINTER(i32)]
    L.qieo_set_barrier_timeout.restype = ctypes.c_int
    L.qieo_set_barrier_timeout.argtypes = [H, i64]
    L.qieo_set_pipeline.restype = ctypes.c_int
    L.qieo_set_pipeline.argtypes = [H, i32]
    L.qieo_stage_time.restype = ctypes.c_int
    L.qieo_stage_time.argtypes = [H, P, P, ctypes.c_int]
    L.qieo_set_convergence.restype = ctypes.c_int
    L.qieo_set_convergence.argtypes = [H, i32]
    L.qieo_converged.restype = ctypes.c_int
    L.qieo_converged.argtypes = [H, ctypes.POINTER(i32), ctypes.POINTER(i64)]
    L.qieo_batch_set_convergence.restype = ctypes.c_int
    L.qieo_batch_set_convergence.argtypes = [H, i32]
    L.qieo_batch_converged.restype = ctypes.c_int
    L.qieo_batch_converged.argtypes = [H, i32, ctypes.POINTER(i32), ctypes.POINTER(i64)]
    L.qieo_export_rows.restype = ctypes.c_int
    L.qieo_export_rows.argtypes = [H, i32, i32, P, P, P, P, P, P, ctypes.POINTER(i32)]
    L.qieo_destroy.restype = None
    L.qieo_destroy.argtypes = [H]
    L.qieo_strerror.restype = ctypes.c_char_p
    L.qieo_strerror.argtypes = [ctypes.c_int]
    L.qieo_last_error.restype = ctypes.c_char_p
    L.qieo_last_error.argtypes = []
    L.qieo_version.restype = ctypes.c_char_p
    L.qieo_version.argtypes = []
    L.qieo_set_tile.restype = ctypes.c_int
    L.qieo_set_tile.argtypes = [H, i32, i32]
    L.qieo_set_kernel_flags.restype = ctypes.c_int
    L.qieo_set_kernel_flags.argtypes = [H, i32]
    L.qieo_get_tile.restype = ctypes.c_int
    L.qieo_get_tile.argtypes = [H, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.qieo_set_timing.restype = ctypes.c_int
    L.qieo_set_timing.argtypes = [H, ctypes.c_int]
    L.qieo_kernel_time.restype = ctypes.c_int
    L.qieo_kernel_time.argtypes = [H, ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_double),
                                   ctypes.c_int]
    L.qieo_batch_create.restype = ctypes.c_int
    L.qieo_batch_create.argtypes = [ctypes.POINTER(qieo_problem), i32,
                                    ctypes.POINTER(qieo_dev_ctx), ctypes.POINTER(H)]
    for n in ("qieo_batch_step", "qieo_batch_step_async"):
        getattr(L, n).restype = ctypes.c_int
        getattr(L, n).argtypes = [H, P]
    L.qieo_batch_sync.restype = ctypes.c_int
    L.qieo_batch_sync.argtypes = [H]
    L.qieo_batch_size.restype = ctypes.c_int
    L.qieo_batch_size.argtypes = [H, ctypes.POINTER(i32)]
    L.qieo_batch_generations.restype = ctypes.c_int
    L.qieo_batch_generations.argtypes = [H, i32, ctypes.POINTER(i64)]
    L.qieo_batch_best.restype = ctypes.c_int
    L.qieo_batch_best.argtypes = [H, i32, ctypes.POINTER(qieo_result), P, ctypes.c_size_t]
    L.qieo_batch_export_rows.restype = ctypes.c_int
    L.qieo_batch_export_rows.argtypes = [H, i32, i32, i32, P, P, P, P, P, P,
                                         ctypes.POINTER(i32)]
    L.qieo_batch_set_tile.restype = ctypes.c_int
    L.qieo_batch_set_tile.argtypes = [H, i32, i32, i32]
    L.qieo_batch_set_persistent.restype = ctypes.c_int
    L.qieo_batch_set_persistent.argtypes = [H, i32]
    L.qieo_batch_set_segment_order.restype = ctypes.c_int
    L.qieo_batch_set_segment_order.argtypes = [H, i32]
    L.qieo_server_set_onchip.restype = ctypes.c_int
    L.qieo_server_set_onchip.argtypes = [H, i32]
    L.qieo_batch_set_onchip.restype = ctypes.c_int
    L.qieo_batch_set_onchip.argtypes = [H, i32]
    L.qieo_batch_onchip_launches.restype = ctypes.c_int
    L.qieo_batch_onchip_launches.argtypes = [H, ctypes.POINTER(i32)]
    L.qieo_batch_set_barrier_timeout.restype = ctypes.c_int
    L.qieo_batch_set_barrier_timeout.argtypes = [H, i64]
    L.qieo_batch_autotune.restype = ctypes.c_int
    L.qieo_batch_autotune.argtypes = [H, ctypes.c_int32, ctypes.POINTER(qieo_class_tune),
                                      ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    L.qieo_batch_set_graph.restype = ctypes.c_int
    L.qieo_batch_set_graph.argtypes = [H, i32]
    L.qieo_batch_destroy.restype = None
    L.qieo_batch_destroy.argtypes = [H]
    L.qieo_server_create.restype = ctypes.c_int
    L.qieo_server_create.argtypes = [ctypes.POINTER(qieo_server_cfg),
                                     ctypes.POINTER(qieo_dev_ctx), ctypes.POINTER(H)]
    L.qieo_server_submit.restype = ctypes.c_int
    L.qieo_server_submit.argtypes = [H, ctypes.POINTER(qieo_problem), i32,
                                     ctypes.POINTER(ctypes.c_uint64)]
    for n in ("qieo_server_poll", "qieo_server_wait"):
        getattr(L, n).restype = ctypes.c_int
        getattr(L, n).argtypes = [H, ctypes.c_uint64, ctypes.POINTER(qieo_result), P,
                                  ctypes.c_size_t, ctypes.POINTER(i64)]
    L.qieo_server_release.restype = ctypes.c_int
    L.qieo_server_release.argtypes = [H, ctypes.c_uint64]
    L.qieo_server_get_stats.restype = ctypes.c_int
    L.qieo_server_get_stats.argtypes = [H, ctypes.POINTER(qieo_server_stats)]
    L.qieo_server_destroy.restype = None
    L.qieo_server_destroy.argtypes = [H]
    return L


lib = _load()


def _strerror(code: int) -> str:
    return lib.qieo_strerror(code).decode()


def qieo_last_error() -> str:
    return lib.qieo_last_error().decode()


def qieo_version() -> str:
    return lib.qieo_version().decode()


def _check(rc: int, where: str):
    if rc != QIEO_OK:
        raise QieoError(rc, where, qieo_last_error())


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def items_array(values, weights):
    v = np.ascontiguousarray(values, dtype=np.int64)
    w = np.ascontiguousarray(weights, dtype=np.int64)
    if v.shape != w.shape or v.ndim != 1:
        raise ValueError("values and weights must be 1-D arrays of equal length")
    if v.size and (v.min() < np.iinfo(np.int32).min or v.max() > np.iinfo(np.int32).max or
                   w.min() < np.iinfo(np.int32).min or w.max() > np.iinfo(np.int32).max):
        raise ValueError("values and weights must fit in int32")
    arr = np.empty((v.size, 2), dtype=np.int32)
    arr[:, 0] = v
    arr[:, 1] = w
    return arr


# --- C-named entry points ---------------------------------------------------

def qieo_autotune(n_items: int, n_pop: int, trial_generations: int = 3, values=None,
                  weights=None, capacity: int = 0) -> dict:
    """Times every work shape on a scratch population and records the best."""
    it = None if values is None else items_array(values, weights)
    r = qieo_tune_result()
    _check(lib.qieo_autotune(int(n_items), int(n_pop), _ptr(it), int(capacity),
                             int(trial_generations), ctypes.byref(r)), "qieo_autotune")
    return {name: getattr(r, name) for name, _ in qieo_tune_result._fields_}


def qieo_tune_db_save(path: str):
    _check(lib.qieo_tune_db_save(path.encode()), "qieo_tune_db_save")


def qieo_tune_db_load(path: str) -> int:
    n = lib.qieo_tune_db_load(path.encode())
    _check(min(n, 0), "qieo_tune_db_load")
    return n


def qieo_tune_db_clear():
    lib.qieo_tune_db_clear()


def qieo_create(items: np.ndarray, n_items: int, capacity: int, n_pop: int, seed: int,
                stream: int | None = None, precision: int = 32,
                ctx: DeviceContext | None = None):
    """items: int32 array [n_items, 2] of (profit, weight).  Returns a handle."""
    h = ctypes.c_void_p()
    ref, _ = _ctx_ref(ctx, stream)
    if precision == 64:
        rc = lib.qieo_create_f64(_ptr(items), n_items, capacity, n_pop, seed & (2**64 - 1), ref,
                                 ctypes.byref(h))
    elif ref is None:
        rc = lib.qieo_create(_ptr(items), n_items, capacity, n_pop, seed & (2**64 - 1),
                             ctypes.byref(h))
    else:
        rc = lib.qieo_create_ex(_ptr(items), n_items, capacity, n_pop, seed & (2**64 - 1),
                                ref, ctypes.byref(h))
    _check(rc, "qieo_create")
    return h


def qieo_step(h, n_generations: int):
    _check(lib.qieo_step(h, int(n_generations)), "qieo_step")


def qieo_step_async(h, n_generations: int):
    _check(lib.qieo_step_async(h, int(n_generations)), "qieo_step_async")


def qieo_sync(h):
    _check(lib.qieo_sync(h), "qieo_sync")


def qieo_best(h, n_items: int | None = None):
    r = qieo_result()
    bits = None
    if n_items is not None:
        bits = np.zeros((n_items + 31) // 32, dtype=np.uint32)
    _check(lib.qieo_best(h, ctypes.byref(r), _ptr(bits), 0 if bits is None else bits.size),
           "qieo_best")
    return r, bits


def qieo_best_noalloc(h, n_items: int | None = None):
    """qieo_best through the library's static staging buffer (no allocation)."""
    r = qieo_result()
    bits = None
    if n_items is not None:
        bits = np.zeros((n_items + 31) // 32, dtype=np.uint32)
    _check(lib.qieo_best_noalloc(h, ctypes.byref(r), _ptr(bits),
                                 0 if bits is None else bits.size), "qieo_best_noalloc")
    return r, bits


def qieo_generations(h) -> int:
    t = ctypes.c_int64()
    _check(lib.qieo_generations(h, ctypes.byref(t)), "qieo_generations")
    return int(t.value)


def qieo_destroy(h):
    if h:
        lib.qieo_destroy(h)


@dataclass
class Result:
    fitness: int
    profit: int
    weight: int
    feasible: bool
    generation: int
    chromosome: int
    bits: np.ndarray | None = None

    def alleles(self, n_items: int) -> np.ndarray:
        """The best string as 0/1 bytes."""
        b = np.unpackbits(self.bits.view(np.uint8), bitorder="little")
        return b[:n_items].astype(np.uint8)


class Instance:
    """One resident QIEO population (owner of a libqieo handle)."""

    def __init__(self, values, weights, capacity: int, n_pop: int, seed: int,
                 stream: int | None = None, precision: int = 32,
                 ctx: DeviceContext | None = None):
        self.items = items_array(values, weights)
        self.n_items = int(self.items.shape[0])
        self.n_pop = int(n_pop)
        self.capacity = int(capacity)
        self.seed = int(seed)
        self.precision = int(precision)
        self._ctx = ctx
        self._h = qieo_create(self.items, self.n_items, self.capacity, self.n_pop, self.seed,
                              stream, self.precision, ctx)

    def close(self):
        h = getattr(self, "_h", None)
        self._h = None
        if h and lib is not None:
            try:
                lib.qieo_destroy(h)
            except Exception:       # interpreter shutdown: the library may be gone
                pass

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def handle(self):
        return self._h

    def step(self, n: int):
        qieo_step(self._h, n)

    def step_async(self, n: int):
        qieo_step_async(self._h, n)

    def sync(self):
        qieo_sync(self._h)

    @property
    def generations(self) -> int:
        return qieo_generations(self._h)

    def best(self) -> Result:
        r, bits = qieo_best(self._h, self.n_items)
        return Result(r.fitness, r.profit, r.weight, bool(r.feasible), r.generation,
                      r.chromosome, bits)

    def export_state(self) -> np.ndarray:
        """Snapshot of the whole state (uint8 array) for import_state."""
        n = ctypes.c_size_t(0)
        _check(lib.qieo_state_size(self._h, ctypes.byref(n)), "qieo_state_size")
        buf = np.empty(n.value, dtype=np.uint8)
        _check(lib.qieo_export_state(self._h, _ptr(buf), buf.nbytes), "qieo_export_state")
        return buf

    def import_state(self, buf):
        """Continues from a snapshot taken by export_state on the same problem."""
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        _check(lib.qieo_import_state(self._h, _ptr(buf), buf.nbytes), "qieo_import_state")

    def export_rows(self, row0: int = 0, n_rows: int | None = None, amplitudes: bool = True,
                    alleles: bool = True):
        """State after the last completed generation (its CIP applied) for
        rows [row0, row0 + n_rows): dict of numpy arrays plus the elite."""
        if n_rows is None:
            n_rows = self.n_pop - row0
        ng = self.n_items
        dt = np.float64 if self.precision == 64 else np.float32
        a = np.empty((n_rows, ng), dt) if amplitudes else None
        b = np.empty((n_rows, ng), dt) if amplitudes else None
        x = np.empty((n_rows, ng), np.uint8) if alleles else None
        f = np.empty(n_rows, np.int32)
        p = np.empty(n_rows, np.int32)
        w = np.empty(n_rows, np.int32)
        e = ctypes.c_int32()
        fn = lib.qieo_export_rows_f64 if self.precision == 64 else lib.qieo_export_rows
        _check(fn(self._h, row0, n_rows, _ptr(a), _ptr(b), _ptr(x), _ptr(f), _ptr(p), _ptr(w),
                  ctypes.byref(e)), "qieo_export_rows")
        return dict(alpha=a, beta=b, alleles=x, fitness=f, profit=p, weight=w,
                    elite=int(e.value))

    def set_tile(self, rows_per_block: int = 0, waves_per_block: int = 0):
        _check(lib.qieo_set_tile(self._h, rows_per_block, waves_per_block), "qieo_set_tile")

    def set_convergence(self, window: int):
        _check(lib.qieo_set_convergence(self._h, int(window)), "qieo_set_convergence")

    def set_graph(self, enabled: bool):
        _check(lib.qieo_set_graph(self._h, int(bool(enabled))), "qieo_set_graph")

    def set_persistent(self, mode: int):
        _check(lib.qieo_set_persistent(self._h, int(mode)), "qieo_set_persistent")

    def set_barrier_timeout(self, microseconds: int):
        _check(lib.qieo_set_barrier_timeout(self._h, int(microseconds)),
               "qieo_set_barrier_timeout")

    def call_path(self) -> int:
        """PATH_* of the last step call (-1 before the first)."""
        p = ctypes.c_int32()
        _check(lib.qieo_get_call_path(self._h, ctypes.byref(p)), "qieo_get_call_path")
        return p.value

    def set_pipeline(self, pipeline: int):
        _check(lib.qieo_set_pipeline(self._h, int(pipeline)), "qieo_set_pipeline")

    def stage_time(self, reset: bool = False) -> dict:
        """{stage: (timed launches, total ms)} for fused, cip, qip, fe, de."""
        n = np.zeros(5, np.int64)
        ms = np.zeros(5, np.float64)
        _check(lib.qieo_stage_time(self._h, _ptr(n), _ptr(ms), int(reset)), "qieo_stage_time")
        return {k: (int(n[i]), float(ms[i])) for i, k in enumerate(STAGES)}

    def converged(self):
        """(converged, generation after which the run stopped or -1)."""
        c, g = ctypes.c_int32(), ctypes.c_int64()
        _check(lib.qieo_converged(self._h, ctypes.byref(c), ctypes.byref(g)), "qieo_converged")
        return bool(c.value), int(g.value)

    def set_kernel_flags(self, flags: int):
        _check(lib.qieo_set_kernel_flags(self._h, int(flags)), "qieo_set_kernel_flags")

    def kernel_flags(self) -> int:
        f = ctypes.c_int32()
        _check(lib.qieo_get_kernel_flags(self._h, ctypes.byref(f)), "qieo_get_kernel_flags")
        return int(f.value)

    def tile(self):
        r, s = ctypes.c_int32(), ctypes.c_int32()
        _check(lib.qieo_get_tile(self._h, ctypes.byref(r), ctypes.byref(s)), "qieo_get_tile")
        return int(r.value), int(s.value)

    def set_timing(self, enabled: bool):
        _check(lib.qieo_set_timing(self._h, int(bool(enabled))), "qieo_set_timing")

    def kernel_time(self, reset: bool = False):
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        _check(lib.qieo_kernel_time(self._h, ctypes.byref(n), ctypes.byref(ms), int(reset)),
               "qieo_kernel_time")
        return int(n.value), float(ms.value)


def _export(fn, n_items, n_pop, row0, n_rows, amplitudes, alleles, where):
    if n_rows is None:
        n_rows = n_pop - row0
    a = np.empty((n_rows, n_items), np.float32) if amplitudes else None
    b = np.empty((n_rows, n_items), np.float32) if amplitudes else None
    x = np.empty((n_rows, n_items), np.uint8) if alleles else None
    f = np.empty(n_rows, np.int32)
    p = np.empty(n_rows, np.int32)
    w = np.empty(n_rows, np.int32)
    e = ctypes.c_int32()
    _check(fn(row0, n_rows, _ptr(a), _ptr(b), _ptr(x), _ptr(f), _ptr(p), _ptr(w),
              ctypes.byref(e)), where)
    return dict(alpha=a, beta=b, alleles=x, fitness=f, profit=p, weight=w, elite=int(e.value))


class Batch:
    """Many resident populations advanced together (qieo_batch_*)."""

    def __init__(self, problems, stream: int | None = None, ctx: DeviceContext | None = None):
        """problems: iterable of (values, weights, capacity, n_pop, seed)."""
        self._items = []
        arr = (qieo_problem * len(problems))()
        self.shapes = []
        for k, (v, w, cap, n_pop, seed) in enumerate(problems):
            it = items_array(v, w)
            self._items.append(it)
            arr[k] = qieo_problem(it.ctypes.data, it.shape[0], int(cap), int(n_pop),
                                  int(seed) & (2**64 - 1))
            self.shapes.append((int(n_pop), int(it.shape[0]), int(cap)))
        h = ctypes.c_void_p()
        ref, self._ctx = _ctx_ref(ctx, stream)
        _check(lib.qieo_batch_create(arr, len(problems), ref, ctypes.byref(h)),
               "qieo_batch_create")
        self._h = h
        self.n = len(problems)

    def close(self):
        h = getattr(self, "_h", None)
        self._h = None
        if h and lib is not None:
            try:
                lib.qieo_batch_destroy(h)
            except Exception:
                pass

    def __del__(self):
        self.close()

    def _counts(self, gens):
        g = np.ascontiguousarray(np.broadcast_to(np.asarray(gens, dtype=np.int32), (self.n,)))
        return g

    def step(self, gens):
        g = self._counts(gens)
        _check(lib.qieo_batch_step(self._h, _ptr(g)), "qieo_batch_step")

    def step_async(self, gens):
        g = self._counts(gens)
        _check(lib.qieo_batch_step_async(self._h, _ptr(g)), "qieo_batch_step_async")

    def sync(self):
        _check(lib.qieo_batch_sync(self._h), "qieo_batch_sync")

    def generations(self, i: int) -> int:
        t = ctypes.c_int64()
        _check(lib.qieo_batch_generations(self._h, i, ctypes.byref(t)), "qieo_batch_generations")
        return int(t.value)

    def best(self, i: int) -> Result:
        r = qieo_result()
        ng = self.shapes[i][1]
        bits = np.zeros((ng + 31) // 32, dtype=np.uint32)
        _check(lib.qieo_batch_best(self._h, i, ctypes.byref(r), _ptr(bits), bits.size),
               "qieo_batch_best")
        return Result(r.fitness, r.profit, r.weight, bool(r.feasible), r.generation,
                      r.chromosome, bits)

    def export_rows(self, i: int, row0: int = 0, n_rows: int | None = None,
                    amplitudes: bool = True, alleles: bool = True):
        n_pop, ng, _ = self.shapes[i]
        fn = lambda *a: lib.qieo_batch_export_rows(self._h, i, *a)
        return _export(fn, ng, n_pop, row0, n_rows, amplitudes, alleles, "qieo_batch_export_rows")

    def set_tile(self, rows_per_block: int = 0, waves_per_block: int = 0, flags: int = 0):
        _check(lib.qieo_batch_set_tile(self._h, rows_per_block, waves_per_block, flags),
               "qieo_batch_set_tile")

    def set_graph(self, enabled: bool):
        _check(lib.qieo_batch_set_graph(self._h, int(bool(enabled))), "qieo_batch_set_graph")

    def autotune(self, trial_generations: int = 5) -> list:
        """qieo_batch_autotune: the tuned shape of every launch class (dicts)."""
        out = (qieo_class_tune * 8)()
        n = ctypes.c_int32()
        _check(lib.qieo_batch_autotune(self._h, int(trial_generations), out, 8, ctypes.byref(n)),
               "qieo_batch_autotune")
        return [{name: getattr(out[k], name) for name, _ in qieo_class_tune._fields_}
                for k in range(min(n.value, 8))]


    def set_convergence(self, window: int):
        _check(lib.qieo_batch_set_convergence(self._h, int(window)), "qieo_batch_set_convergence")

    def set_persistent(self, enabled: bool):
        _check(lib.qieo_batch_set_persistent(self._h, int(bool(enabled))),
               "qieo_batch_set_persistent")

    def set_segment_order(self, mode):
        """1 / True (default): members with rows of 8 or more chunks in
        segment order when the batch streams; 2: rows of 32 or more chunks
        only; 0 / False: row order for every member."""
        _check(lib.qieo_batch_set_segment_order(self._h, int(mode)),
               "qieo_batch_set_segment_order")

    def set_onchip(self, enabled: bool):
        """True (default): members of rows under 32 chunks that would run in
        row order run each call inside batched on-chip launches."""
        _check(lib.qieo_batch_set_onchip(self._h, int(bool(enabled))), "qieo_batch_set_onchip")

    def onchip_launches(self) -> int:
        n = ctypes.c_int32()
        _check(lib.qieo_batch_onchip_launches(self._h, ctypes.byref(n)),
               "qieo_batch_onchip_launches")
        return int(n.value)

    def set_barrier_timeout(self, microseconds: int):
        _check(lib.qieo_batch_set_barrier_timeout(self._h, int(microseconds)),
               "qieo_batch_set_barrier_timeout")

    def converged(self, i: int):
        c, g = ctypes.c_int32(), ctypes.c_int64()
        _check(lib.qieo_batch_converged(self._h, i, ctypes.byref(c), ctypes.byref(g)),
               "qieo_batch_converged")
        return bool(c.value), int(g.value)


class Server:
    """Continuous-batching request server (qieo_server_*)."""

    def __init__(self, hbm_budget_bytes: int, max_resident: int = 0, gens_per_iter: int = 0,
                 convergence_window: int = 0, stream: int | None = None,
                 ctx: DeviceContext | None = None):
        cfg = qieo_server_cfg(int(hbm_budget_bytes), int(max_resident), int(gens_per_iter),
                              int(convergence_window))
        h = ctypes.c_void_p()
        ref, self._ctx = _ctx_ref(ctx, stream)
        _check(lib.qieo_server_create(ctypes.byref(cfg), ref, ctypes.byref(h)),
               "qieo_server_create")
        self._h = h
        self._n_items = {}

    def close(self):
        h = getattr(self, "_h", None)
        self._h = None
        if h and lib is not None:
            try:
                lib.qieo_server_destroy(h)
            except Exception:
                pass

    def __del__(self):
        self.close()

    def set_onchip(self, enabled: bool):
        """True (default): residents run in batched on-chip launches where
        they fit; False: per-generation launches only."""
        _check(lib.qieo_server_set_onchip(self._h, int(bool(enabled))), "qieo_server_set_onchip")

    def submit(self, values, weights, capacity: int, n_pop: int, seed: int, n_gen: int) -> int:
        it = items_array(values, weights)
        prob = qieo_problem(it.ctypes.data, it.shape[0], int(capacity), int(n_pop),
                            int(seed) & (2**64 - 1))
        t = ctypes.c_uint64()
        _check(lib.qieo_server_submit(self._h, ctypes.byref(prob), int(n_gen), ctypes.byref(t)),
               "qieo_server_submit")
        self._n_items[int(t.value)] = it.shape[0]
        return int(t.value)

    def _result(self, fn, ticket):
        ng = self._n_items[ticket]
        r = qieo_result()
        bits = np.zeros((ng + 31) // 32, dtype=np.uint32)
        lat = ctypes.c_int64()
        rc = fn(self._h, ticket, ctypes.byref(r), _ptr(bits), bits.size, ctypes.byref(lat))
        if rc == QIEO_EAGAIN:
            return None
        _check(rc, "qieo_server_result")
        return Result(r.fitness, r.profit, r.weight, bool(r.feasible), r.generation,
                      r.chromosome, bits), int(lat.value)

    def poll(self, ticket: int):
        """(Result, latency_ns) when finished, None while pending."""
        return self._result(lib.qieo_server_poll, ticket)

    def wait(self, ticket: int):
        return self._result(lib.qieo_server_wait, ticket)

    def release(self, ticket: int):
        _check(lib.qieo_server_release(self._h, ticket), "qieo_server_release")
        self._n_items.pop(ticket, None)

    def stats(self) -> dict:
        st = qieo_server_stats()
        _check(lib.qieo_server_get_stats(self._h, ctypes.byref(st)), "qieo_server_get_stats")
        return {name: getattr(st, name) for name, _ in qieo_server_stats._fields_}

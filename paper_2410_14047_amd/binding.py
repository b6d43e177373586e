"""Thin ctypes binding of libimx.so (include/im.h).  Argument marshalling only:
every step of the method runs in the library's HIP kernels.

Function names mirror the C ABI (im_graph_load, im_sketch_build,
im_select_seeds, ...).  `stream` arguments take a hipStream_t as an int (for
example torch.cuda.current_stream().cuda_stream) or None for the null stream.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libimx.so")

IM_OK, IM_EINVAL, IM_ENOMEM, IM_EDEVICE, IM_ESTATE = range(5)
_STATUS = {1: "IM_EINVAL", 2: "IM_ENOMEM", 3: "IM_EDEVICE", 4: "IM_ESTATE"}


class IMError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class im_stats(ctypes.Structure):
    _fields_ = [
        ("build_sweeps", ctypes.c_int32),
        ("rebuilds", ctypes.c_int32),
        ("total_sweeps", ctypes.c_int64),
        ("cascade_levels", ctypes.c_int64),
        ("build_ms", ctypes.c_double),
        ("select_ms", ctypes.c_double),
        ("propagate_ms", ctypes.c_double),
        ("cascade_ms", ctypes.c_double),
        ("prop_launches", ctypes.c_int64),
        ("prop_kernel_ms", ctypes.c_double),
        ("prop_alg_bytes", ctypes.c_double),
        ("prop_tasks", ctypes.c_int64),
        ("prop_rows_read", ctypes.c_int64),
        ("prop_bytes_written", ctypes.c_int64),
        ("prop_arcs_scanned", ctypes.c_int64),
        ("prop_arcs_active", ctypes.c_int64),
        ("prop_sectors", ctypes.c_int64),
        ("prop_rows_visited", ctypes.c_int64),
        ("prop_rows_changed", ctypes.c_int64),
    ]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


# Every symbol declared in include/im.h.
EXPORTS = [
    "im_last_error", "im_version", "im_set_profiling", "im_graph_load", "im_graph_info", "im_graph_free",
    "im_sketch_build", "im_select_seeds", "im_select_seeds_until", "im_sketch_registers", "im_sketch_register_rows", "im_sketch_estimates",
    "im_sketch_stats", "im_sketch_sim_values", "im_sketch_free",
    "im_engine_create", "im_engine_submit", "im_engine_step", "im_engine_poll", "im_engine_result",
    "im_engine_info", "im_query_footprint", "im_engine_free", "im_select_seeds_batch",
    "im_engine_set_tuning", "im_engine_get_tuning", "im_set_allocator", "im_engine_counters",
    "im_select_seeds_noalloc",
]
_VOID = ("im_last_error", "im_graph_free", "im_sketch_free", "im_engine_free", "im_query_footprint")

_lib = None

_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)
# Every hook pair ever installed stays referenced for the life of the process:
# a buffer is returned to the hooks that allocated it (also after the hooks
# change), so a ctypes thunk must never be collected while such a buffer may
# still be freed.
_hooks_installed: list = []


def lib() -> ctypes.CDLL:
    """Load libimx.so.  Raises if the HIP library has not been built: there is no
    fallback implementation."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"HIP library missing: {LIB_PATH} (run __graft_entry__.build())")
        # One HIP runtime per process: PyTorch ships its own copy of the HIP
        # runtime, with the same soname as the system one this library links.
        # Loading PyTorch first makes the library bind to that copy, so the
        # two share one runtime, device context and stream namespace (torch
        # streams can be passed in).  Loaded the other way round, two
        # runtimes would coexist and the second one could not open the GPU.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
        L.im_last_error.argtypes = []
        L.im_last_error.restype = ctypes.c_char_p
        L.im_version.argtypes = [P, P]
        L.im_set_profiling.argtypes = [i32]
        L.im_engine_counters.argtypes = [P, P, P, P]
        L.im_set_allocator.argtypes = [_ALLOC_FN, _FREE_FN, P]
        L.im_graph_load.argtypes = [i64, i64, P, P, P, P, P]
        L.im_graph_info.argtypes = [P, P, P]
        L.im_graph_free.argtypes = [P]
        L.im_graph_free.restype = None
        L.im_sketch_build.argtypes = [P, i32, u64, P, P]
        L.im_select_seeds.argtypes = [P, i32, P, P, P, P, P]
        L.im_select_seeds_until.argtypes = [P, i32, i32, P, P]
        L.im_sketch_registers.argtypes = [P, P]
        L.im_sketch_register_rows.argtypes = [P, P, i32, P]
        L.im_sketch_estimates.argtypes = [P, P, P]
        L.im_sketch_stats.argtypes = [P, P]
        L.im_sketch_sim_values.argtypes = [P, P]
        L.im_sketch_free.argtypes = [P]
        L.im_sketch_free.restype = None
        L.im_engine_create.argtypes = [i32, u64, P, P]
        L.im_engine_submit.argtypes = [P, P, i32, u64, i32, P]
        L.im_engine_step.argtypes = [P, P]
        L.im_engine_poll.argtypes = [P, P, i32, P]
        L.im_engine_result.argtypes = [P, i64, P, P, P, P, P]
        L.im_engine_info.argtypes = [P, P, P, P, P]
        L.im_query_footprint.argtypes = [P, i32, i32]
        L.im_query_footprint.restype = u64
        L.im_engine_free.argtypes = [P]
        L.im_engine_free.restype = None
        L.im_select_seeds_batch.argtypes = [i32, P, P, P, P, P, P, P]
        L.im_engine_set_tuning.argtypes = [P, P]
        L.im_engine_get_tuning.argtypes = [P, P]
        L.im_select_seeds_noalloc.argtypes = [P, i32, u64, i32, P, P, P, P, P]
        for name in EXPORTS:
            if name not in _VOID:
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(st: int) -> None:
    if st != IM_OK:
        raise IMError(st, lib().im_last_error().decode(errors="replace"))


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _stream(stream) -> Optional[int]:
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):
        return int(stream.cuda_stream)
    return int(stream)


# ---------------------------------------------------------------- C-named wrappers

def im_graph_load(n: int, rowptr: np.ndarray, col: np.ndarray, p: np.ndarray, stream=None) -> ctypes.c_void_p:
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    p = np.ascontiguousarray(p, dtype=np.float32)
    if rowptr.shape[0] != n + 1:
        raise IMError(IM_EINVAL, "rowptr must have n+1 entries")
    m = int(col.shape[0])
    if p.shape[0] != m:
        raise IMError(IM_EINVAL, "p must have m entries")
    out = ctypes.c_void_p()
    _check(lib().im_graph_load(n, m, _p(rowptr), _p(col), _p(p), _stream(stream), ctypes.byref(out)))
    return out


def im_set_profiling(level: int) -> None:
    _check(lib().im_set_profiling(level))


def im_set_allocator(alloc=None, free=None) -> None:
    """Install device memory hooks: alloc(nbytes) -> int device pointer (0 on
    failure), free(ptr) -> None.  Both None restores hipMalloc/hipFree."""
    if (alloc is None) != (free is None):
        raise ValueError("give both hooks or neither")
    if alloc is None:
        _check(lib().im_set_allocator(_ALLOC_FN(), _FREE_FN(), None))
        return

    def _a(nbytes, ctx):
        try:
            return int(alloc(int(nbytes))) or None
        except Exception:  # an exception must not cross the C boundary
            return None

    def _f(ptr, ctx):
        try:
            free(int(ptr))
        except Exception:
            pass

    hooks = (_ALLOC_FN(_a), _FREE_FN(_f))
    _hooks_installed.append(hooks)
    _check(lib().im_set_allocator(hooks[0], hooks[1], None))


def use_torch_allocator(enable: bool = True, device: int = 0) -> None:
    """Make PyTorch's caching allocator own the library's device memory (graphs,
    sketches and engines created afterwards); enable=False restores hipMalloc."""
    if not enable:
        im_set_allocator()
        return
    import torch

    def _alloc(nbytes):
        return torch.cuda.caching_allocator_alloc(nbytes, device=device)

    def _free(ptr):
        torch.cuda.caching_allocator_delete(ptr)

    im_set_allocator(_alloc, _free)


def im_graph_free(g) -> None:
    lib().im_graph_free(g)


def im_sketch_build(g, J: int, seed: int, stream=None) -> ctypes.c_void_p:
    out = ctypes.c_void_p()
    _check(lib().im_sketch_build(g, J, seed & (2**64 - 1), _stream(stream), ctypes.byref(out)))
    return out


def im_select_seeds(s, K: int):
    seeds = np.zeros(K, dtype=np.int32)
    est = np.zeros(K, dtype=np.float64)
    T = np.zeros(K, dtype=np.uint64)
    spread = ctypes.c_double()
    stats = im_stats()
    _check(lib().im_select_seeds(s, K, _p(seeds), ctypes.byref(spread), _p(est), _p(T), ctypes.byref(stats)))
    return dict(seeds=seeds, spread=spread.value, est=est, T=T, stats=stats.as_dict())


def im_select_seeds_until(s, K: int, k_stop: int):
    """Picks before pick number k_stop (parity hook); returns (seeds, T) so far."""
    seeds = np.zeros(max(k_stop, 1), dtype=np.int32)
    T = np.zeros(max(k_stop, 1), dtype=np.uint64)
    _check(lib().im_select_seeds_until(s, K, k_stop, _p(seeds), _p(T)))
    return seeds[:k_stop], T[:k_stop]


def im_select_seeds_noalloc(g, J: int, seed: int, K: int, registers_dev: int, stream=None):
    """im_sketch_build + im_select_seeds without device allocation; the
    registers live in the caller's device buffer at address registers_dev
    (n*J bytes)."""
    seeds = np.zeros(K, dtype=np.int32)
    est = np.zeros(K, dtype=np.float64)
    spread = ctypes.c_double()
    _check(lib().im_select_seeds_noalloc(g, J, seed, K, ctypes.c_void_p(registers_dev), _p(seeds),
                                         ctypes.byref(spread), _p(est), _stream(stream)))
    return dict(seeds=seeds, spread=spread.value, est=est)


def im_sketch_registers(s, n: int, J: int) -> np.ndarray:
    M = np.zeros((n, J), dtype=np.uint8)
    _check(lib().im_sketch_registers(s, _p(M)))
    return M


def im_sketch_register_rows(s, rows, J: int) -> np.ndarray:
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    out = np.zeros((rows.size, J), dtype=np.uint8)
    _check(lib().im_sketch_register_rows(s, _p(rows), rows.size, _p(out)))
    return out


def im_sketch_estimates(s, n: int):
    Ju = np.zeros(n, dtype=np.uint32)
    Hu = np.zeros(n, dtype=np.uint64)
    _check(lib().im_sketch_estimates(s, _p(Ju), _p(Hu)))
    return Ju, Hu


def im_sketch_stats(s) -> dict:
    st = im_stats()
    _check(lib().im_sketch_stats(s, ctypes.byref(st)))
    return st.as_dict()


def im_sketch_sim_values(s, J: int) -> np.ndarray:
    X = np.zeros(J, dtype=np.uint32)
    _check(lib().im_sketch_sim_values(s, _p(X)))
    return X


def im_sketch_free(s) -> None:
    lib().im_sketch_free(s)


# ---------------------------------------------------------------- convenience handles

class Graph:
    """Device-resident graph (owns an im_graph handle)."""

    def __init__(self, n: int, rowptr, col, p, stream=None):
        self.n = int(n)
        self.m = int(len(col))
        self.handle = im_graph_load(self.n, rowptr, col, p, stream)

    @classmethod
    def from_graphgen(cls, g, stream=None) -> "Graph":
        return cls(g.n, g.rowptr, g.col, g.p, stream)

    def free(self) -> None:
        if self.handle:
            im_graph_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Sketch:
    """Sketches of a graph (owns an im_sketch handle)."""

    def __init__(self, graph: Graph, J: int, seed: int, stream=None):
        self.graph = graph
        self.J = int(J)
        self.seed = int(seed)
        self.handle = im_sketch_build(graph.handle, self.J, self.seed, stream)

    def select(self, K: int) -> dict:
        return im_select_seeds(self.handle, K)

    def select_until(self, K: int, k_stop: int):
        """Run the selection of K seeds up to pick k_stop and pause there
        (parity hook); select(K) finishes it.  Returns (seeds, T) so far."""
        return im_select_seeds_until(self.handle, K, k_stop)

    def registers(self) -> np.ndarray:
        return im_sketch_registers(self.handle, self.graph.n, self.J)

    def register_rows(self, rows) -> np.ndarray:
        return im_sketch_register_rows(self.handle, rows, self.J)

    def estimates(self):
        return im_sketch_estimates(self.handle, self.graph.n)

    def sim_values(self) -> np.ndarray:
        return im_sketch_sim_values(self.handle, self.J)

    def stats(self) -> dict:
        return im_sketch_stats(self.handle)

    def free(self) -> None:
        if self.handle:
            im_sketch_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


# ---------------------------------------------------------------- engines (batched / served queries)

class im_tuning(ctypes.Structure):
    _fields_ = [("group_first", ctypes.c_int32), ("group_rest", ctypes.c_int32),
                ("rounds_per_step", ctypes.c_int32), ("dense_div", ctypes.c_int32),
                ("use_graphs", ctypes.c_int32), ("grid_cap", ctypes.c_int32), ("tails", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


def im_query_footprint(g, J: int, K: int) -> int:
    return int(lib().im_query_footprint(g, J, K))


class Engine:
    """Many queries (graph, J, seed, K) advanced together by one native engine.
    submit() raises IMError with status IM_ENOMEM when the query does not fit the
    memory budget (nothing changes; retry after collecting results)."""

    def __init__(self, max_queries: int = 64, hbm_budget_bytes: int = 0, stream=None):
        out = ctypes.c_void_p()
        _check(lib().im_engine_create(max_queries, hbm_budget_bytes, _stream(stream), ctypes.byref(out)))
        self.handle = out
        self._K = {}

    def submit(self, graph: "Graph", J: int, seed: int, K: int) -> int:
        qid = ctypes.c_int64()
        _check(lib().im_engine_submit(self.handle, graph.handle, J, seed & (2**64 - 1), K, ctypes.byref(qid)))
        self._K[qid.value] = K
        return qid.value

    def step(self) -> int:
        n = ctypes.c_int32()
        _check(lib().im_engine_step(self.handle, ctypes.byref(n)))
        return n.value

    def poll(self) -> list:
        cap = max(1, len(self._K))
        ids = np.zeros(cap, dtype=np.int64)
        n = ctypes.c_int32()
        _check(lib().im_engine_poll(self.handle, _p(ids), cap, ctypes.byref(n)))
        return [int(x) for x in ids[: min(n.value, cap)]]

    def result(self, qid: int) -> dict:
        K = self._K[qid]
        seeds = np.zeros(K, dtype=np.int32)
        est = np.zeros(K, dtype=np.float64)
        T = np.zeros(K, dtype=np.uint64)
        spread = ctypes.c_double()
        stats = im_stats()
        _check(lib().im_engine_result(self.handle, qid, _p(seeds), ctypes.byref(spread), _p(est), _p(T),
                                      ctypes.byref(stats)))
        del self._K[qid]
        return dict(seeds=seeds, spread=spread.value, est=est, T=T, stats=stats.as_dict())

    def set_tuning(self, group_first: int = 0, group_rest: int = 0, rounds_per_step: int = 8,
                   dense_div: int = 16, use_graphs: int = 0, grid_cap: int = 0, tails: int = 2) -> None:
        t = im_tuning(group_first, group_rest, rounds_per_step, dense_div, int(use_graphs), grid_cap, tails)
        _check(lib().im_engine_set_tuning(self.handle, ctypes.byref(t)))

    def get_tuning(self) -> dict:
        t = im_tuning()
        _check(lib().im_engine_get_tuning(self.handle, ctypes.byref(t)))
        return t.as_dict()

    def counters(self) -> dict:
        st, gb, gr = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().im_engine_counters(self.handle, ctypes.byref(st), ctypes.byref(gb), ctypes.byref(gr)))
        return dict(steps=st.value, graphs_built=gb.value, graph_replays=gr.value)

    def info(self) -> dict:
        nq, nr = ctypes.c_int32(), ctypes.c_int32()
        used, budget = ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib().im_engine_info(self.handle, ctypes.byref(nq), ctypes.byref(nr), ctypes.byref(used),
                                    ctypes.byref(budget)))
        return dict(queries=nq.value, running=nr.value, bytes_used=used.value, bytes_budget=budget.value)

    def run(self) -> dict:
        """Step until every admitted query finished; return {id: result}."""
        while self.step() > 0:
            pass
        return {q: self.result(q) for q in self.poll()}

    def free(self) -> None:
        if self.handle:
            lib().im_engine_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def im_select_seeds_batch(graphs, J, seeds, K, stream=None):
    """G independent queries in one engine; returns (list of seed arrays, spreads)."""
    G = len(graphs)
    gh = (ctypes.c_void_p * G)(*[g.handle.value for g in graphs])
    Ja = np.ascontiguousarray(J, dtype=np.int32)
    Sa = np.ascontiguousarray(np.asarray(seeds, dtype=np.uint64))
    Ka = np.ascontiguousarray(K, dtype=np.int32)
    outs = [np.zeros(int(k), dtype=np.int32) for k in Ka]
    optr = (ctypes.c_void_p * G)(*[o.ctypes.data for o in outs])
    spread = np.zeros(G, dtype=np.float64)
    _check(lib().im_select_seeds_batch(G, gh, _p(Ja), _p(Sa), _p(Ka), optr, _p(spread), _stream(stream)))
    return outs, spread

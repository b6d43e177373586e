"""ctypes front end of the plain C oracle (im_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the CPU-baseline
leg of the benchmark.  It is a slow, obviously-correct CPU implementation of the
sketch-based influence-maximisation method and shares no code with the HIP path.
Every oracle function follows the step of the paper named in its C docstring.

The hash functions (Eq. 1 and the per-register hash of Eq. 3) are pinned in the
tests against scikit-learn's independent MurmurHash3 implementation and the
SMHasher verification value; SplitMix64 against its published first outputs.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "im_oracle.c")
_LIB = os.path.join(_HERE, "liborcim.so")

CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared", "-Wall", "-Wextra"]


def compile_lib(force: bool = True) -> str:
    """Compile the oracle into oracle/liborcim.so with gcc."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            compile_lib()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, i32, u32, u64, dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double
        L.orc_murmur3_32.argtypes = [P, i64, u32]
        L.orc_murmur3_32.restype = u32
        L.orc_splitmix64_at.argtypes = [u64, u64]
        L.orc_splitmix64_at.restype = u64
        L.orc_edge_hash.argtypes = [u32, u32]
        L.orc_edge_hash.restype = u32
        L.orc_rank.argtypes = [u64, u32, u32]
        L.orc_rank.restype = ctypes.c_uint8
        L.orc_threshold.argtypes = [ctypes.c_float]
        L.orc_threshold.restype = u32
        L.orc_live.argtypes = [u32, u32, u32]
        L.orc_live.restype = ctypes.c_int
        L.orc_sim_values.argtypes = [u64, i32, P]
        L.orc_sim_values.restype = None
        L.orc_alpha.argtypes = [i32]
        L.orc_alpha.restype = dbl
        L.orc_fill.argtypes = [i64, i32, u64, P, P]
        L.orc_fill.restype = None
        L.orc_build.argtypes = [i64, P, P, P, i32, u64, P, P]
        L.orc_build.restype = ctypes.c_int
        L.orc_sweeps_sample.argtypes = [i64, P, P, P, i32, u64, P, i32, i32, P, P]
        L.orc_sweeps_sample.restype = ctypes.c_int
        L.orc_estimates.argtypes = [i64, i32, P, P, P, P]
        L.orc_estimates.restype = None
        L.orc_argmax.argtypes = [i64, P, P, P]
        L.orc_argmax.restype = i64
        L.orc_estimate_value.argtypes = [i32, u32, u64]
        L.orc_estimate_value.restype = dbl
        L.orc_greedy.argtypes = [i64, P, P, P, i32, u64, i32, P, P, P, P, P, P, P, P, P]
        L.orc_greedy.restype = ctypes.c_int
        L.orc_graph_hashes.argtypes = [i64, P, P, P, P, P]
        L.orc_graph_hashes.restype = None
        L.orc_reach_max.argtypes = [i64, P, P, P, P, u32, u64, i32, i64, P]
        L.orc_reach_max.restype = ctypes.c_int
        L.orc_cover_from.argtypes = [i64, P, P, P, P, u32, P, i64, P]
        L.orc_cover_from.restype = i64
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _graph_arrays(g):
    rowptr = np.ascontiguousarray(g.rowptr, dtype=np.int64)
    col = np.ascontiguousarray(g.col, dtype=np.int32)
    p = np.ascontiguousarray(g.p, dtype=np.float32)
    return rowptr, col, p


# ---------------------------------------------------------------- primitives

def murmur3_32(key: bytes, seed: int = 0) -> int:
    buf = np.frombuffer(key, dtype=np.uint8) if key else np.zeros(1, np.uint8)
    return int(lib().orc_murmur3_32(_ptr(buf), len(key), seed & 0xFFFFFFFF))


def splitmix64_at(seed: int, i: int) -> int:
    return int(lib().orc_splitmix64_at(seed & (2**64 - 1), i))


def edge_hash(u: int, v: int) -> int:
    return int(lib().orc_edge_hash(u, v))


def rank(seed: int, u: int, j: int) -> int:
    return int(lib().orc_rank(seed & (2**64 - 1), u, j))


def threshold(p: float) -> int:
    return int(lib().orc_threshold(float(np.float32(p))))


def live(X: int, h: int, W: int) -> bool:
    return bool(lib().orc_live(X, h, W))


def sim_values(seed: int, J: int) -> np.ndarray:
    X = np.zeros(J, dtype=np.uint32)
    lib().orc_sim_values(seed & (2**64 - 1), J, _ptr(X))
    return X


def alpha(J: int) -> float:
    return float(lib().orc_alpha(J))


def fill(n: int, J: int, seed: int, cov: Optional[np.ndarray] = None) -> np.ndarray:
    M = np.zeros((n, J), dtype=np.uint8)
    c = None if cov is None else np.ascontiguousarray(cov, dtype=np.uint8)
    lib().orc_fill(n, J, seed & (2**64 - 1), _ptr(c), _ptr(M))
    return M


# ---------------------------------------------------------------- method steps

def build(g, J: int, seed: int):
    """Alg. 1 then Alg. 2 sweeps to the fixed point. Returns (M[n,J] uint8, sweeps)."""
    rowptr, col, p = _graph_arrays(g)
    M = np.zeros((g.n, J), dtype=np.uint8)
    sw = np.zeros(1, dtype=np.int32)
    st = lib().orc_build(g.n, _ptr(rowptr), _ptr(col), _ptr(p), J, seed & (2**64 - 1), _ptr(M), _ptr(sw))
    if st:
        raise RuntimeError(f"orc_build failed: {st}")
    return M, int(sw[0])


def sweeps_sample(g, J: int, seed: int, sims, nsweeps: int, registers: bool = False):
    """`nsweeps` synchronous sweeps (Alg. 2) from Fill (Alg. 1) over the
    simulation columns `sims` only.  Returns the number of registers the last
    sweep changed, and with registers=True also the registers uint8[n, len(sims)]."""
    rowptr, col, p = _graph_arrays(g)
    sims = np.ascontiguousarray(sims, dtype=np.int32)
    ch = np.zeros(1, dtype=np.int64)
    M = np.zeros((g.n, len(sims)), dtype=np.uint8) if registers else None
    st = lib().orc_sweeps_sample(g.n, _ptr(rowptr), _ptr(col), _ptr(p), J, seed & (2**64 - 1),
                                 _ptr(sims), len(sims), nsweeps, _ptr(ch), _ptr(M))
    if st:
        raise RuntimeError(f"orc_sweeps_sample failed: {st}")
    return (int(ch[0]), M) if registers else int(ch[0])


def estimates(M: np.ndarray, cov: Optional[np.ndarray] = None):
    """Per-vertex (J_u, H_u) of Eq. 7's harmonic form, over uncovered registers."""
    M = np.ascontiguousarray(M, dtype=np.uint8)
    n, J = M.shape
    Ju = np.zeros(n, dtype=np.uint32)
    Hu = np.zeros(n, dtype=np.uint64)
    c = None if cov is None else np.ascontiguousarray(cov, dtype=np.uint8)
    lib().orc_estimates(n, J, _ptr(M), _ptr(c), _ptr(Ju), _ptr(Hu))
    return Ju, Hu


def argmax(Ju: np.ndarray, Hu: np.ndarray, is_seed: Optional[np.ndarray] = None) -> int:
    Ju = np.ascontiguousarray(Ju, dtype=np.uint32)
    Hu = np.ascontiguousarray(Hu, dtype=np.uint64)
    s = None if is_seed is None else np.ascontiguousarray(is_seed, dtype=np.uint8)
    return int(lib().orc_argmax(len(Ju), _ptr(Ju), _ptr(Hu), _ptr(s)))


def estimate_value(J: int, Js: int, Hs: int) -> float:
    return float(lib().orc_estimate_value(J, Js, Hs))


def greedy(g, J: int, seed: int, K: int, keep_registers: bool = True) -> dict:
    """Alg. 4 on one device.  Returns seeds, per-pick estimates, covered-pair
    counts T after each cascade, sweep counts, spread = T_K/J and (optionally)
    registers after the initial build and at the end."""
    rowptr, col, p = _graph_arrays(g)
    n = g.n
    seeds = np.zeros(K, dtype=np.int32)
    est = np.zeros(K, dtype=np.float64)
    T = np.zeros(K, dtype=np.uint64)
    sweeps = np.zeros(K, dtype=np.int32)
    Mb = np.zeros((n, J), dtype=np.uint8) if keep_registers else None
    Mf = np.zeros((n, J), dtype=np.uint8) if keep_registers else None
    Ju0 = np.zeros(n, dtype=np.uint32)
    Hu0 = np.zeros(n, dtype=np.uint64)
    spread = np.zeros(1, dtype=np.float64)
    st = lib().orc_greedy(n, _ptr(rowptr), _ptr(col), _ptr(p), J, seed & (2**64 - 1), K,
                          _ptr(seeds), _ptr(est), _ptr(T), _ptr(sweeps), _ptr(Mb), _ptr(Ju0), _ptr(Hu0),
                          _ptr(Mf), _ptr(spread))
    if st:
        raise RuntimeError(f"orc_greedy failed: {st}")
    return dict(seeds=seeds, est=est, T=T, sweeps=sweeps, M_build0=Mb, Ju0=Ju0, Hu0=Hu0,
                M_final=Mf, spread=float(spread[0]))


# ---------------------------------------------------------------- closed forms (pins)

class LiveGraph:
    """Per-arc hashes (Eq. 1) and thresholds of a graph, for closed-form checks."""

    def __init__(self, g):
        self.g = g
        self.rowptr, self.col, self.p = _graph_arrays(g)
        self.h = np.zeros(g.m, dtype=np.uint32)
        self.W = np.zeros(g.m, dtype=np.uint32)
        lib().orc_graph_hashes(g.n, _ptr(self.rowptr), _ptr(self.col), _ptr(self.p), _ptr(self.h), _ptr(self.W))

    def reach_max(self, Xj: int, seed: int, j: int, u: int, covered_j: Optional[np.ndarray] = None) -> int:
        """Closed-form register of (u, j): max rank over vertices reachable from u
        in simulation j's live graph avoiding covered vertices (0 if u covered)."""
        c = None if covered_j is None else np.ascontiguousarray(covered_j, dtype=np.uint8)
        r = lib().orc_reach_max(self.g.n, _ptr(self.rowptr), _ptr(self.col), _ptr(self.h), _ptr(self.W),
                                int(Xj), seed & (2**64 - 1), j, u, _ptr(c))
        if r < 0:
            raise MemoryError("orc_reach_max")
        return int(r)

    def cover_from(self, Xj: int, sources) -> np.ndarray:
        """Covered flags of one simulation: union of reachability sets of `sources`."""
        src = np.ascontiguousarray(sources, dtype=np.int32)
        out = np.zeros(self.g.n, dtype=np.uint8)
        r = lib().orc_cover_from(self.g.n, _ptr(self.rowptr), _ptr(self.col), _ptr(self.h), _ptr(self.W),
                                 int(Xj), _ptr(src), len(src), _ptr(out))
        if r < 0:
            raise MemoryError("orc_cover_from")
        return out

"""Seeded synthetic inputs: directed graphs in CSR form plus per-edge probabilities.

This module is shared by the HIP path's tests/benchmarks and by the CPU oracle's
tests.  It holds only input generation (graph topology and the edge-probability
scheme handed to the library as float32); none of the influence-maximisation
arithmetic (hashing, thresholds, sketches, estimates) lives here.

Graph families stand in for the paper's social networks (Table 2), which are not
available here: Erdos-Renyi, R-MAT (power-law, like the SNAP social graphs) and
Barabasi-Albert (undirected, stored as two arcs per edge as the paper does for
its undirected graphs).  Probability schemes follow Section 2.1: uniform IC,
weighted cascade (w_uv = 1/indeg(v)) and the trivalency mix.
"""
from __future__ import annotations

import dataclasses
import os
from typing import Optional

import numpy as np

__all__ = [
    "Graph", "csr_from_edges", "erdos_renyi", "rmat", "barabasi_albert", "road_grid",
    "uniform_p", "weighted_cascade_p", "trivalency_p", "with_p",
    "save_npz", "load_npz", "cached", "SERVED_SCALES", "served_graph_names", "served_graph", "served_requests",
    "batched_specs", "batched_graph",
]


@dataclasses.dataclass
class Graph:
    """CSR by source: out-edges of u are col[rowptr[u]:rowptr[u+1]], sorted ascending,
    no duplicates, no self-loops.  p[e] is the float32 IC probability of edge e."""
    n: int
    rowptr: np.ndarray          # int64[n+1]
    col: np.ndarray             # int32[m]
    p: Optional[np.ndarray]     # float32[m]
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.col.shape[0])

    def src(self) -> np.ndarray:
        """Source vertex of every edge (int32[m])."""
        return np.repeat(np.arange(self.n, dtype=np.int32), np.diff(self.rowptr))

    def out_degree(self) -> np.ndarray:
        return np.diff(self.rowptr)

    def in_degree(self) -> np.ndarray:
        return np.bincount(self.col, minlength=self.n).astype(np.int64)


def csr_from_edges(n: int, src: np.ndarray, dst: np.ndarray) -> Graph:
    """Build a CSR graph: self-loops dropped, duplicate arcs merged to one arc."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    keep = src != dst
    key = np.unique(src[keep] * np.int64(n) + dst[keep])
    s = key // n
    d = (key % n).astype(np.int32)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(s, minlength=n), out=rowptr[1:])
    return Graph(n=n, rowptr=rowptr, col=np.ascontiguousarray(d), p=None)


def erdos_renyi(n: int, m: int, seed: int = 1) -> Graph:
    """m distinct directed arcs with uniform endpoints; self-loops and repeats redrawn."""
    if m > n * (n - 1):
        raise ValueError("too many edges for a simple digraph")
    rng = np.random.Generator(np.random.PCG64(seed))
    keys = np.empty(0, dtype=np.int64)
    while keys.size < m:
        need = m - keys.size
        s = rng.integers(0, n, size=need, dtype=np.int64)
        d = rng.integers(0, n, size=need, dtype=np.int64)
        k = s * n + d
        k = k[s != d]
        allk = np.concatenate([keys, k])
        # keep first occurrence in draw order so the result is independent of batch size
        _, first = np.unique(allk, return_index=True)
        first.sort()
        keys = allk[first][:m]
    g = csr_from_edges(n, keys // n, keys % n)
    g.name = f"er_n{n}_m{m}_s{seed}"
    return g


def _rmat_chunk(child, cnt, scale, a, b, c):
    rng = np.random.Generator(np.random.PCG64(child))
    s = np.zeros(cnt, dtype=np.int64)
    d = np.zeros(cnt, dtype=np.int64)
    ab, abc = a + b, a + b + c
    for lvl in range(scale):
        r = rng.random(cnt)
        s |= (r >= ab).astype(np.int64) << lvl
        d |= (((r >= a) & (r < ab)) | (r >= abc)).astype(np.int64) << lvl
    return s, d


def rmat(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19,
         c: float = 0.19, seed: int = 1, relabel: bool = True,
         chunk: int = 1 << 22, threads: Optional[int] = None) -> Graph:
    """R-MAT: edge_factor * 2^scale recursive-quadrant draws, then dedup and
    self-loop removal.  Draws come in chunks with independent child seeds of
    `seed`, so the graph does not depend on the thread count.  With relabel,
    vertex ids get a seeded random permutation so hubs are scattered."""
    from concurrent.futures import ThreadPoolExecutor
    n = 1 << scale
    m_draw = edge_factor << scale
    nchunks = (m_draw + chunk - 1) // chunk
    children = np.random.SeedSequence(seed).spawn(nchunks + 1)
    sizes = [min(chunk, m_draw - i * chunk) for i in range(nchunks)]
    workers = threads or min(16, os.cpu_count() or 1)
    with ThreadPoolExecutor(max_workers=workers) as ex:
        parts = list(ex.map(lambda i: _rmat_chunk(children[i], sizes[i], scale, a, b, c), range(nchunks)))
    s = np.concatenate([p[0] for p in parts])
    d = np.concatenate([p[1] for p in parts])
    del parts
    if relabel:
        perm = np.random.Generator(np.random.PCG64(children[-1])).permutation(n).astype(np.int64)
        s, d = perm[s], perm[d]
    g = csr_from_edges(n, s, d)
    g.name = f"rmat{scale}_ef{edge_factor}_s{seed}"
    return g


def barabasi_albert(n: int, m0: int = 8, seed: int = 0) -> Graph:
    """Undirected preferential-attachment graph, two arcs per edge.

    Vertex m0 joins vertices 0..m0-1; every later vertex t adds m0 edges whose
    far ends are uniform picks among the endpoints of all earlier edges, i.e.
    proportional to degree (the Bollobas-Riordan linearized chord diagram
    form of the Barabasi-Albert model).  The picks are resolved with pointer
    jumping, so generation is vectorised.  Repeated picks by one vertex
    collapse to one edge."""
    if n <= m0:
        raise ValueError("n must exceed m0")
    rng = np.random.Generator(np.random.PCG64(seed))
    E = m0 + (n - m0 - 1) * m0
    k = np.arange(E, dtype=np.int64)
    src = np.empty(E, dtype=np.int64)
    src[:m0] = m0
    src[m0:] = m0 + 1 + (k[m0:] - m0) // m0
    # first edge index of each edge's source vertex: picks come from earlier vertices only
    k0 = np.where(k < m0, 0, m0 + ((k - m0) // m0) * m0)
    val = np.full(2 * E, -1, dtype=np.int64)   # endpoint value per position (2k: src, 2k+1: target)
    val[0::2] = src
    val[1:2 * m0:2] = np.arange(m0)
    ptr = np.arange(2 * E, dtype=np.int64)
    late = np.arange(m0, E)
    ptr[2 * late + 1] = (rng.random(late.size) * (2 * k0[late])).astype(np.int64)
    todo = 2 * late + 1
    while todo.size:
        q = ptr[todo]
        got = val[q] >= 0
        val[todo[got]] = val[q[got]]
        todo = todo[~got]
        ptr[todo] = ptr[ptr[todo]]
    tgt = val[1::2]
    g = csr_from_edges(n, np.concatenate([src, tgt]), np.concatenate([tgt, src]))
    g.name = f"ba_n{n}_m{m0}_s{seed}"
    return g


# ---------------------------------------------------------------- probability schemes

def road_grid(width: int, height: int, drop: float = 0.1, seed: int = 1) -> Graph:
    """A road-network stand-in with the structure the paper names as its
    method's weak case (many vertices, few edges, high diameter): a
    width x height lattice whose horizontal and vertical links are two-way
    roads (two arcs each), with a seeded fraction `drop` of the links removed.
    Vertex ids are row-major, so nearby intersections have nearby ids."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = width * height
    ids = np.arange(n, dtype=np.int64).reshape(height, width)
    a = np.concatenate([ids[:, :-1].ravel(), ids[:-1, :].ravel()])  # right and down links
    b = np.concatenate([ids[:, 1:].ravel(), ids[1:, :].ravel()])
    keep = rng.random(a.size) >= drop
    a, b = a[keep], b[keep]
    g = csr_from_edges(n, np.concatenate([a, b]), np.concatenate([b, a]))
    g.name = f"road{width}x{height}"
    return g


def uniform_p(g: Graph, p: float) -> np.ndarray:
    return np.full(g.m, p, dtype=np.float32)


def weighted_cascade_p(g: Graph) -> np.ndarray:
    """Weighted cascade: every in-arc of v gets 1/indeg(v) (indeg of the final,
    deduplicated, loop-free graph), rounded to float32."""
    indeg = g.in_degree()
    return (1.0 / indeg[g.col].astype(np.float64)).astype(np.float32)


def trivalency_p(g: Graph, seed: int = 2) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    choices = np.array([0.1, 0.01, 0.001], dtype=np.float32)
    return choices[rng.integers(0, 3, size=g.m)]


def normal_p(g: Graph, mean: float = 0.05, sd: float = 0.025, seed: int = 2) -> np.ndarray:
    """Per-arc probabilities drawn from N(mean, sd), clipped to [0, 1]: the
    mixed-weight setting N0.05 of the paper's experiments (Section 5, edge
    weight settings)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.clip(rng.normal(mean, sd, size=g.m), 0.0, 1.0).astype(np.float32)


def uniform_range_p(g: Graph, lo: float = 0.0, hi: float = 0.1, seed: int = 2) -> np.ndarray:
    """Per-arc probabilities drawn uniformly from [lo, hi): the setting U0.1 of
    the paper's experiments (Section 5, edge weight settings)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(lo, hi, size=g.m).astype(np.float32)


def with_p(g: Graph, scheme: str, seed: int = 2) -> Graph:
    """Return a shallow copy of g carrying the named probability scheme:
    'wc', 'trivalency', 'normal' (N(0.05, 0.025) clipped to [0, 1]),
    'uniform01' (U(0, 0.1)), or a float literal such as '0.01'."""
    if scheme == "wc":
        p = weighted_cascade_p(g)
    elif scheme == "trivalency":
        p = trivalency_p(g, seed)
    elif scheme == "normal":
        p = normal_p(g, seed=seed)
    elif scheme == "uniform01":
        p = uniform_range_p(g, seed=seed)
    else:
        p = uniform_p(g, float(scheme))
    return Graph(n=g.n, rowptr=g.rowptr, col=g.col, p=p, name=f"{g.name}_{scheme}")


# ---------------------------------------------------------------- caching

def save_npz(g: Graph, path: str) -> None:
    np.savez(path, n=np.int64(g.n), rowptr=g.rowptr, col=g.col,
             p=(g.p if g.p is not None else np.empty(0, np.float32)),
             name=np.array(g.name))


def load_npz(path: str) -> Graph:
    z = np.load(path, allow_pickle=False)
    p = z["p"]
    return Graph(n=int(z["n"]), rowptr=z["rowptr"], col=z["col"],
                 p=(p if p.size else None), name=str(z["name"]))


def cached(path: Optional[str], make) -> Graph:
    """Load a graph from `path` if present, else build it with make() and store it."""
    if path and os.path.exists(path):
        return load_npz(path)
    g = make()
    if path:
        os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
        save_npz(g, path)
    return g


# ---------------------------------------------------------------------------
# Served-queries workload: resident RMAT graphs (edge factor 16) at these
# scales, the last with another generator seed, each under p = 0.01 and
# weighted cascade; a request stream over them.

SERVED_SCALES = (16, 17, 18, 19, 20, 21, 22, 22)


def served_graph_names(scales=SERVED_SCALES):
    """Graph names of the served workload, sorted: rmat<scale>_<index>_<scheme>."""
    return sorted(f"rmat{sc}_{i}_{scheme}" for i, sc in enumerate(scales) for scheme in ("0.01", "wc"))


def served_graph(name: str, scales=SERVED_SCALES) -> Graph:
    """The graph of a served-workload name (generated; seed 1, or 2 for a
    repeated scale's later copy)."""
    _, idx, scheme = name.split("_")
    i = int(idx)
    sc = scales[i]
    seed = 1 if i < len(scales) - 1 or list(scales).count(sc) == 1 else 2
    return with_p(rmat(sc, 16, seed=seed), scheme)


def served_requests(count: int, scales=SERVED_SCALES, seed: int = 1):
    """The served workload's request stream: (graph name, J, sketch seed, K)
    with the graph uniform over the names, J uniform over {128, 512}, K
    uniform in [10, 100] and the sketch seed = the request's index."""
    names = served_graph_names(scales)
    rng = np.random.Generator(np.random.PCG64(seed))
    return [(names[int(rng.integers(len(names)))], int(rng.choice([128, 512])), int(i), int(rng.integers(10, 101)))
            for i in range(count)]


# ---------------------------------------------------------------------------
# Batched-queries workload: 64 graphs of uneven size, weighted cascade.

def batched_specs():
    """(kind, size, index) of the 64 graphs: 32 RMAT with scales uniform in
    12..18, then 32 Barabasi-Albert with n uniform in 10k..200k (m0 = 8)."""
    rng = np.random.Generator(np.random.PCG64(4))
    specs = [("rmat", int(rng.integers(12, 19)), i) for i in range(32)]
    specs += [("ba", int(rng.integers(10_000, 200_001)), i) for i in range(32)]
    return specs


def batched_graph(spec) -> Graph:
    """The weighted-cascade graph of one batched-workload spec."""
    kind, size, i = spec
    g = rmat(size, 16, seed=100 + i) if kind == "rmat" else barabasi_albert(size, 8, seed=i)
    return with_p(g, "wc")


"""Independent re-derivations used to pin the oracle (tests only).

Nothing here calls the oracle's hash, threshold or propagation code:
  - hashes come from scikit-learn's MurmurHash3_x86_32 (a separate implementation),
  - leading-zero counts from Python's int.bit_length,
  - thresholds from exact rational arithmetic (fractions.Fraction),
  - reachability from networkx graph traversal.
"""
from __future__ import annotations

import struct
from fractions import Fraction

import networkx as nx
import numpy as np
from sklearn.utils import murmurhash3_32


def sk_hash(key: bytes, seed: int) -> int:
    return int(murmurhash3_32(key, seed=seed, positive=True))


def sk_edge_hash(u: int, v: int) -> int:
    """Eq. 1 via scikit-learn: Murmur3(LE32(u) || LE32(v), seed 0) mod 2^31."""
    return sk_hash(struct.pack("<II", u, v), 0) % (1 << 31)


def clz32(x: int) -> int:
    return 32 - int(x).bit_length()


def sk_rank(seed: int, u: int, j: int) -> int:
    key = struct.pack("<IIII", seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF, u, j)
    return clz32(sk_hash(key, 1)) + 1


def exact_threshold(p) -> int:
    """floor(p * 2^31) capped at 2^31, with p taken as the exact float32 value."""
    f = Fraction(float(np.float32(p)))
    return int(min(Fraction(1 << 31), f * (1 << 31)) // 1)


def live_digraphs(g, X):
    """One networkx DiGraph per simulation j holding the arcs live in j (Eq. 2)."""
    src = g.src()
    H = [sk_edge_hash(int(u), int(v)) for u, v in zip(src, g.col)]
    W = [exact_threshold(p) for p in g.p]
    out = []
    for xj in X:
        G = nx.DiGraph()
        G.add_nodes_from(range(g.n))
        G.add_edges_from((int(u), int(v)) for u, v, h, w in zip(src, g.col, H, W) if (int(xj) ^ h) < w)
        out.append(G)
    return out


def hop_limited_registers(g, X, seed, sims, hops):
    """Registers after `hops` synchronous sweeps from the fill, nothing covered:
    register (u, j) is the max rank over the vertices within `hops` live arcs
    of u in simulation j (a sweep extends every register by one arc).  Returns
    uint8[n, len(sims)], column s for simulation sims[s]."""
    graphs = live_digraphs(g, [X[j] for j in sims])
    M = np.zeros((g.n, len(sims)), dtype=np.uint8)
    for s, (j, G) in enumerate(zip(sims, graphs)):
        for u in range(g.n):
            near = nx.single_source_shortest_path_length(G, u, cutoff=hops)
            M[u, s] = max(sk_rank(seed, w, int(j)) for w in near)
    return M


def closed_form_registers(g, X, seed, covered=None):
    """Registers at the fixed point: for uncovered (u, j), the max rank over the
    vertices reachable from u in the live graph of j through uncovered vertices."""
    J = len(X)
    M = np.zeros((g.n, J), dtype=np.uint8)
    for j, G in enumerate(live_digraphs(g, X)):
        if covered is not None:
            G = G.subgraph([u for u in range(g.n) if not covered[u, j]]).copy()
        for u in G.nodes:
            reach = nx.descendants(G, u) | {u}
            M[u, j] = max(sk_rank(seed, w, j) for w in reach)
    return M

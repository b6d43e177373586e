"""Input generators: structure and determinism (CPU)."""
import numpy as np

import graphgen


def _check_csr(g):
    assert g.rowptr[0] == 0 and g.rowptr[-1] == g.m
    assert np.all(np.diff(g.rowptr) >= 0)
    src = g.src()
    assert np.all(src != g.col), "self-loop"
    for u in range(min(g.n, 2000)):
        row = g.col[g.rowptr[u]:g.rowptr[u + 1]]
        assert np.all(np.diff(row) > 0), "row not strictly increasing"


def test_er_exact_size_and_simple():
    g = graphgen.erdos_renyi(1000, 5000, 1)
    assert g.n == 1000 and g.m == 5000
    _check_csr(g)


def test_rmat_deterministic_across_thread_counts():
    a = graphgen.rmat(12, 16, seed=3, threads=1)
    b = graphgen.rmat(12, 16, seed=3, threads=4)
    assert np.array_equal(a.rowptr, b.rowptr) and np.array_equal(a.col, b.col)
    _check_csr(a)
    assert 0.8 * 16 * 4096 < a.m <= 16 * 4096


def test_ba_undirected_two_arcs():
    g = graphgen.barabasi_albert(500, 4, seed=1)
    _check_csr(g)
    pairs = set(zip(g.src().tolist(), g.col.tolist()))
    assert all((v, u) in pairs for u, v in pairs)


def test_probability_schemes():
    g = graphgen.rmat(10, 8, seed=2)
    wc = graphgen.with_p(g, "wc")
    indeg = g.in_degree()
    assert np.array_equal(wc.p, (1.0 / indeg[g.col]).astype(np.float32))
    tri = graphgen.with_p(g, "trivalency")
    assert set(np.unique(tri.p).tolist()) <= {np.float32(0.1), np.float32(0.01), np.float32(0.001)}
    u = graphgen.with_p(g, "0.01")
    assert np.all(u.p == np.float32(0.01))

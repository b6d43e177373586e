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


def test_mixed_weight_settings():
    """N(0.05, 0.025) clipped to [0, 1] and U(0, 0.1): ranges, moments,
    determinism for a seed."""
    g = graphgen.rmat(12, 16, seed=3)
    nrm = graphgen.with_p(g, "normal").p
    assert nrm.dtype == np.float32 and nrm.min() >= 0.0 and nrm.max() <= 1.0
    assert abs(float(nrm.mean()) - 0.05) < 0.002 and abs(float(nrm.std()) - 0.025) < 0.002
    uni = graphgen.with_p(g, "uniform01").p
    assert uni.min() >= 0.0 and uni.max() < 0.1
    assert abs(float(uni.mean()) - 0.05) < 0.002
    assert np.array_equal(graphgen.with_p(g, "normal").p, nrm)
    assert not np.array_equal(graphgen.with_p(g, "normal", seed=9).p, nrm)


def test_bench_monte_carlo_evaluator():
    """The quality report's evaluator: p = 1 reaches everything reachable,
    p = 0 only the seeds, and a path's spread under p is 1 + p + p^2 + ..."""
    import bench
    n = 40
    cyc = graphgen.Graph(n=n, rowptr=np.arange(n + 1, dtype=np.int64),
                         col=((np.arange(n) + 1) % n).astype(np.int32), p=np.ones(n, np.float32))
    rng = np.random.default_rng(0)
    assert np.all(bench.mc_spread(cyc, [3], 5, rng) == n)
    cyc0 = graphgen.Graph(n=n, rowptr=cyc.rowptr, col=cyc.col, p=np.zeros(n, np.float32))
    assert np.all(bench.mc_spread(cyc0, [3, 7], 5, rng) == 2)
    path = graphgen.Graph(n=3, rowptr=np.array([0, 1, 2, 2], np.int64), col=np.array([1, 2], np.int32),
                          p=np.full(2, 0.5, np.float32))
    s = bench.mc_spread(path, [0], 4000, rng)
    assert abs(s.mean() - 1.75) < 0.06


def test_served_and_batched_workload_recipes():
    """The served and batched workloads' inputs: 16 resident graph names, a
    request stream with J in {128, 512}, K in [10, 100] and the sketch seed
    equal to the index, uniform over the graphs; 64 batched specs (32 RMAT of
    scales 12..18, then 32 BA of 10k..200k vertices); all deterministic."""
    import collections
    names = graphgen.served_graph_names()
    assert len(names) == 16 and names == sorted(names)
    assert {n.split("_")[2] for n in names} == {"0.01", "wc"}
    reqs = graphgen.served_requests(1000)
    assert reqs == graphgen.served_requests(1000) and reqs[:10] == graphgen.served_requests(10)
    assert [r[2] for r in reqs] == list(range(1000))
    assert {r[1] for r in reqs} == {128, 512} and all(10 <= r[3] <= 100 for r in reqs)
    counts = collections.Counter(r[0] for r in reqs)
    assert set(counts) == set(names) and min(counts.values()) > 30  # ~62 each
    g = graphgen.served_graph("rmat16_0_wc")
    assert g.n == 1 << 16 and g.p is not None
    # the repeated scale's second copy uses another generator seed
    assert graphgen.served_graph_names().count("rmat22_6_wc") == 1 and "rmat22_7_wc" in names
    specs = graphgen.batched_specs()
    assert len(specs) == 64 and specs == graphgen.batched_specs()
    assert all(k == "rmat" and 12 <= s <= 18 for k, s, _ in specs[:32])
    assert all(k == "ba" and 10_000 <= s <= 200_000 for k, s, _ in specs[32:])
    assert [i for _, _, i in specs] == list(range(32)) * 2
    small = min(specs[:32], key=lambda sp: sp[1])
    gb = graphgen.batched_graph(small)
    assert gb.n == 1 << small[1] and np.all(gb.p > 0)

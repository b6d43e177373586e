"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Everything the method computes is integer, so the bar is bit-exact: simulation
values, registers after the build, estimate terms (J_u, H_u), seeds, covered
counts T per pick, final registers; the reported estimates are one IEEE double
expression of exact integers and must match to the last bit as well.
"""
import sys

import numpy as np
import pytest

import graphgen

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def run_gpu(imx, g, J, seed, K):
    G = imx.Graph.from_graphgen(g)
    S = imx.Sketch(G, J, seed)
    out = dict(X=S.sim_values(), M0=S.registers())
    out["Ju0"], out["Hu0"] = S.estimates()
    out.update(S.select(K))
    out["Mf"] = S.registers()
    out["Juf"], out["Huf"] = S.estimates()
    S.free()
    G.free()
    return out


def assert_parity(orc, gpu, ref, J, seed):
    assert np.array_equal(gpu["X"], orc.sim_values(seed, J)), "simulation values"
    assert np.array_equal(gpu["M0"], ref["M_build0"]), "registers after build"
    assert np.array_equal(gpu["Ju0"], ref["Ju0"]), "J_u after build"
    assert np.array_equal(gpu["Hu0"], ref["Hu0"]), "H_u after build"
    assert list(gpu["seeds"]) == list(ref["seeds"]), "seeds"
    assert list(gpu["T"]) == list(ref["T"]), "T per pick"
    assert gpu["est"].tobytes() == ref["est"].tobytes(), "estimates"
    assert gpu["spread"] == ref["spread"]
    assert np.array_equal(gpu["Mf"], ref["M_final"]), "final registers"
    Ju, Hu = orc.estimates(gpu["Mf"])
    assert np.array_equal(gpu["Juf"], Ju) and np.array_equal(gpu["Huf"], Hu), "final estimate terms"
    rebuilds = int(np.count_nonzero(ref["sweeps"][1:]))
    assert gpu["stats"]["rebuilds"] == rebuilds
    # in-place sweeps reach the fixed point no later than synchronous ones
    assert gpu["stats"]["build_sweeps"] <= int(ref["sweeps"][0]), (gpu["stats"]["build_sweeps"], ref["sweeps"][0])
    assert gpu["stats"]["total_sweeps"] <= int(ref["sweeps"].sum())


def _hub_graph():
    # one hub with 1500 out-arcs (split into several propagation tasks) plus
    # random arcs; ragged row lengths everywhere.
    rng = np.random.default_rng(9)
    n = 2000
    src = np.concatenate([np.zeros(1500, np.int64), rng.integers(0, n, 6000)])
    dst = np.concatenate([rng.permutation(np.arange(1, n))[:1500], rng.integers(0, n, 6000)])
    return graphgen.with_p(graphgen.csr_from_edges(n, src, dst), "0.2")


def _cycle(n):
    return graphgen.with_p(graphgen.csr_from_edges(n, np.arange(n), (np.arange(n) + 1) % n), "1.0")


CASES = {
    "c1_er1k_p0.1_J64_s1": (lambda: graphgen.with_p(graphgen.erdos_renyi(1000, 5000, 1), "0.1"), 64, 1, 10),
    "c1_er1k_p0.1_J64_s2": (lambda: graphgen.with_p(graphgen.erdos_renyi(1000, 5000, 1), "0.1"), 64, 2, 10),
    "c1_er1k_p0.1_J64_s3": (lambda: graphgen.with_p(graphgen.erdos_renyi(1000, 5000, 1), "0.1"), 64, 3, 10),
    "er400_wc_J128": (lambda: graphgen.with_p(graphgen.erdos_renyi(400, 4000, 2), "wc"), 128, 5, 8),
    "er300_tri_J192": (lambda: graphgen.with_p(graphgen.erdos_renyi(300, 2000, 3), "trivalency"), 192, 6, 6),
    "er500_p0.5_J320": (lambda: graphgen.with_p(graphgen.erdos_renyi(500, 3000, 4), "0.5"), 320, 7, 5),
    "er200_p0.01_J1024": (lambda: graphgen.with_p(graphgen.erdos_renyi(200, 1200, 5), "0.01"), 1024, 8, 5),
    "er150_p0.3_J4096": (lambda: graphgen.with_p(graphgen.erdos_renyi(150, 800, 6), "0.3"), 4096, 9, 3),
    "hub2000_p0.2_J256": (_hub_graph, 256, 10, 5),
    "rmat12_wc_J512": (lambda: graphgen.with_p(graphgen.rmat(12, 16, seed=3), "wc"), 512, 11, 5),
    "ba3000_wc_J256": (lambda: graphgen.with_p(graphgen.barabasi_albert(3000, 8, seed=1), "wc"), 256, 12, 5),
    "er100_p0_J64": (lambda: graphgen.with_p(graphgen.erdos_renyi(100, 500, 7), "0"), 64, 13, 4),
    "cycle50_p1_J64": (lambda: _cycle(50), 64, 14, 5),
    "er60_p1_J128_Kn": (lambda: graphgen.with_p(graphgen.erdos_renyi(60, 150, 8), "1.0"), 128, 15, 60),
    "er400_normal_J128": (lambda: graphgen.with_p(graphgen.erdos_renyi(400, 4000, 9), "normal"), 128, 16, 8),
    "rmat11_uniform01_J256": (lambda: graphgen.with_p(graphgen.rmat(11, 16, seed=4), "uniform01"), 256, 17, 6),
    "rmat11_p0.005_J1024": (lambda: graphgen.with_p(graphgen.rmat(11, 16, seed=6), "0.005"), 1024, 18, 6),
    # road-network stand-ins (lattice, 10% of links removed): high diameter,
    # degree <= 4, so the tail kernels run by default
    "road48_p0.6_J256": (lambda: graphgen.with_p(graphgen.road_grid(48, 48, 0.1, seed=3), "0.6"), 256, 20, 8),
    "road64_p0.3_J64": (lambda: graphgen.with_p(graphgen.road_grid(64, 64, 0.1, seed=3), "0.3"), 64, 20, 10),
}


@pytest.mark.parametrize("name", list(CASES))
def test_parity_with_oracle(imx, orc, name):
    make, J, seed, K = CASES[name]
    g = make()
    _say(f"[parity] {name}: n={g.n} m={g.m} J={J} K={K} seed={seed}")
    ref = orc.greedy(g, J, seed, K)
    gpu = run_gpu(imx, g, J, seed, K)
    assert_parity(orc, gpu, ref, J, seed)


# The lane-group propagation kernels (16/32/64 lanes per task), selected
# through the environment at sketch creation; the default is the packed kernel.
LANE_GROUP_CASES = ["er300_tri_J192", "er200_p0.01_J1024", "er150_p0.3_J4096", "hub2000_p0.2_J256",
                    "rmat12_wc_J512"]


@pytest.mark.parametrize("groups", [("64", "64"), ("16", "32"), ("32", "16")])
@pytest.mark.parametrize("name", LANE_GROUP_CASES)
def test_lane_group_kernels_with_oracle(imx, orc, monkeypatch, name, groups):
    make, J, seed, K = CASES[name]
    g = make()
    monkeypatch.setenv("IMX_GROUP_FIRST", groups[0])
    monkeypatch.setenv("IMX_GROUP", groups[1])
    _say(f"[lane groups {groups}] {name}")
    ref = orc.greedy(g, J, seed, K)
    gpu = run_gpu(imx, g, J, seed, K)
    assert_parity(orc, gpu, ref, J, seed)


# Tail kernels (one workgroup per query runs many sweeps or cascade levels of
# a small frontier): forced for every frontier (limits huge, two rounds per
# launch so that launches hand over to each other), with tiny limits (frequent
# hand-backs to the full-grid path), and switched off.  A dense ER graph makes
# frontiers overflow the LDS set (flag hand-backs).
TAIL_SETTINGS = {
    "forced": {"IMX_TAIL": "1", "IMX_TAIL_ROWS": "1000000000", "IMX_TAIL_TASKS": "1000000000", "IMX_TAIL_ROUNDS": "2"},
    "tiny": {"IMX_TAIL": "1", "IMX_TAIL_ROWS": "4", "IMX_TAIL_TASKS": "3", "IMX_TAIL_ROUNDS": "3"},
    "off": {"IMX_TAIL": "0"},
}
TAIL_CASES = dict(CASES)
TAIL_CASES["er6000_p0.5_J64"] = (lambda: graphgen.with_p(graphgen.erdos_renyi(6000, 60000, 11), "0.5"), 64, 19, 4)
TAIL_CASE_NAMES = ["c1_er1k_p0.1_J64_s1", "er400_wc_J128", "er300_tri_J192", "er150_p0.3_J4096", "hub2000_p0.2_J256",
                   "rmat12_wc_J512", "ba3000_wc_J256", "cycle50_p1_J64", "er60_p1_J128_Kn", "er6000_p0.5_J64",
                   "road48_p0.6_J256"]


@pytest.mark.parametrize("setting", list(TAIL_SETTINGS))
@pytest.mark.parametrize("name", TAIL_CASE_NAMES)
def test_tail_kernels_with_oracle(imx, orc, monkeypatch, name, setting):
    make, J, seed, K = TAIL_CASES[name]
    g = make()
    for k, v in TAIL_SETTINGS[setting].items():
        monkeypatch.setenv(k, v)
    _say(f"[tail {setting}] {name}")
    ref = orc.greedy(g, J, seed, K)
    gpu = run_gpu(imx, g, J, seed, K)
    assert_parity(orc, gpu, ref, J, seed)


@pytest.mark.parametrize("n,K", [(1, 1), (10, 10)])
def test_edgeless_graphs(imx, orc, n, K):
    g = graphgen.Graph(n=n, rowptr=np.zeros(n + 1, np.int64), col=np.zeros(0, np.int32),
                       p=np.zeros(0, np.float32))
    _say(f"[edgeless] n={n} K={K}")
    ref = orc.greedy(g, 64, 1, K)
    gpu = run_gpu(imx, g, 64, 1, K)
    assert_parity(orc, gpu, ref, 64, 1)


def test_cycle_tie_break(imx):
    gpu = run_gpu(imx, _cycle(30), 64, 3, 4)
    assert list(gpu["seeds"]) == [0, 1, 2, 3]
    assert list(gpu["T"]) == [30 * 64] * 4


def test_schedule_independence_of_split(imx, orc, monkeypatch):
    """Splitting hub rows into different numbers of tasks changes the schedule
    of the in-place sweeps but not the fixed point or any output."""
    g = _hub_graph()
    outs = []
    for split in ("64", "4096"):
        monkeypatch.setenv("IMX_SPLIT", split)
        _say(f"[schedule] split={split}")
        outs.append(run_gpu(imx, g, 256, 21, 4))
    a, b = outs
    for key in ("M0", "Mf", "Ju0", "Hu0", "seeds", "T"):
        assert np.array_equal(a[key], b[key]), key


@pytest.mark.parametrize("grid", ["1", "3"])
@pytest.mark.parametrize("name", ["rmat12_wc_J512", "hub2000_p0.2_J256", "er150_p0.3_J4096", "er400_normal_J128"])
def test_packed_kernel_on_few_workgroups(imx, orc, monkeypatch, name, grid):
    """With the propagation grid capped at 1 or 3 workgroups, each workgroup
    takes many packs and its waves draw them from the shared counter; the
    results are the oracle's all the same."""
    make, J, seed, K = CASES[name]
    g = make()
    monkeypatch.setenv("IMX_PROP_GRID", grid)
    _say(f"[few workgroups {grid}] {name}")
    ref = orc.greedy(g, J, seed, K)
    gpu = run_gpu(imx, g, J, seed, K)
    assert_parity(orc, gpu, ref, J, seed)


def test_repeat_builds_identical(imx):
    g = graphgen.with_p(graphgen.rmat(11, 16, seed=5), "0.1")
    a = run_gpu(imx, g, 512, 2, 6)
    b = run_gpu(imx, g, 512, 2, 6)
    for key in ("M0", "Mf", "seeds", "T", "est"):
        assert np.array_equal(a[key], b[key]), key


def test_select_twice_is_state_error(imx):
    g = graphgen.with_p(graphgen.erdos_renyi(50, 200, 1), "0.1")
    G = imx.Graph.from_graphgen(g)
    S = imx.Sketch(G, 64, 1)
    S.select(2)
    with pytest.raises(imx.IMError) as ei:
        S.select(2)
    assert ei.value.status == 4
    with pytest.raises(imx.IMError) as ei:
        imx.Sketch(G, 100, 1)
    assert ei.value.status == 1
    S2 = imx.Sketch(G, 64, 1)
    with pytest.raises(imx.IMError):
        S2.select(51)


# ---------------------------------------------------------------- full-size workloads, pick by pick

def _cover(lg, X, j, seeds):
    """Covered set of simulation j for a seed prefix (the cascade's result:
    union of the seeds' live-graph reachability sets), by the oracle."""
    if len(seeds) == 0:
        return np.zeros(lg.g.n, np.uint8)
    return lg.cover_from(int(X[j]), [int(s) for s in seeds])


def stepwise_check(imx, orc, g, J, seed, K, *, reg_samples, reg_sims, full_picks=(), T_sims=None,
                   extra_reg_picks=(), label=""):
    """Run the selection of K seeds pick by pick (paused before every pick
    through the parity hook) and check, at full size, what each pick reads:
      - every pick equals the oracle's exact argmax over the downloaded
        (J_u, H_u) with the seeds so far excluded, and its reported estimate
        equals the oracle's value of those terms;
      - (J_u, H_u) of sampled rows equal the oracle's terms of those rows;
      - after the initial build and after every rebuild (and at the picks in
        `extra_reg_picks`), sampled registers equal the closed form: 0 where
        the simulation's covered set (cascades of the seeds so far) holds the
        vertex, else the max rank reachable without entering the covered set of
        the last rebuild;
      - at the picks in `full_picks`, every (J_u, H_u) equals the oracle's
        terms of the downloaded registers (all of them);
      - T after each pick equals the covered-pair count of the sampled
        simulations' covered sets, summed over `T_sims` (all J when None) at
        the picks in `full_picks`.
    Returns the final results and the number of rebuilds seen."""
    rng = np.random.default_rng(seed + 7)
    G = imx.Graph.from_graphgen(g)
    S = imx.Sketch(G, J, seed)
    X = S.sim_values()
    assert np.array_equal(X, orc.sim_values(seed, J)), "simulation values"
    lg = orc.LiveGraph(g)
    hubs = np.argsort(g.out_degree())[-8:]
    is_seed = np.zeros(g.n, np.uint8)
    seeds, expect_est, T_seen = [], [], []
    last_build, T_old, rebuilds = 0, 0, 0
    for k in range(K):
        if k % 10 == 0:
            _say(f"[{label}] pick {k}/{K}, rebuilds so far {rebuilds}")
        got_s, got_T = S.select_until(K, k)
        assert list(got_s) == seeds, f"{label} seeds before pick {k}"
        T_seen = [int(t) for t in got_T]
        if k > 0:
            T = T_seen[-1]
            if 100 * (T - T_old) > T:  # the rebuild rule after pick k-1 (< K-1)
                T_old, last_build = T, k
                rebuilds += 1
        Ju, Hu = S.estimates()
        s_k = orc.argmax(Ju, Hu, is_seed)
        expect_est.append(orc.estimate_value(J, int(Ju[s_k]), int(Hu[s_k])))
        us = np.unique(np.concatenate([rng.integers(0, g.n, 24), hubs])).astype(np.int32)
        rows = S.register_rows(us)
        Jr, Hr = orc.estimates(rows)
        assert np.array_equal(Ju[us], Jr) and np.array_equal(Hu[us], Hr), f"{label} estimate terms of rows, pick {k}"
        if k == last_build or k in extra_reg_picks:
            js = rng.choice(J, reg_sims, replace=False)
            checked = 0
            for j in js:
                cov_now = _cover(lg, X, j, seeds)
                cov_build = _cover(lg, X, j, seeds[:last_build])
                for u in rng.choice(us, max(1, reg_samples // reg_sims)):
                    i = int(np.searchsorted(us, u))
                    want = 0 if cov_now[u] else lg.reach_max(int(X[j]), seed, int(j), int(u), cov_build)
                    assert rows[i, j] == want, f"{label} register ({u}, {j}) before pick {k}"
                    checked += 1
                # uncovered at the build, covered since: zero; uncovered now: nonzero
                fresh = np.flatnonzero(cov_now != cov_build)[:200].astype(np.int32)
                if fresh.size:
                    assert np.all(S.register_rows(fresh)[:, j] == 0), f"{label} newly covered, sim {j}, pick {k}"
            assert checked >= min(100, reg_samples)
        if k in full_picks:
            M = S.registers()
            Jf, Hf = orc.estimates(M)
            assert np.array_equal(Ju, Jf) and np.array_equal(Hu, Hf), f"{label} all estimate terms, pick {k}"
            if k > 0:
                sims = range(J) if T_sims is None else T_sims
                zeros = M == 0
                assert int(zeros.sum()) == T_seen[-1], f"{label} T equals the covered registers, pick {k}"
                for j in sims:
                    assert np.array_equal(zeros[:, j], _cover(lg, X, j, seeds).astype(bool)), f"{label} covered set {j}"
            del M
        seeds.append(int(s_k))
        is_seed[s_k] = 1
    r = S.select(K)
    assert list(r["seeds"]) == seeds, f"{label} picks"
    assert [float(e) for e in r["est"]] == expect_est, f"{label} estimates"
    assert [int(t) for t in r["T"][:K - 1]] == T_seen, f"{label} T"
    assert r["stats"]["rebuilds"] == rebuilds, f"{label} rebuilds"
    assert r["spread"] == int(r["T"][-1]) / J
    S.free()
    G.free()
    return r, rebuilds


_GRAPHS = {}


def _cached_graph(key, make):
    if key not in _GRAPHS:
        _GRAPHS[key] = make()
    return _GRAPHS[key]


def test_rmat20_wc_full_size_every_pick(imx, orc):
    """RMAT scale 20, weighted cascade, J=512, K=50 (the many-rebuild
    workload): every pick, estimate and rebuild checked against the oracle at
    full size; all estimate terms and every simulation's covered set at
    several picks."""
    g = _cached_graph("rmat20_wc", lambda: graphgen.with_p(graphgen.rmat(20, 16, seed=1), "wc"))
    _say(f"[c2 every pick] n={g.n} m={g.m}")
    r, rebuilds = stepwise_check(imx, orc, g, 512, 1, 50, reg_samples=120, reg_sims=8,
                                 full_picks=(0, 1, 17, 49), extra_reg_picks=(25, 49), label="c2")
    assert rebuilds >= 10
    _say(f"[c2 every pick] ok: rebuilds={rebuilds} spread={r['spread']:.1f}")


def test_rmat24_p001_full_size_every_pick(imx, orc):
    """RMAT scale 24, p = 0.01, J=1024, K=50 (16 GiB of registers, offsets
    above 2^32): every pick and estimate against the oracle's exact argmax of
    the downloaded terms, sampled registers against the closed form after the
    initial build and the rebuild, covered sets of sampled vertices."""
    base = _cached_graph("rmat24", lambda: graphgen.rmat(24, 16, seed=1))
    g = graphgen.with_p(base, "0.01")
    _say(f"[c3 every pick] n={g.n} m={g.m}")
    r, rebuilds = stepwise_check(imx, orc, g, 1024, 1, 50, reg_samples=120, reg_sims=6,
                                 extra_reg_picks=(20, 49), label="c3")
    assert rebuilds >= 1
    _say(f"[c3 every pick] ok: rebuilds={rebuilds} spread={r['spread']:.1f}")


def test_rmat24_trivalency_full_size_every_pick(imx, orc):
    """The trivalency variant of RMAT-24 (p uniform over {0.1, 0.01, 0.001}
    per arc, seed 2), same topology and checks as the p = 0.01 case."""
    base = _cached_graph("rmat24", lambda: graphgen.rmat(24, 16, seed=1))
    g = graphgen.with_p(base, "trivalency")
    _say(f"[c3 tri every pick] n={g.n} m={g.m}")
    r, rebuilds = stepwise_check(imx, orc, g, 1024, 1, 50, reg_samples=120, reg_sims=6, extra_reg_picks=(49,),
                                 label="c3-tri")
    assert rebuilds >= 1
    _say(f"[c3 tri every pick] ok: rebuilds={rebuilds} spread={r['spread']:.1f}")


def test_pause_and_resume_is_invisible(imx, orc):
    """Pausing before picks (parity hook) changes no output; bad pause points
    are rejected."""
    g = graphgen.with_p(graphgen.rmat(12, 16, seed=3), "wc")
    J, seed, K = 256, 4, 12
    ref = orc.greedy(g, J, seed, K, keep_registers=False)
    G = imx.Graph.from_graphgen(g)
    S = imx.Sketch(G, J, seed)
    s3, T3 = S.select_until(K, 3)
    assert list(s3) == list(ref["seeds"][:3]) and list(T3) == list(ref["T"][:3])
    with pytest.raises(imx.IMError):
        S.select_until(K, 2)  # already past pick 2
    with pytest.raises(imx.IMError):
        S.select_until(K + 1, 5)  # another K
    S.select_until(K, 7)
    r = S.select(K)
    assert list(r["seeds"]) == list(ref["seeds"]) and list(r["T"]) == list(ref["T"])
    assert r["est"].tobytes() == ref["est"].tobytes()
    with pytest.raises(imx.IMError) as ei:
        S.select_until(K, 1)
    assert ei.value.status == 4
    S.free()
    G.free()

"""Host logic of the request loop and the autotuner, with a stand-in engine
(no GPU): FIFO admission, waiting on a full budget, completion of futures,
errors reaching every client, and the autotuner's refusal of tunings that
change outputs."""
import threading

import numpy as np
import pytest

from paper_2410_14047_amd import autotune, serve
from paper_2410_14047_amd.binding import IM_EINVAL, IM_ENOMEM, IMError


class FakeEngine:
    """Admits up to `slots` queries; each finishes after K ticks with a
    deterministic result computed from (J, seed, K)."""

    def __init__(self, max_queries=4, hbm_budget_bytes=0, stream=None, slots=None, fail_at=None):
        self.slots = slots or max_queries
        self.live = {}
        self.done = []
        self.next = 1
        self.ticks = 0
        self.freed = False
        self.admit_order = []
        self.fail_at = fail_at
        self.tuning = None

    def set_tuning(self, **t):
        self.tuning = t

    def submit(self, G, J, seed, K):
        if J <= 0:
            raise IMError(IM_EINVAL, "bad J")
        if len(self.live) >= self.slots:
            raise IMError(IM_ENOMEM, "full")
        qid = self.next
        self.next += 1
        self.live[qid] = [G, J, seed, K, K]
        self.admit_order.append(seed)
        return qid

    def step(self):
        self.ticks += 1
        if self.fail_at is not None and self.ticks >= self.fail_at:
            raise IMError(4, "device failure")
        for qid, q in list(self.live.items()):
            q[4] -= 1
            if q[4] <= 0:
                self.done.append(qid)

    def poll(self):
        out, self.done = self.done, []
        return out

    def result(self, qid):
        G, J, seed, K, _ = self.live.pop(qid)
        return {"seeds": np.arange(K) + seed, "T": np.full(K, J), "spread": float(J * seed), "graph": G}

    def free(self):
        self.freed = True


@pytest.fixture
def fake(monkeypatch):
    made = []

    def factory(**kw):
        def mk(*a, **k):
            e = FakeEngine(*a, **{**k, **kw})
            made.append(e)
            return e
        return mk

    def use(**kw):
        monkeypatch.setattr(serve, "Engine", factory(**kw))
        return made

    return use


def test_server_fifo_admission_and_results(fake):
    made = fake(slots=2)
    srv = serve.Server({"a": "GA", "b": "GB"}, max_queries=2).start()
    futs = [srv.submit("a" if i % 2 else "b", 64, i, 1 + i % 3) for i in range(9)]
    res = [f.result(timeout=10) for f in futs]
    srv.stop()
    eng = made[0]
    assert eng.freed
    assert eng.admit_order == list(range(9))  # arrival order, waiting while full
    for i, r in enumerate(res):
        assert list(r["seeds"]) == list(np.arange(1 + i % 3) + i)
        assert r["graph"] == ("GA" if i % 2 else "GB")
        assert r["latency_s"] >= r["queue_s"] >= 0
    assert len(srv.completed) == 9


def test_server_unknown_graph_and_rejected_query(fake):
    fake(slots=2)
    srv = serve.Server({"a": "GA"}, max_queries=2).start()
    with pytest.raises(KeyError):
        srv.submit("zzz", 64, 0, 1)
    bad = srv.submit("a", 0, 0, 1)  # rejected by the engine: the client sees the error
    good = srv.submit("a", 64, 1, 2)
    with pytest.raises(IMError):
        bad.result(timeout=10)
    assert good.result(timeout=10)["spread"] == 64.0
    srv.stop()


def test_server_loop_failure_reaches_clients(fake):
    fake(slots=4, fail_at=2)
    srv = serve.Server({"a": "GA"}, max_queries=4).start()
    futs = [srv.submit("a", 64, i, 5) for i in range(3)]
    for f in futs:
        with pytest.raises(IMError):
            f.result(timeout=10)
    with pytest.raises(IMError):
        srv.stop()  # the loop's exception is raised to the owner as well


def test_replay_and_summary(fake):
    fake(slots=3)
    srv = serve.Server({"a": "GA"}, max_queries=3).start()
    trace = [(0.001 * i, "a", 64, i, 2) for i in range(12)]
    res, span = serve.replay(srv, trace)
    srv.stop()
    s = serve.latency_summary(res, span)
    assert s["queries"] == 12 and s["p99_ms"] >= s["p50_ms"] > 0 and s["throughput_qps"] > 0


def test_autotune_picks_fastest_and_rejects_changed_outputs(monkeypatch):
    calls = []

    class TEngine:
        def __init__(self, max_queries=1, stream=None):
            self.t = None
            self.q = {}

        def set_tuning(self, **t):
            self.t = t

        def submit(self, G, J, s, K):
            self.q[len(self.q) + 1] = (J, s, K)
            return len(self.q)

        def run(self):
            calls.append(self.t)
            bad = self.t.get("dense_div") == 3
            return {i: {"seeds": np.array([s + (1 if bad else 0)]), "T": np.array([J]),
                        "est": np.array([1.0])} for i, (J, s, K) in self.q.items()}

        def free(self):
            pass

    monkeypatch.setattr(autotune, "Engine", TEngine)
    clock = iter(np.arange(0, 1000, 0.5).tolist())
    monkeypatch.setattr(autotune.time, "perf_counter", lambda: next(clock))
    qs = [("G", 64, s, 2) for s in range(3)]
    cands = [dict(group_first=64, group_rest=64, rounds_per_step=4, dense_div=16),
             dict(group_first=32, group_rest=16, rounds_per_step=2, dense_div=8)]
    out = autotune.autotune(qs, candidates=cands)
    assert out["best"] in cands and len(out["table"]) == 2
    assert calls[0] == autotune.DEFAULT  # reference run first
    with pytest.raises(RuntimeError):
        autotune.autotune(qs, candidates=[dict(group_first=64, group_rest=64, rounds_per_step=4, dense_div=3)])


def test_candidate_grid_respects_row_width():
    ok = lambda v, lo: v == 0 or v >= lo  # 0 = packed propagation
    assert all(ok(c["group_first"], 32) and ok(c["group_rest"], 32) for c in autotune.candidate_grid(2048))
    assert all(ok(c["group_first"], 64) for c in autotune.candidate_grid(4096))
    assert {c["group_first"] for c in autotune.candidate_grid(512)} == {0, 16, 32, 64}


class _G:
    def __init__(self, name):
        self.handle = name


def test_server_routes_by_footprint(fake, monkeypatch):
    made = fake(slots=2)
    monkeypatch.setattr(serve, "im_query_footprint", lambda h, J, K: J * 1000)
    srv = serve.Server({"a": _G("A")}, max_queries=2, lanes=[200_000], streams=[None, None]).start()
    futs = [srv.submit("a", J, i, 2) for i, J in enumerate([64, 512, 128, 1024, 192])]
    res = [f.result(timeout=10) for f in futs]
    srv.stop()
    assert [r["lane"] for r in res] == [0, 1, 0, 1, 0]
    small, large = made
    assert small.admit_order == [0, 2, 4] and large.admit_order == [1, 3]
    assert small.freed and large.freed


def test_server_routes_quick_classes_to_first_lane(fake, monkeypatch):
    """A class (graph, J) seen to finish within quick_s goes to the first lane
    whatever its footprint; classes not seen yet, or slower, keep the
    footprint's lane."""
    fake(slots=2)
    monkeypatch.setattr(serve, "im_query_footprint", lambda h, J, K: J * 1000)
    srv = serve.Server({"a": _G("A"), "b": _G("B")}, max_queries=2, lanes=[200_000], streams=[None, None],
                       quick_s=60.0).start()
    first = srv.submit("a", 512, 1, 2).result(timeout=10)
    assert first["lane"] == 1                      # not seen yet: by footprint
    again = srv.submit("a", 512, 2, 2).result(timeout=10)
    other_j = srv.submit("a", 1024, 3, 2).result(timeout=10)
    other_g = srv.submit("b", 512, 4, 2).result(timeout=10)
    srv.stop()
    assert again["lane"] == 0                      # seen to finish within quick_s
    assert other_j["lane"] == 1 and other_g["lane"] == 1
    assert list(again["seeds"]) == [2, 3]          # results do not depend on the lane

    srv = serve.Server({"a": _G("A")}, max_queries=2, lanes=[200_000], streams=[None, None], quick_s=0.0).start()
    srv._observe("a", 512, 0.001)
    assert srv._route("a", 512, 2) is srv.lanes[1]  # quick_s = 0: footprint only
    srv.stop()
    srv = serve.Server({"a": _G("A")}, max_queries=2, lanes=[200_000], streams=[None, None], quick_s=0.05).start()
    srv._observe("a", 512, 0.2)
    assert srv._route("a", 512, 2) is srv.lanes[1]  # slower than quick_s
    srv._observe("a", 512, 0.04)
    assert srv._route("a", 512, 2) is srv.lanes[0]  # the shortest time counts
    srv.stop()

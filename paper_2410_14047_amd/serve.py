"""Serving loop: IM queries (graph, J, seed, K) arrive at any time and are
served by continuous batching.

Graphs (one per topology and probability scheme) stay resident on the device.
Each *lane* is one engine with its own stream and loop thread: it admits its
waiting requests in arrival order while their device footprint fits its
budget and a slot is free, advances every admitted query one stage per engine
step (their kernels share launches), and completes each request's future when
its query finishes, releasing its memory for the next admissions.

Queries are routed to lanes by device footprint (n * J plus work arrays):
small queries finish in a few hundred launches, large ones in a few
thousand, and a step lasts as long as its largest query, so keeping them on
separate engines (whose streams run concurrently on the GPU) stops small
queries from waiting in lock step behind large ones.  Footprint is not
work, though: on a subcritical probability setting a query on a large graph
converges in a few sweeps and short cascades.  With `quick_s` set, the server
learns, per (graph, J), the shortest time a query of that class has spent in
an engine (admission to completion), and sends a class seen to finish within
`quick_s` to the first lane whatever its footprint, so such queries do not
queue behind the long ones of their footprint's lane.  Latency is measured
from submit() to completion.  Results do not depend on the lane or the mix.
"""
from __future__ import annotations

import collections
import threading
import time
from concurrent.futures import Future
from typing import Dict, List, Optional, Sequence

from .binding import IM_ENOMEM, Engine, Graph, IMError, im_query_footprint


class _Lane:
    def __init__(self, server: "Server", index: int, max_queries: int, hbm_budget_bytes: int,
                 tuning: Optional[dict], stream):
        self.server = server
        self.index = index
        self.engine = Engine(max_queries=max_queries, hbm_budget_bytes=hbm_budget_bytes, stream=stream)
        if tuning:
            self.engine.set_tuning(**tuning)
        self.stream = stream
        self.wait = collections.deque()
        self.live = {}
        self.steps = 0
        self.thread: Optional[threading.Thread] = None

    def admit(self) -> None:
        srv = self.server
        while True:
            with srv._cv:
                if not self.wait:
                    return
                req = self.wait[0]
            try:
                qid = self.engine.submit(srv.graphs[req["graph"]], req["J"], req["seed"], req["K"])
            except IMError as e:
                if e.status == IM_ENOMEM and self.live:
                    return  # wait for memory or a slot to free up
                with srv._cv:
                    self.wait.popleft()
                req["future"].set_exception(e)
                continue
            req["t_admit"] = time.perf_counter()
            with srv._cv:
                self.wait.popleft()
            self.live[qid] = req

    def loop(self) -> None:
        srv = self.server
        try:
            while True:
                with srv._cv:
                    while not srv._stop and not self.wait and not self.live and srv.error is None:
                        srv._cv.wait()
                    if srv.error is not None or (srv._stop and not self.live and not self.wait):
                        return
                self.admit()
                if self.live:
                    self.engine.step()
                    self.steps += 1
                    for qid in self.engine.poll():
                        req = self.live.pop(qid)
                        res = self.engine.result(qid)
                        req["t_done"] = time.perf_counter()
                        srv._observe(req["graph"], req["J"], req["t_done"] - req["t_admit"])
                        res["latency_s"] = req["t_done"] - req["t_arrival"]
                        res["queue_s"] = req["t_admit"] - req["t_arrival"]
                        res["lane"] = self.index
                        with srv._cv:
                            srv.completed.append(res)
                        req["future"].set_result(res)
        except BaseException as e:  # surface loop failures to every client and to stop()
            srv._fail(e)


class Server:
    """lanes: ascending footprint bounds in bytes of every lane but the last;
    a query goes to the first lane whose bound is at least its footprint, and
    to the last lane otherwise (None: one lane).  max_queries (one value, or one per lane)
    and hbm_budget_bytes apply per lane; a lane of large queries with one slot
    serves them first come, first served while the other lanes interleave
    small ones.  `tuning` (one engine tuning, or one per lane) can cap the
    workgroups of the small-query lanes' launches (grid_cap), so that their
    work fills the device around a large query instead of displacing it.
    `streams` (optional) gives each lane's stream; by default a new torch
    stream per lane, or `stream` when there is one lane.  `quick_s` (seconds,
    0: off) routes classes (graph, J) seen to finish within it in an engine to
    the first lane."""

    def __init__(self, graphs: Dict[str, Graph], max_queries=32, hbm_budget_bytes: int = 0,
                 tuning: Optional[dict] = None, stream=None, lanes: Optional[Sequence[int]] = None,
                 streams: Optional[Sequence] = None, quick_s: float = 0.0):
        self.graphs = dict(graphs)
        self.quick_s = float(quick_s)
        self._shortest: Dict[tuple, float] = {}  # (graph, J) -> shortest admission-to-completion time
        self.bounds: List[int] = list(lanes) if lanes else []
        nl = len(self.bounds) + 1
        if streams is None:
            if nl == 1:
                streams = [stream]
            else:
                import torch
                streams = [torch.cuda.Stream() for _ in range(nl)]
        self._cv = threading.Condition()
        self._stop = False
        self.error: Optional[BaseException] = None
        self.completed = []
        slots = list(max_queries) if isinstance(max_queries, (list, tuple)) else [max_queries] * nl
        if len(slots) != nl:
            raise ValueError("max_queries needs one value per lane")
        tunings = list(tuning) if isinstance(tuning, (list, tuple)) else [tuning] * nl
        if len(tunings) != nl:
            raise ValueError("tuning needs one value per lane")
        self.lanes = [_Lane(self, i, slots[i], hbm_budget_bytes, tunings[i], streams[i]) for i in range(nl)]

    @property
    def steps(self) -> int:
        return sum(l.steps for l in self.lanes)

    def _observe(self, graph: str, J: int, seconds: float) -> None:
        with self._cv:
            key = (graph, J)
            self._shortest[key] = min(seconds, self._shortest.get(key, float("inf")))

    def _route(self, graph: str, J: int, K: int) -> _Lane:
        if len(self.lanes) == 1:
            return self.lanes[0]
        if self.quick_s > 0 and self._shortest.get((graph, J), float("inf")) <= self.quick_s:
            return self.lanes[0]
        need = im_query_footprint(self.graphs[graph].handle, J, K)
        for lane, bound in zip(self.lanes, self.bounds):
            if need <= bound:
                return lane
        return self.lanes[-1]

    # -------------------------------------------------------------- client side
    def submit(self, graph: str, J: int, seed: int, K: int) -> Future:
        if graph not in self.graphs:
            raise KeyError(graph)
        lane = self._route(graph, J, K)
        fut: Future = Future()
        req = dict(graph=graph, J=J, seed=seed, K=K, t_arrival=time.perf_counter(), future=fut)
        with self._cv:
            if self.error is not None:
                raise RuntimeError("the serving loop has failed") from self.error
            lane.wait.append(req)
            self._cv.notify_all()
        return fut

    def start(self) -> "Server":
        for lane in self.lanes:
            lane.thread = threading.Thread(target=lane.loop, name=f"im-serve-{lane.index}", daemon=True)
            lane.thread.start()
        return self

    def stop(self) -> None:
        with self._cv:
            self._stop = True
            self._cv.notify_all()
        for lane in self.lanes:
            if lane.thread:
                lane.thread.join()
        for lane in self.lanes:
            lane.engine.free()
        if self.error is not None:
            raise self.error

    def _fail(self, e: BaseException) -> None:
        with self._cv:
            if self.error is None:
                self.error = e
            reqs = []
            for lane in self.lanes:
                reqs += list(lane.live.values()) + list(lane.wait)
                lane.wait.clear()
            self._cv.notify_all()
        for lane in self.lanes:
            lane.live.clear()
        for req in reqs:
            if not req["future"].done():
                req["future"].set_exception(e)


def replay(server: Server, trace, time_scale: float = 1.0, progress=None, every: int = 50):
    """Submit a trace of (t_arrival_s, graph, J, seed, K) at its arrival times;
    return (results in trace order, makespan seconds).  `progress(i, n)` (if
    given) is called after every `every` submissions and completions."""
    t0 = time.perf_counter()
    futs = []
    for i, (ta, graph, J, seed, K) in enumerate(trace):
        delay = t0 + ta * time_scale - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        futs.append(server.submit(graph, J, seed, K))
        if progress and (i + 1) % every == 0:
            progress("submitted", i + 1)
    res = []
    for i, f in enumerate(futs):
        res.append(f.result())
        if progress and (i + 1) % every == 0:
            progress("completed", i + 1)
    return res, time.perf_counter() - t0


def latency_summary(results, makespan: float) -> dict:
    import numpy as np
    lat = np.array([r["latency_s"] for r in results]) * 1e3
    return {"queries": len(results), "throughput_qps": len(results) / makespan,
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "makespan_s": makespan}

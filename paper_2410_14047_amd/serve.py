"""Serving loop: IM queries (graph, J, seed, K) arrive at any time and are
served by continuous batching on one engine.

Graphs (one per topology and probability scheme) stay resident on the device.
A loop thread admits waiting requests in arrival order while their device
footprint fits the engine's budget and a slot is free, advances every admitted
query one stage per engine step (their kernels share launches), and completes
each request's future when its query finishes, releasing its memory for the
next admissions.  Latency is measured from submit() to completion.
"""
from __future__ import annotations

import collections
import threading
import time
from concurrent.futures import Future
from typing import Dict, Optional

from .binding import IM_ENOMEM, Engine, Graph, IMError


class Server:
    def __init__(self, graphs: Dict[str, Graph], max_queries: int = 32, hbm_budget_bytes: int = 0,
                 tuning: Optional[dict] = None, stream=None):
        self.graphs = dict(graphs)
        self.engine = Engine(max_queries=max_queries, hbm_budget_bytes=hbm_budget_bytes, stream=stream)
        if tuning:
            self.engine.set_tuning(**tuning)
        self._wait = collections.deque()
        self._live = {}
        self._cv = threading.Condition()
        self._stop = False
        self._thread: Optional[threading.Thread] = None
        self.steps = 0
        self.completed = []
        self.error: Optional[BaseException] = None

    # -------------------------------------------------------------- client side
    def submit(self, graph: str, J: int, seed: int, K: int) -> Future:
        if graph not in self.graphs:
            raise KeyError(graph)
        fut: Future = Future()
        req = dict(graph=graph, J=J, seed=seed, K=K, t_arrival=time.perf_counter(), future=fut)
        with self._cv:
            if self.error is not None:
                raise RuntimeError("the serving loop has failed") from self.error
            self._wait.append(req)
            self._cv.notify()
        return fut

    def start(self) -> "Server":
        self._thread = threading.Thread(target=self._loop, name="im-serve", daemon=True)
        self._thread.start()
        return self

    def stop(self) -> None:
        with self._cv:
            self._stop = True
            self._cv.notify()
        if self._thread:
            self._thread.join()
        self.engine.free()
        if self.error is not None:
            raise self.error

    # -------------------------------------------------------------- loop thread
    def _admit(self) -> None:
        while True:
            with self._cv:
                if not self._wait:
                    return
                req = self._wait[0]
            try:
                qid = self.engine.submit(self.graphs[req["graph"]], req["J"], req["seed"], req["K"])
            except IMError as e:
                if e.status == IM_ENOMEM and self._live:
                    return  # wait for memory or a slot to free up
                with self._cv:
                    self._wait.popleft()
                req["future"].set_exception(e)
                continue
            req["t_admit"] = time.perf_counter()
            with self._cv:
                self._wait.popleft()
            self._live[qid] = req

    def _loop(self) -> None:
        try:
            while True:
                with self._cv:
                    while not self._stop and not self._wait and not self._live:
                        self._cv.wait()
                    if self._stop and not self._live and not self._wait:
                        return
                self._admit()
                if self._live:
                    self.engine.step()
                    self.steps += 1
                    for qid in self.engine.poll():
                        req = self._live.pop(qid)
                        res = self.engine.result(qid)
                        req["t_done"] = time.perf_counter()
                        res["latency_s"] = req["t_done"] - req["t_arrival"]
                        res["queue_s"] = req["t_admit"] - req["t_arrival"]
                        self.completed.append(res)
                        req["future"].set_result(res)
        except BaseException as e:  # surface loop failures to every client and to stop()
            with self._cv:
                self.error = e
                reqs = list(self._live.values()) + list(self._wait)
                self._wait.clear()
            self._live.clear()
            for req in reqs:
                if not req["future"].done():
                    req["future"].set_exception(e)


def replay(server: Server, trace, time_scale: float = 1.0):
    """Submit a trace of (t_arrival_s, graph, J, seed, K) at its arrival times;
    return (results in trace order, makespan seconds)."""
    t0 = time.perf_counter()
    futs = []
    for (ta, graph, J, seed, K) in trace:
        delay = t0 + ta * time_scale - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        futs.append(server.submit(graph, J, seed, K))
    res = [f.result() for f in futs]
    return res, time.perf_counter() - t0


def latency_summary(results, makespan: float) -> dict:
    import numpy as np
    lat = np.array([r["latency_s"] for r in results]) * 1e3
    return {"queries": len(results), "throughput_qps": len(results) / makespan,
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "makespan_s": makespan}

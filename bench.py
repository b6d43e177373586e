#!/usr/bin/env python
"""Benchmark of the sketch-based IM hot path on one MI355X.

One step = im_sketch_build (fill + propagation to the fixed point + estimate
terms) followed by im_select_seeds(K) (K x [argmax, covering cascade, score,
error-adaptive rebuild]) on a device-resident synthetic graph.

value = live-edge register updates per second over the whole step:
        sum over steps of J * m * sweeps / wall time of the timed steps,
where `sweeps` counts every propagation sweep the step ran (initial build and
rebuilds).  The JSON line also carries the propagation kernel's HBM roofline
(algorithmic bytes per launch / average launch time, from HIP events around
each launch) and the CPU oracle's rate on a bounded sample of the same
workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "live-edge register updates/sec (J×edges×iters/s), %HBM peak; K-seed wall time; p50/p99 query latency"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    # RMAT scale 20, edge factor 16, weighted cascade, J=512, K=50 (single query, plain method)
    "rmat20_wc_J512_K50": dict(kind="rmat", scale=20, ef=16, scheme="wc", J=512, K=50, gseed=1, sseed=1),
    # Erdos-Renyi n=1000, m=5000, p=0.1, J=64, K=10
    "er1k_p0.1_J64_K10": dict(kind="er", n=1000, m=5000, scheme="0.1", J=64, K=10, gseed=1, sseed=1),
    # RMAT scale 24, edge factor 16, J=1024, K=50: uniform p=0.01 and the trivalency mix
    "rmat24_p0.01_J1024_K50": dict(kind="rmat", scale=24, ef=16, scheme="0.01", J=1024, K=50, gseed=1, sseed=1),
    "rmat24_tri_J1024_K50": dict(kind="rmat", scale=24, ef=16, scheme="trivalency", J=1024, K=50, gseed=1,
                                 sseed=1),
}
# Ablation: the same RMAT-24 graph without the random vertex relabelling
# (RMAT's own id order, hubs at ids with many zero bits).
WORKLOADS["rmat24_p0.01_J1024_K50_unpermuted"] = dict(WORKLOADS["rmat24_p0.01_J1024_K50"], relabel=False)
# Road-network stand-in (the paper's named weak case: high diameter, few arcs
# per vertex): 1024 x 1024 lattice of two-way links, 10% removed.
WORKLOADS["road1024_p0.3_J256_K50"] = dict(kind="road", width=1024, drop=0.1, scheme="0.3", J=256, K=50, gseed=1,
                                           sseed=1)
WORKLOADS["road1024_p0.6_J256_K50"] = dict(kind="road", width=1024, drop=0.1, scheme="0.6", J=256, K=50, gseed=1,
                                           sseed=1)
DEFAULT = "rmat24_p0.01_J1024_K50"
# Workloads measured beside the default in the same run (same topology, another
# probability scheme), reported in the line's `variants` field.
VARIANTS = {"rmat24_p0.01_J1024_K50": ["rmat24_tri_J1024_K50"]}


def make_graph(w):
    import graphgen
    if w["kind"] == "rmat":
        g = graphgen.rmat(w["scale"], w["ef"], seed=w["gseed"], relabel=w.get("relabel", True))
    elif w["kind"] == "road":
        g = graphgen.road_grid(w["width"], w["width"], w["drop"], seed=w["gseed"])
    else:
        g = graphgen.erdos_renyi(w["n"], w["m"], w["gseed"])
    return graphgen.with_p(g, w["scheme"])


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("kernels.hip", "imx_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_2410_14047_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def pmc_traffic(workload: str, launches_bytes_per_launch: float):
    """HBM traffic per propagation launch from committed rocprofv3 counter runs,
    if they were taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"propagate_{workload}_pmc.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def _counter_rows(path: str, counter: str):
    """(kernel name, value) per dispatch from a rocprofv3 counter_collection.csv."""
    import csv
    out = []
    with open(path, newline="") as f:
        for r in csv.DictReader(f):
            if r.get("Counter_Name") == counter:
                out.append((r["Kernel_Name"], float(r["Counter_Value"])))
    return out


def pmc_summary(args):
    """HBM bytes per k_propagate launch from FETCH_SIZE and WRITE_SIZE (KiB per
    dispatch), each scaled by the factor that makes the same counter read the
    known traffic of a plain device copy (read n bytes, write n bytes)."""
    import numpy as np
    fetch, write, cfetch, cwrite = args.pmc_summary
    copy_bytes = args.copy_calibration << 20 if args.copy_calibration else 1 << 30

    def big(rows):  # the copy kernel is the dispatch with the largest count
        return max(v for _, v in rows)

    f_fetch = copy_bytes / (big(_counter_rows(cfetch, "FETCH_SIZE")) * 1024)
    f_write = copy_bytes / (big(_counter_rows(cwrite, "WRITE_SIZE")) * 1024)
    fr = [v for k, v in _counter_rows(fetch, "FETCH_SIZE") if "k_propagate" in k]
    wr = [v for k, v in _counter_rows(write, "WRITE_SIZE") if "k_propagate" in k]
    if not fr or not wr:
        raise SystemExit("no k_propagate dispatches in the counter files")
    fb = float(np.mean(fr)) * 1024 * f_fetch
    wb = float(np.mean(wr)) * 1024 * f_write
    d = {"workload": args.workload, "kernel": "k_propagate_pack", "kernel_source_hash": kernel_source_hash(),
         "dispatches": [len(fr), len(wr)], "fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb,
         "hbm_bytes_per_launch": fb + wb, "copy_calibration": {"bytes": copy_bytes, "fetch_factor": f_fetch,
                                                               "write_factor": f_write},
         "command": args.pmc_command}
    path = os.path.join(ROOT, "profiles", f"propagate_{args.workload}_pmc.json")
    with open(path, "w") as f:
        json.dump(d, f, indent=1)
    print(json.dumps(d))


def liveness_stats():
    """How an arc's live simulations spread over the J = 1024 sorted
    simulation values, which decides what sample-space tiling could save on
    one GPU: live simulations per arc, arcs dead in all of them, 128-simulation
    tiles with a live one, and 64-byte register sectors the candidate range
    touches.  Uniform 31-bit arc hashes and uniform simulation values (the
    distribution the hash and the simulation-value generator are built to
    give); CPU only."""
    import numpy as np
    rng = np.random.default_rng(7)
    J, T = 1024, 128
    X = np.sort(rng.integers(0, 2**31, J, dtype=np.int64))
    for p in (0.001, 0.005, 0.01, 0.1):
        W = int(np.floor(np.float32(p) * 2**31))
        h = rng.integers(0, 2**31, 200_000, dtype=np.int64)
        live = (X[None, :] ^ h[:, None]) < W  # arcs x simulations
        nlive = live.sum(1)
        tiles = live.reshape(len(h), J // T, T).any(2).sum(1)
        first = np.where(nlive > 0, live.argmax(1), 0)
        last = np.where(nlive > 0, J - 1 - live[:, ::-1].argmax(1), -1)
        sectors = np.where(nlive > 0, last // 64 - first // 64 + 1, 0)
        print(json.dumps({"p": p, "live_sims_per_arc": float(nlive.mean()), "dead_arcs": float(np.mean(nlive == 0)),
                          f"live_{T}_sim_tiles_per_arc": float(tiles.mean()),
                          "sectors_per_arc": float(sectors.mean())}), flush=True)


def gather_calibration(mib: int):
    """Access-rate ceilings of the device memory (libimx_probe.so): random
    gathers of 16 B (from 64-byte-aligned positions), 64, 128, 256 and 1024 B,
    a streaming read and a streaming copy, on a MIB MiB buffer; one JSON line."""
    import ctypes

    import torch
    torch.cuda.set_device(0)  # the probe library then binds torch's HIP runtime
    from paper_2410_14047_amd.build import PROBE_LIB
    if not os.path.exists(PROBE_LIB):
        raise SystemExit(f"{PROBE_LIB} missing: run __graft_entry__.build()")
    L = ctypes.CDLL(PROBE_LIB)
    L.imx_probe_rates.argtypes = [ctypes.c_uint64, ctypes.POINTER(ctypes.c_double)]
    L.imx_probe_rates.restype = ctypes.c_int
    r = (ctypes.c_double * 7)()
    rc = L.imx_probe_rates(ctypes.c_uint64(mib << 20), r)
    if rc != 0:
        raise SystemExit(f"probe failed with HIP error {rc}")
    sizes = (16, 64, 128, 256, 1024)
    out = {"buffer_bytes": mib << 20,
           "gathers": [{"bytes": b, "per_s": r[i], "lines128_per_s": r[i] * max(1, b // 128),
                        "GBps_at_gather_size": r[i] * b / 1e9} for i, b in enumerate(sizes)],
           "stream_read_GBps": r[5] / 1e9, "stream_copy_GBps": r[6] / 1e9}
    print(json.dumps(out), flush=True)


def cpu_info():
    """Host CPU as /proc/cpuinfo names it: model name, with the family, model
    and stepping numbers and the clock (a virtual machine may report only a
    generic model name)."""
    f = {}
    try:
        for line in open("/proc/cpuinfo"):
            if ":" in line:
                k, v = (x.strip() for x in line.split(":", 1))
                if k in ("model name", "cpu family", "model", "stepping", "cpu MHz") and k not in f:
                    f[k] = v
            elif f:
                break
    except OSError:
        pass
    if not f:
        return ""
    return (f"{f.get('model name', '?')} (family {f.get('cpu family', '?')}, model {f.get('model', '?')}, "
            f"stepping {f.get('stepping', '?')}, {f.get('cpu MHz', '?')} MHz)")


def cpu_baseline(g, w, budget_s: float, threads: int):
    """The oracle, as it stands, running full synchronous sweeps over a sample
    of the J simulation columns of the same graph; the columns are split over
    `threads` host threads, each running the oracle on its own columns
    (simulations are independent)."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np
    import oracle
    J, seed = w["J"], w["sseed"]
    t0 = time.perf_counter()
    oracle.sweeps_sample(g, J, seed, np.arange(16, dtype=np.int32), 1)
    per_col_sweep = max((time.perf_counter() - t0) / 16, 1e-4)
    per_thread = int(max(1, min(J // threads if J >= threads else 1, budget_s / per_col_sweep / 2)))
    S = min(J, per_thread * threads)
    # more sweeps when every column fits in the budget (at most 8)
    sweeps = int(max(2, min(8, budget_s / (per_col_sweep * max(1, S // threads)))))
    sims = np.linspace(0, J - 1, S).astype(np.int32)
    parts = [p for p in np.array_split(sims, threads) if len(p)]
    t0 = time.perf_counter()
    with ThreadPoolExecutor(len(parts)) as ex:
        list(ex.map(lambda p: oracle.sweeps_sample(g, J, seed, p, sweeps), parts))
    dt = time.perf_counter() - t0
    rate = S * g.m * sweeps / dt
    return {"value": rate, "unit": "register updates/s", "cores": len(parts), "kind": "oracle",
            "cpu": cpu_info(), "host_cpus": os.cpu_count(),
            "sample": f"{sweeps} synchronous sweeps (from fill) over {S} of {J} simulation columns, "
                      f"all {g.m} arcs, {len(parts)} threads over disjoint columns; {dt:.1f} s"}


def batched_main(args):
    print(json.dumps(batched_result(tune=True)), flush=True)


def batched_result(tune: bool = True) -> dict:
    """64 independent graphs of uneven size (32 RMAT, scales 12-18; 32
    Barabasi-Albert, n 10k-200k, m0=8), weighted cascade, J=256, K=20, sketch
    seeds 0..63: one engine (batched launches) against one query per launch
    (sequential one-query engines), with identical outputs required.  With
    `tune`, the engine's tuning is autotuned on every 8th query first;
    otherwise the library's defaults are used."""
    import torch

    import graphgen
    import paper_2410_14047_amd as imx
    from paper_2410_14047_amd import autotune

    t0 = time.perf_counter()
    gs = [graphgen.batched_graph(spec) for spec in graphgen.batched_specs()]
    print(f"[bench] 64 graphs, {sum(g.m for g in gs)} arcs ({time.perf_counter() - t0:.1f} s)", file=sys.stderr,
          flush=True)
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    Gs = [imx.Graph.from_graphgen(g, stream=stream) for g in gs]
    J, K = 256, 20
    queries = [(G, J, i, K) for i, G in enumerate(Gs)]

    # autotune on every 8th query (not timed)
    if tune:
        tuned = autotune.autotune(queries[::8], candidates=[
            dict(group_first=gf, group_rest=gr, rounds_per_step=r, dense_div=16)
            for gf in (0, 64) for gr in (0, 32, 64) for r in (4, 8, 16)], stream=stream)
        tuning = tuned["best"]
    else:
        tuning = {}
    print(f"[bench] tuning {tuning or 'library defaults'}", file=sys.stderr, flush=True)

    counters = {}

    def run_batched(graphs=0):
        E = imx.Engine(max_queries=64, stream=stream)
        E.set_tuning(**{**tuning, "use_graphs": graphs})
        ids = [E.submit(*q) for q in queries]
        res = E.run()
        counters["graphs" if graphs else "direct"] = E.counters()
        E.free()
        return [res[i] for i in ids]

    def run_single():
        out = []
        for (G, J_, s, K_) in queries:
            S = imx.Sketch(G, J_, s, stream=stream)
            out.append(S.select(K_))
            S.free()
        return out

    run_batched()  # warm-up
    times = {}
    run_batched(1)  # warm-up of graph mode
    for name, fn in (("batched", run_batched), ("batched_hip_graphs", lambda: run_batched(1)),
                     ("one_query_per_launch", run_single)):
        torch.cuda.synchronize()
        t = time.perf_counter()
        res = fn()
        torch.cuda.synchronize()
        times[name] = (time.perf_counter() - t, res)
        print(f"[bench] {name}: {times[name][0]:.3f} s", file=sys.stderr, flush=True)
    a, b = times["batched"][1], times["one_query_per_launch"][1]
    for other in (b, times["batched_hip_graphs"][1]):
        for ra, rb in zip(a, other):
            assert list(ra["seeds"]) == list(rb["seeds"]) and list(ra["T"]) == list(rb["T"]), "outputs differ"
    upd = sum(J * G.m * r["stats"]["total_sweeps"] for G, r in zip(Gs, a))
    tb, ts = times["batched"][0], times["one_query_per_launch"][0]
    for G in Gs:
        G.free()
    return {
        "metric": "batched IM queries: wall time of 64 queries (and register updates/s)",
        "value": 64 / tb, "unit": "queries/s", "n_gpus": 1, "higher_is_better": True,
        "batched_s": tb, "batched_hip_graphs_s": times["batched_hip_graphs"][0], "one_query_per_launch_s": ts,
        "speedup": ts / tb, "engine_counters": counters,
        "register_updates_per_s": upd / tb, "identical_outputs": True, "tuning": tuning,
        "config": {"workload": "batched64_rmat12-18_ba10k-200k_wc_J256_K20", "graphs": 64,
                   "arcs": int(sum(g.m for g in gs)), "J": J, "K": K},
        "data": "synthetic", "dtype": "u8"}


def fifo_latencies(arrivals, service):
    """Time in system of each request at one first-come-first-served server
    that is never idle while requests wait: request i starts at the later of
    its arrival and the previous finish.  Returns (latencies, last finish)."""
    fin, lat = 0.0, []
    for ta, st in zip(arrivals, service):
        fin = max(fin, float(ta)) + float(st)
        lat.append(fin - float(ta))
    return lat, fin


def served_main(args):
    """Poisson stream of IM queries over device-resident graphs (RMAT scales
    given by --served-scales, edge factor 16, two p-schemes each), J in
    {128, 512}, K uniform in [10, 100]: continuous batching against a serial
    one-query-at-a-time server.

    The serial server is measured once per query: every query runs alone,
    back to back, through a one-slot server (submit to result), which gives its
    service time and its outputs.  A FIFO single server is work-conserving, so
    its latencies on any arrival trace follow exactly from those service times
    (start = max(arrival, previous finish)).  Continuous batching is replayed
    in real time on the trace of each load level; its outputs must equal the
    serial ones query by query.  --served-service-out / --served-service-in
    save and reuse the serial pass, so the load levels of a long run can be
    replayed in separate processes."""
    import numpy as np
    import torch

    import graphgen
    import paper_2410_14047_amd as imx
    from paper_2410_14047_amd import serve

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    scales = [int(x) for x in args.served_scales.split(",")]
    graphs = {}
    t0 = time.perf_counter()
    for name in graphgen.served_graph_names(scales):
        graphs[name] = imx.Graph.from_graphgen(graphgen.served_graph(name, scales), stream=stream)
    print(f"[bench] {len(graphs)} resident graphs ({time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)
    nq = args.served_queries
    reqs = graphgen.served_requests(nq, scales)

    if args.served_service_in:
        sv = json.load(open(args.served_service_in))
        assert sv["queries"] == nq and sv["scales"] == args.served_scales, "service file of another workload"
        service, serial_out = sv["service_s"], sv["outputs"]
    else:
        srv = serve.Server(graphs, max_queries=1, stream=stream).start()
        service, serial_out = [], []
        for i, (gname, J, s, K) in enumerate(reqs):
            r = srv.submit(gname, J, s, K).result()
            service.append(r["latency_s"])
            serial_out.append({"seeds": [int(x) for x in r["seeds"]], "T": [int(x) for x in r["T"]]})
            if i % 50 == 0:
                print(f"[bench] serial pass {i}/{nq}: {sum(service):.1f} s", file=sys.stderr, flush=True)
        srv.stop()
        if args.served_service_out:
            json.dump({"queries": nq, "scales": args.served_scales, "service_s": service, "outputs": serial_out},
                      open(args.served_service_out, "w"))
    svc = float(np.mean(service))
    # the trace of each load level: arrivals from their own seeded stream
    out = {"metric": "served IM queries: throughput and p50/p99 latency",
           "unit": "queries/s", "n_gpus": 1, "mean_serial_service_s": svc, "levels": []}
    lanes = [int(x) << 20 for x in args.served_lanes_mib.split(",")]
    nl = len(lanes) + 1

    def per_lane(text, what):  # one value for every lane, or one per lane
        v = [int(x) for x in text.split(",")]
        if len(v) == 1:
            v = v * nl
        if len(v) != nl:
            raise SystemExit(f"--served-{what} needs 1 or {nl} values")
        return v

    slots = per_lane(args.served_slots, "slots")
    tunings = [dict(grid_cap=c, use_graphs=u) for c, u in
               zip(per_lane(args.served_caps, "caps"), per_lane(args.served_graphs, "graphs"))]
    for load in [float(x) for x in args.served_loads.split(",")]:
        lam = load / svc
        arr = np.cumsum(np.random.Generator(np.random.PCG64(int(round(load * 1000)))).exponential(1.0 / lam, size=nq))
        trace = [(float(t), *r) for t, r in zip(arr, reqs)]
        # serial: FIFO single server on the measured service times
        lat, fin = fifo_latencies(arr, service)
        lat = np.array(lat) * 1e3
        row = {"load": load, "lambda_qps": lam,
               "serial": {"queries": nq, "throughput_qps": nq / fin, "p50_ms": float(np.percentile(lat, 50)),
                          "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(lat.mean()), "makespan_s": fin}}
        srv = serve.Server(graphs, max_queries=slots, stream=stream, lanes=lanes, tuning=tunings,
                           quick_s=args.served_quick_ms * 1e-3).start()
        t_rep = time.perf_counter()
        res, span = serve.replay(srv, trace, progress=lambda what, i: print(
            f"[bench] load {load}: {what} {i}/{nq} ({time.perf_counter() - t_rep:.0f} s)", file=sys.stderr, flush=True))
        srv.stop()
        row["continuous_batching"] = serve.latency_summary(res, span)
        for r, ref in zip(res, serial_out):
            assert [int(x) for x in r["seeds"]] == ref["seeds"] and [int(x) for x in r["T"]] == ref["T"], \
                "outputs differ"
        row["identical_outputs"] = True
        if args.served_dump:
            dump = json.load(open(args.served_dump)) if os.path.exists(args.served_dump) else {}
            dump[str(load)] = {"serial_ms": lat.tolist(), "cb_ms": [r["latency_s"] * 1e3 for r in res]}
            json.dump(dump, open(args.served_dump, "w"))
        print(f"[bench] load {load}: serial {row['serial']} | continuous batching {row['continuous_batching']}",
              file=sys.stderr, flush=True)
        out["levels"].append(row)
    out["value"] = max(r["continuous_batching"]["throughput_qps"] for r in out["levels"])
    out["config"] = {"workload": "served_rmat" + "-".join(map(str, scales)) + "_p0.01+wc_J128|512_K10-100",
                     "queries_per_level": nq, "slots_per_lane": args.served_slots,
                     "lanes_mib": args.served_lanes_mib, "lane_grid_caps": args.served_caps,
                     "lane_graph_mode": args.served_graphs, "quick_ms": args.served_quick_ms}
    print(json.dumps(out), flush=True)


def mc_spread(g, seeds, worlds: int, rng) -> np.ndarray:
    """Independent evaluation of an IC seed set: `worlds` live-edge graphs
    drawn with a standard RNG (every arc live with its own probability), and
    the number of vertices reachable from the seeds in each (BFS from a
    super-source).  No hashing and nothing shared with the method."""
    import numpy as np
    import scipy.sparse as sp
    from scipy.sparse.csgraph import breadth_first_order
    src = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.rowptr))
    out = np.empty(worlds, np.int64)
    s = np.asarray(seeds, np.int64)
    for r in range(worlds):
        live = rng.random(g.m) < g.p
        rows = np.concatenate([src[live], np.full(len(s), g.n)])
        cols = np.concatenate([g.col[live].astype(np.int64), s])
        A = sp.csr_matrix((np.ones(len(rows), np.int8), (rows, cols)), shape=(g.n + 1, g.n + 1))
        out[r] = len(breadth_first_order(A, g.n, directed=True, return_predecessors=False)) - 1
    return out


def quality_main(args):
    """Seed quality under the paper's weight settings (constant 0.005, 0.01,
    0.1; N(0.05, 0.025); U(0, 0.1)) on an RMAT graph: the GPU's seeds and
    sketch estimate T/J, against the spread of the same seeds by independent
    Monte-Carlo (3 runs of `--quality-worlds` worlds, standard RNG).  The 15
    Monte-Carlo runs go to a pool of worker processes forked before anything
    touches the GPU."""
    import multiprocessing

    import numpy as np

    import graphgen
    settings = ("0.005", "0.01", "0.1", "normal", "uniform01")
    pool = multiprocessing.get_context("fork").Pool(min(3 * len(settings), max(1, os.cpu_count() or 1)))

    import torch

    import paper_2410_14047_amd as imx
    torch.cuda.set_device(0)
    base = graphgen.rmat(args.quality_scale, 16, seed=1)
    J, K = 1024, 50
    rows, jobs = [], []
    for scheme in settings:
        g = graphgen.with_p(base, scheme)
        G = imx.Graph.from_graphgen(g)
        t = time.perf_counter()
        S = imx.Sketch(G, J, 1)
        r = S.select(K)
        S.free()
        torch.cuda.synchronize()
        gpu_ms = (time.perf_counter() - t) * 1e3
        G.free()
        jobs += [pool.apply_async(mc_spread, (g, [int(x) for x in r["seeds"]], args.quality_worlds,
                                              np.random.default_rng(100 + i))) for i in range(3)]
        rows.append({"setting": scheme, "sketch_spread": float(r["spread"]), "gpu_ms": gpu_ms})
    for i, row in enumerate(rows):
        runs = [float(jobs[3 * i + k].get().mean()) for k in range(3)]
        mc = float(np.mean(runs))
        row.update({"mc_spread": mc, "mc_run_spreads": runs, "sketch_over_mc": row["sketch_spread"] / mc})
        print(f"[bench] quality {row['setting']}: sketch {row['sketch_spread']:.1f} MC {mc:.1f}", file=sys.stderr,
              flush=True)
    pool.close()
    pool.join()
    out = {"metric": "seed quality: sketch estimate vs independent Monte-Carlo spread of the same seeds",
           "unit": "vertices", "n_gpus": 1, "data": "synthetic", "dtype": "u8",
           "config": {"workload": f"quality_rmat{args.quality_scale}_J{J}_K{K}", "n": base.n, "m": base.m,
                      "worlds_per_run": args.quality_worlds, "runs": 3},
           "settings": rows}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default=DEFAULT, choices=sorted(WORKLOADS) + ["batched64", "served", "quality"])
    ap.add_argument("--quality-scale", type=int, default=16, help="RMAT scale of the quality workload")
    ap.add_argument("--quality-worlds", type=int, default=1000, help="Monte-Carlo worlds per run (quality)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--no-roofline", action="store_true", help="skip the instrumented byte-count pass")
    ap.add_argument("--no-tail", action="store_true",
                    help="run every sweep and cascade level on the full grid (no single-workgroup tail kernels); "
                         "the profile that the roofline's mean launch time is checked against uses it")
    ap.add_argument("--no-batched", action="store_true",
                    help="default workload only: skip the batched-queries comparison in the line")
    ap.add_argument("--no-variants", action="store_true",
                    help="measure only the named workload (not the variants reported beside it)")
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle work in cpu_baseline")
    ap.add_argument("--cpu-threads", type=int, default=min(16, os.cpu_count() or 1),
                    help="host threads of the cpu_baseline oracle run (default: all cores, at most 16)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (calibrates rocprofv3 "
                         "FETCH_SIZE / WRITE_SIZE against a kernel of known traffic)")
    ap.add_argument("--served-scales", default="16,17,18,19,20,21,22,22")
    ap.add_argument("--served-queries", type=int, default=64)
    ap.add_argument("--served-loads", default="0.5,0.8,1.0")
    ap.add_argument("--served-slots", default="16,1", help="queries each lane holds at once")
    ap.add_argument("--served-caps", default="0",
                    help="workgroup cap of every launch of each lane's engine (0: none)")
    ap.add_argument("--served-quick-ms", type=float, default=100.0,
                    help="route (graph, J) classes seen to finish within this many ms to the first lane (0: off)")
    ap.add_argument("--served-dump", default="", help="write every query's latency (serial and batched) here")
    ap.add_argument("--served-graphs", default="0",
                    help="graph mode (captured steps, device-side splits) of each lane's engine")
    ap.add_argument("--served-service-out", default="", help="write the serial pass (service times, outputs) here")
    ap.add_argument("--served-service-in", default="", help="reuse a serial pass written by --served-service-out")
    ap.add_argument("--served-lanes-mib", default="128",
                    help="footprint bounds (MiB) of the serving lanes; larger queries take the last lane")
    ap.add_argument("--liveness-stats", action="store_true",
                    help="print how arcs' live simulations spread over the sorted values (CPU only)")
    ap.add_argument("--gather-calibration", type=int, default=0, metavar="MIB",
                    help="only measure random gathers of 64/128/1024-byte rows from a MIB MiB buffer "
                         "and a streaming copy (the access-rate ceilings of the propagation kernel)")
    ap.add_argument("--pmc-summary", nargs=4, metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV", "COPY_WRITE_CSV"),
                    help="turn rocprofv3 counter_collection.csv files of this workload and of the copy "
                         "calibration into profiles/propagate_<workload>_pmc.json and print it")
    ap.add_argument("--pmc-command", default="", help="the command line recorded in the --pmc-summary output")
    args = ap.parse_args()
    if args.no_tail:
        os.environ["IMX_TAIL"] = "0"
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (the simulation-column "
              f"split across GPUs is not built).", file=sys.stderr)
        sys.exit(2)
    if args.pmc_summary:
        return pmc_summary(args)
    if args.workload == "batched64":
        return batched_main(args)
    if args.workload == "served":
        return served_main(args)
    if args.workload == "quality":
        return quality_main(args)
    if args.liveness_stats:
        return liveness_stats()
    if args.gather_calibration:
        return gather_calibration(args.gather_calibration)
    if args.copy_calibration:
        import torch
        nbytes = args.copy_calibration << 20
        a = torch.ones(nbytes, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": nbytes, "launches": 3}), flush=True)
        return

    import torch

    import graphgen
    import paper_2410_14047_amd as imx

    w = WORKLOADS[args.workload]
    t0 = time.perf_counter()
    g = make_graph(w)
    print(f"[bench] graph {args.workload}: n={g.n} m={g.m} ({time.perf_counter() - t0:.1f} s)",
          file=sys.stderr, flush=True)
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    out = {
        "metric": METRIC,
        "value": None,
        "unit": "register updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
    }
    main_res = measure(imx, g, w, args.workload, args.steps, args.warmup, not args.no_roofline, stream)
    out.update(main_res)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(g, w, args.cpu_budget, args.cpu_threads)
    if not args.no_variants and VARIANTS.get(args.workload):
        out["variants"] = {}
        for name in VARIANTS[args.workload]:
            wv = WORKLOADS[name]
            gv = graphgen.with_p(g, wv["scheme"])  # same topology, another probability scheme
            res = measure(imx, gv, wv, name, max(1, args.steps // 2 + 1), args.warmup, not args.no_roofline, stream)
            out["variants"][name] = {k: res[k] for k in ("value", "unit", "ms_per_step", "config", "k_seed_wall_ms_median",
                                                         "sweeps_per_step", "rebuilds_per_step", "spread",
                                                         "propagate_kernel_ms_per_step", "roofline") if k in res}
            out["variants"][name]["unit"] = "register updates/s"
            out["variants"][name]["steps"] = max(1, args.steps // 2 + 1)
            del gv
    if args.workload == DEFAULT and not args.no_batched:
        # the batched-queries comparison (library default tuning), so the
        # default line carries it too
        b = batched_result(tune=False)
        out["batched"] = {k: b[k] for k in ("value", "unit", "batched_s", "batched_hip_graphs_s",
                                            "one_query_per_launch_s", "speedup", "identical_outputs", "config")}
    print(json.dumps(out), flush=True)


def measure(imx, g, w, workload, steps, warmup, roofline, stream):
    """Load the graph, run `warmup` untimed and `steps` timed build + select
    steps and (optionally) the instrumented pass for the roofline; returns the
    fields of the bench line for this workload."""
    import torch
    torch.cuda.synchronize()
    t_load = time.perf_counter()
    G = imx.Graph.from_graphgen(g, stream=stream)
    torch.cuda.synchronize()
    load_ms = (time.perf_counter() - t_load) * 1e3
    J, K, seed = w["J"], w["K"], w["sseed"]
    step_ms = []
    imx.im_set_profiling(1)  # per-launch kernel times (HIP events) in the timed steps

    def step():
        t = time.perf_counter()
        S = imx.Sketch(G, J, seed, stream=stream)
        r = S.select(K)
        S.free()
        step_ms.append((time.perf_counter() - t) * 1e3)
        return r

    for i in range(warmup):
        r = step()
        print(f"[bench] {workload} warmup {i}: {r['stats']['select_ms'] + r['stats']['build_ms']:.1f} ms",
              file=sys.stderr, flush=True)

    torch.cuda.synchronize()
    step_ms.clear()
    t_start = time.perf_counter()
    results = [step() for _ in range(steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    for r in results[1:]:
        assert list(r["seeds"]) == list(results[0]["seeds"]), "steps disagree"

    sweeps = sum(r["stats"]["total_sweeps"] for r in results)
    launches = sum(r["stats"]["prop_launches"] for r in results)
    kms = sum(r["stats"]["prop_kernel_ms"] for r in results)
    out = {
        "value": J * g.m * sweeps / wall,
        "ms_per_step": wall / steps * 1e3,
        "config": {"workload": workload, "n": g.n, "m": g.m, "J": J, "K": K, "p_scheme": w["scheme"],
                   "graph_seed": w["gseed"], "sketch_seed": seed, "parallelism": "single GPU"},
        "k_seed_wall_ms": wall / steps * 1e3,
        "k_seed_wall_ms_median": float(sorted(step_ms)[len(step_ms) // 2]),
        "graph_load_ms": load_ms,
        "sweeps_per_step": sweeps / steps,
        "rebuilds_per_step": results[0]["stats"]["rebuilds"],
        "spread": results[0]["spread"],
        "propagate_kernel_ms_per_step": kms / steps,
        "propagate_launch_avg_us": kms / launches * 1e3,
    }
    print(f"[bench] {workload}: {out['ms_per_step']:.1f} ms/step, {out['value']:.3e} updates/s",
          file=sys.stderr, flush=True)

    if roofline:
        # The roofline covers the full-grid propagation kernel over every
        # sweep: one timed step with the tail kernels off (every sweep is then
        # a k_propagate_pack launch), and the instrumented step (which never
        # uses them) for the algorithmic bytes of the same launches.
        prev = os.environ.get("IMX_TAIL")
        os.environ["IMX_TAIL"] = "0"
        S = imx.Sketch(G, J, seed, stream=stream)
        r0 = S.select(K)
        S.free()
        imx.im_set_profiling(2)
        S = imx.Sketch(G, J, seed, stream=stream)
        rr = S.select(K)
        S.free()
        imx.im_set_profiling(1)
        if prev is None:
            del os.environ["IMX_TAIL"]
        else:
            os.environ["IMX_TAIL"] = prev
        st = rr["stats"]
        assert list(rr["seeds"]) == list(results[0]["seeds"]), "instrumented run disagrees"
        assert list(r0["seeds"]) == list(results[0]["seeds"]), "run without tail kernels disagrees"
        bpl = st["prop_alg_bytes"] / st["prop_launches"]
        tpl = r0["stats"]["prop_kernel_ms"] / r0["stats"]["prop_launches"] * 1e-3
        achieved = bpl / tpl / 1e9
        traffic = pmc_traffic(workload, bpl)
        out["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                           "kernel": "k_propagate_pack", "alg_bytes_per_launch": bpl,
                           "avg_launch_us": tpl * 1e6,
                           "traffic_over_algorithmic": (traffic / bpl) if traffic else None,
                           "per_launch": {k: st[k] / st["prop_launches"] for k in
                                          ("prop_rows_visited", "prop_rows_changed", "prop_arcs_active",
                                           "prop_sectors", "prop_tasks", "prop_rows_read", "prop_bytes_written",
                                           "prop_arcs_scanned")}}
        print(f"[bench] {workload} roofline: {bpl / 1e6:.1f} MB/launch, {tpl * 1e6:.1f} us/launch, "
              f"{achieved:.0f} GB/s", file=sys.stderr, flush=True)
    G.free()
    return out


if __name__ == "__main__":
    main()

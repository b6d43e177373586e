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
DEFAULT = "rmat20_wc_J512_K50"


def make_graph(w):
    import graphgen
    if w["kind"] == "rmat":
        g = graphgen.rmat(w["scale"], w["ef"], seed=w["gseed"])
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


def cpu_baseline(g, w, budget_s: float):
    """The oracle (single thread, as it stands) running full synchronous sweeps
    over a subset of the J simulation columns of the same graph."""
    import numpy as np
    import oracle
    J, seed = w["J"], w["sseed"]
    t0 = time.perf_counter()
    oracle.sweeps_sample(g, J, seed, np.arange(16, dtype=np.int32), 1)
    per_col_sweep = max((time.perf_counter() - t0) / 16, 1e-4)
    sweeps = 2
    S = int(max(1, min(J, budget_s / per_col_sweep / sweeps)))
    sims = np.linspace(0, J - 1, S).astype(np.int32)
    t0 = time.perf_counter()
    oracle.sweeps_sample(g, J, seed, sims, sweeps)
    dt = time.perf_counter() - t0
    rate = S * g.m * sweeps / dt
    return {"value": rate, "unit": "register updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{sweeps} synchronous sweeps (from fill) over {S} of {J} simulation columns, "
                      f"all {g.m} arcs, single thread; {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default=DEFAULT, choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--no-roofline", action="store_true", help="skip the instrumented byte-count pass")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (calibrates rocprofv3 "
                         "FETCH_SIZE / WRITE_SIZE against a kernel of known traffic)")
    args = ap.parse_args()
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
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (the method's "
              f"multi-GPU split is described in DESIGN.md but not built).", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2410_14047_amd as imx

    w = WORKLOADS[args.workload]
    t0 = time.perf_counter()
    g = make_graph(w)
    print(f"[bench] graph {args.workload}: n={g.n} m={g.m} ({time.perf_counter() - t0:.1f} s)",
          file=sys.stderr, flush=True)
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    G = imx.Graph.from_graphgen(g, stream=stream)
    J, K, seed = w["J"], w["K"], w["sseed"]

    def step():
        S = imx.Sketch(G, J, seed, stream=stream)
        r = S.select(K)
        S.free()
        return r

    for i in range(args.warmup):
        r = step()
        print(f"[bench] warmup {i}: {r['stats']['select_ms'] + r['stats']['build_ms']:.1f} ms", file=sys.stderr,
              flush=True)

    torch.cuda.synchronize()
    t_start = time.perf_counter()
    results = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    for r in results[1:]:
        assert list(r["seeds"]) == list(results[0]["seeds"]), "steps disagree"

    sweeps = sum(r["stats"]["total_sweeps"] for r in results)
    launches = sum(r["stats"]["prop_launches"] for r in results)
    kms = sum(r["stats"]["prop_kernel_ms"] for r in results)
    value = J * g.m * sweeps / wall
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "register updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": g.n, "m": g.m, "J": J, "K": K, "p_scheme": w["scheme"],
                   "graph_seed": w["gseed"], "sketch_seed": seed, "parallelism": "single GPU"},
        "k_seed_wall_ms": wall / args.steps * 1e3,
        "sweeps_per_step": sweeps / args.steps,
        "rebuilds_per_step": results[0]["stats"]["rebuilds"],
        "spread": results[0]["spread"],
        "propagate_kernel_ms_per_step": kms / args.steps,
        "propagate_launch_avg_us": kms / launches * 1e3,
    }

    if not args.no_roofline:
        imx.im_set_profiling(2)
        S = imx.Sketch(G, J, seed, stream=stream)
        rr = S.select(K)
        S.free()
        imx.im_set_profiling(0)
        st = rr["stats"]
        assert list(rr["seeds"]) == list(results[0]["seeds"]), "instrumented run disagrees"
        bpl = st["prop_alg_bytes"] / st["prop_launches"]
        tpl = kms / launches * 1e-3
        achieved = bpl / tpl / 1e9
        traffic = pmc_traffic(args.workload, bpl)
        out["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                           "kernel": "k_propagate", "alg_bytes_per_launch": bpl,
                           "avg_launch_us": tpl * 1e6,
                           "per_launch": {k: st[k] / st["prop_launches"] for k in
                                          ("prop_tasks", "prop_rows_read", "prop_bytes_written",
                                           "prop_arcs_scanned", "prop_arcs_active", "prop_sectors")}}
        print(f"[bench] roofline: {bpl / 1e6:.1f} MB/launch, {tpl * 1e6:.1f} us/launch, {achieved:.0f} GB/s",
              file=sys.stderr, flush=True)

    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(g, w, args.cpu_budget)
        out["cpu_baseline"]["cores"] = 1
    G.free()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

"""Writes batched_sample.json: the oracle's results for a sample of the
batched-queries workload (64 weighted-cascade graphs of uneven size, J = 256,
K = 20, sketch seed = the query's index), so that a GPU test can check the
batched engine's outputs on that workload against the oracle.

Sample: the queries on the eight smallest graphs by arc count, plus the one
on the smallest Barabasi-Albert graph.  Only `graphgen` (the inputs) and
`oracle` are used.

    python tests/golden/make_batched_sample.py     (a few minutes, 8 processes)
"""
import json
import multiprocessing
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import graphgen  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "batched_sample.json")
J, K = 256, 20


def sample():
    specs = graphgen.batched_specs()
    sizes = [(graphgen.batched_graph(sp).m, q) for q, sp in enumerate(specs)]
    picked = [q for _, q in sorted(sizes)[:8]]
    ba = min((m, q) for m, q in sizes if specs[q][0] == "ba")[1]
    if ba not in picked:
        picked.append(ba)
    return sorted(picked)


def run(q):
    import oracle
    spec = graphgen.batched_specs()[q]
    r = oracle.greedy(graphgen.batched_graph(spec), J, q, K, keep_registers=False)
    return {"query": q, "spec": list(spec), "J": J, "seed": q, "K": K,
            "seeds": [int(x) for x in r["seeds"]], "T": [int(x) for x in r["T"]],
            "est_hex": [float(x).hex() for x in r["est"]], "spread_hex": float(r["spread"]).hex(),
            "rebuilds": int(np.count_nonzero(r["sweeps"][1:]))}


def main():
    qs = sample()
    with multiprocessing.get_context("fork").Pool(min(len(qs), os.cpu_count() or 1)) as pool:
        res = pool.map(run, qs, chunksize=1)
    with open(OUT, "w") as f:
        json.dump({"queries": res}, f, indent=1)
    print(f"wrote {OUT}: {len(res)} queries")


if __name__ == "__main__":
    main()

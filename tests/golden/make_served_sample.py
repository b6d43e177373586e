"""Writes served_sample.json: the oracle's results for a sample of the
served-queries workload's request stream, so that a GPU test can check the
serving loop's outputs on that workload against the oracle without running
the (slow) oracle on the GPU host.

Sample: the first eight requests of the 1,000-request stream that fall on the
scale-16 and scale-17 graphs, leaving out those with J = 512 on a
weighted-cascade graph (their oracle runs take hours).  Only `graphgen` (the
inputs) and `oracle` are used.

    python tests/golden/make_served_sample.py     (about 10 minutes, 8 processes)
"""
import json
import multiprocessing
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import graphgen  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "served_sample.json")
STREAM = 1000
COUNT = 8


def sample():
    out = []
    for name, J, seed, K in graphgen.served_requests(STREAM):
        if not name.startswith(("rmat16_", "rmat17_")):
            continue
        if J == 512 and name.endswith("_wc"):
            continue
        out.append((name, J, seed, K))
        if len(out) == COUNT:
            break
    return out


def run(q):
    import oracle
    name, J, seed, K = q
    r = oracle.greedy(graphgen.served_graph(name), J, seed, K, keep_registers=False)
    return {"graph": name, "J": J, "seed": seed, "K": K,
            "seeds": [int(x) for x in r["seeds"]], "T": [int(x) for x in r["T"]],
            "est_hex": [float(x).hex() for x in r["est"]], "spread_hex": float(r["spread"]).hex(),
            "rebuilds": int(np.count_nonzero(r["sweeps"][1:]))}


def main():
    qs = sample()
    with multiprocessing.get_context("fork").Pool(min(len(qs), os.cpu_count() or 1)) as pool:
        res = pool.map(run, qs, chunksize=1)
    with open(OUT, "w") as f:
        json.dump({"stream": STREAM, "scales": list(graphgen.SERVED_SCALES), "queries": res}, f, indent=1)
    print(f"wrote {OUT}: {len(res)} queries")


if __name__ == "__main__":
    main()

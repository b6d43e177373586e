"""The no-allocation entry point (im_select_seeds_noalloc) against the
allocating one (im_sketch_build + im_select_seeds) and the oracle: seeds,
estimates, spread and final registers identical, on two calls in a row, the
second on a smaller input (the fixed scratch array keeps the first call's
contents); a query above the scratch maximum is rejected before any work."""
import sys

import numpy as np
import pytest

import graphgen

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _reference(imx, G, J, seed, K):
    S = imx.Sketch(G, J, seed)
    r = S.select(K)
    r["M"] = S.registers()
    S.free()
    return r


def test_noalloc_matches_allocating_entry_point(imx, orc):
    import torch
    cases = [
        ("rmat12_wc_J512_K8", graphgen.with_p(graphgen.rmat(12, 16, seed=3), "wc"), 512, 11, 8),
        ("er1k_p0.1_J64_K10", graphgen.with_p(graphgen.erdos_renyi(1000, 5000, 1), "0.1"), 64, 1, 10),
    ]
    for name, g, J, seed, K in cases:  # second call: smaller graph, J and registers
        _say(f"[noalloc] {name}: n={g.n} m={g.m} J={J} K={K}")
        G = imx.Graph.from_graphgen(g)
        ref = _reference(imx, G, J, seed, K)
        regs = torch.full((g.n * J,), 0xAB, dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        r = imx.im_select_seeds_noalloc(G.handle, J, seed, K, regs.data_ptr())
        M = regs.cpu().numpy().reshape(g.n, J)
        assert list(r["seeds"]) == list(ref["seeds"]), name
        assert r["est"].tobytes() == ref["est"].tobytes(), name
        assert r["spread"] == ref["spread"], name
        assert np.array_equal(M, ref["M"]), name
        orc_r = orc.greedy(g, J, seed, K)
        assert list(r["seeds"]) == list(orc_r["seeds"]), name
        assert r["est"].tobytes() == orc_r["est"].tobytes(), name
        assert np.array_equal(M, orc_r["M_final"]), name
        del regs
        G.free()


def test_noalloc_rejects_query_above_scratch_maximum(imx):
    import torch
    n = 4 << 20  # about 24 bytes of working memory per vertex: above 64 MiB
    g = graphgen.Graph(n=n, rowptr=np.zeros(n + 1, np.int64), col=np.zeros(0, np.int32), p=np.zeros(0, np.float32))
    G = imx.Graph.from_graphgen(g)
    dummy = torch.zeros(1, dtype=torch.uint8, device="cuda")
    with pytest.raises(imx.IMError) as ei:
        imx.im_select_seeds_noalloc(G.handle, 64, 1, 1, dummy.data_ptr())
    assert ei.value.status == 1 and "scratch" in str(ei.value)
    G.free()

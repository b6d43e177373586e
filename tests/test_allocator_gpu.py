"""Device memory from PyTorch's caching allocator (im_set_allocator): results
are unchanged and the library's buffers are PyTorch's."""
import pytest

import graphgen

pytestmark = pytest.mark.gpu


def test_torch_allocator_owns_memory_and_keeps_results(imx):
    import torch
    g = graphgen.with_p(graphgen.rmat(11, 16, seed=5), "wc")
    G0 = imx.Graph.from_graphgen(g)
    S0 = imx.Sketch(G0, 256, 3)
    ref = S0.select(6)
    regs_ref = S0.registers()
    S0.free()
    G0.free()
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    imx.use_torch_allocator()
    try:
        G = imx.Graph.from_graphgen(g)
        S = imx.Sketch(G, 256, 3)
        held = torch.cuda.memory_allocated() - base
        assert held >= g.n * 256  # at least the registers come from PyTorch
        r = S.select(6)
        assert list(r["seeds"]) == list(ref["seeds"]) and list(r["T"]) == list(ref["T"])
        assert (S.registers() == regs_ref).all()
        S.free()
        G.free()
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == base  # everything returned
    finally:
        imx.use_torch_allocator(False)

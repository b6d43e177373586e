"""MI355X-native sketch-based influence maximisation (DiFuseR method).

The compute path is libimx.so (HIP kernels for gfx950, C ABI in include/im.h);
this package holds its build script and a thin ctypes binding.
"""
from .binding import (  # noqa: F401
    EXPORTS, Engine, Graph, IMError, Sketch, im_query_footprint, im_select_seeds_batch, im_graph_free, im_graph_load, im_select_seeds, im_sketch_build,
    im_sketch_estimates, im_sketch_free, im_sketch_register_rows, im_sketch_registers, im_sketch_sim_values, im_sketch_stats, im_set_profiling, lib,
    im_set_allocator, use_torch_allocator, im_select_seeds_noalloc,
)

__version__ = "0.1.0"

"""C-ABI checks that need no GPU: the library loads, exports every declared
symbol, and rejects malformed input with IM_EINVAL before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "im.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(im_[a-z_0-9]+)\s*\(", text)))


def test_header_and_binding_agree(imx):
    assert _declared_symbols() == sorted(imx.EXPORTS)


def test_library_exports_every_declared_symbol(imx):
    L = ctypes.CDLL(imx.binding.LIB_PATH)
    for name in _declared_symbols():
        assert hasattr(L, name), name


def test_version(imx):
    a, b = ctypes.c_int32(), ctypes.c_int32()
    assert imx.lib().im_version(ctypes.byref(a), ctypes.byref(b)) == 0
    assert (a.value, b.value) >= (0, 1)


def _load(imx, n, rowptr, col, p):
    return imx.im_graph_load(n, np.asarray(rowptr, np.int64), np.asarray(col, np.int32), np.asarray(p, np.float32))


@pytest.mark.parametrize("n,rowptr,col,p,msg", [
    (3, [1, 1, 2, 2], [1, 2], [0.1, 0.1], "rowptr[0]"),
    (3, [0, 2, 1, 2], [1, 2], [0.1, 0.1], "decreases"),
    (3, [0, 1, 1, 1], [1, 2], [0.1, 0.1], "rowptr[n]"),
    (3, [0, 1, 2, 2], [1, 3], [0.1, 0.1], "out of range"),
    (3, [0, 1, 2, 2], [1, -1], [0.1, 0.1], "out of range"),
    (3, [0, 2, 2, 2], [2, 1], [0.1, 0.1], "strictly increasing"),
    (3, [0, 2, 2, 2], [1, 1], [0.1, 0.1], "strictly increasing"),
    (3, [0, 1, 2, 2], [1, 2], [0.1, float("nan")], "p outside"),
    (3, [0, 1, 2, 2], [1, 2], [1.5, 0.1], "p outside"),
    (3, [0, 1, 2, 2], [1, 2], [0.1, -0.01], "p outside"),
])
def test_graph_load_rejects_malformed_csr(imx, n, rowptr, col, p, msg):
    with pytest.raises(imx.IMError) as ei:
        _load(imx, n, rowptr, col, p)
    assert ei.value.status == 1 and msg in str(ei.value)


def test_graph_load_rejects_empty_vertex_set(imx):
    out = ctypes.c_void_p()
    assert imx.lib().im_graph_load(0, 0, None, None, None, None, ctypes.byref(out)) == 1
    assert out.value is None


def test_null_handles_are_rejected(imx):
    L = imx.lib()
    out = ctypes.c_void_p()
    assert L.im_sketch_build(None, 64, 1, None, ctypes.byref(out)) == 1
    assert L.im_select_seeds(None, 1, None, None, None, None, None) == 1
    assert L.im_sketch_registers(None, None) == 1
    assert L.im_graph_info(None, None, None) == 1
    L.im_graph_free(None)
    L.im_sketch_free(None)


def test_no_silent_cpu_fallback(imx):
    """Without a GPU the library fails loudly instead of computing on the host."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(imx.IMError) as ei:
        _load(imx, 3, [0, 1, 2, 2], [1, 2], [0.5, 0.5])
    assert ei.value.status == 3


def test_footprint_of_null_graph_is_zero(imx):
    assert imx.lib().im_query_footprint(None, 64, 1) == 0


def test_set_allocator_arguments(imx):
    import ctypes
    from paper_2410_14047_amd import binding
    L = imx.lib()
    null_a, null_f = binding._ALLOC_FN(), binding._FREE_FN()
    hook_a = binding._ALLOC_FN(lambda n, c: None)
    hook_f = binding._FREE_FN(lambda p, c: None)
    assert L.im_set_allocator(hook_a, null_f, None) == 1  # IM_EINVAL: one hook only
    assert L.im_set_allocator(null_a, hook_f, None) == 1
    assert L.im_set_allocator(null_a, null_f, None) == 0  # back to hipMalloc
    with pytest.raises(ValueError):
        imx.im_set_allocator(lambda n: 0, None)
    imx.im_set_allocator()  # no-op reset


def test_profiling_levels(imx):
    L = imx.lib()
    for level in (1, 2, 0):
        assert L.im_set_profiling(level) == 0
    assert L.im_set_profiling(3) == 1  # IM_EINVAL
    assert L.im_set_profiling(-1) == 1


def test_allocator_hooks_outlive_reinstallation(imx):
    """A buffer is returned to the hooks that allocated it, even after other
    hooks were installed or the default restored; the ctypes thunks of every
    installed pair must therefore stay valid for the life of the process."""
    import gc

    from paper_2410_14047_amd import binding
    freed = []
    binding.im_set_allocator(lambda n: 0, lambda p: freed.append(p))
    first = binding._hooks_installed[-1]
    binding.im_set_allocator(lambda n: 0, lambda p: None)
    binding.im_set_allocator()  # back to hipMalloc / hipFree
    gc.collect()
    assert any(h is first for h in binding._hooks_installed)
    # the first pair's free thunk, called through its C function pointer as the
    # library would when a block it allocated is released, still reaches Python
    fptr = ctypes.cast(first[1], ctypes.c_void_p).value
    ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)(fptr)(ctypes.c_void_p(0x1234), None)
    assert freed == [0x1234]


def test_plain_c_program_compiles_links_and_runs(imx, tmp_path):
    """The header is plain C (C99, pedantic) and a C program links against
    libimx.so and calls it: version, and a malformed graph rejected with
    IM_EINVAL and a message (no device needed)."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    src = tmp_path / "use_im.c"
    src.write_text(r'''
#include <stdio.h>
#include "im.h"
int main(void)
{
    int32_t major = 0, minor = 0;
    if (im_version(&major, &minor) != IM_OK || (major == 0 && minor < 1)) return 1;
    const int64_t rowptr[3] = {0, 1, 3};          /* rowptr[n] != m */
    const int32_t col[2] = {1, 0};
    const float p[2] = {0.5f, 0.5f};
    im_graph* g = NULL;
    if (im_graph_load(2, 2, rowptr, col, p, NULL, &g) != IM_EINVAL || g != NULL) return 2;
    const char* msg = im_last_error();
    if (!msg || !msg[0]) return 3;
    printf("%d.%d %s\n", major, minor, msg);
    return 0;
}
''')
    lib_dir = os.path.dirname(imx.binding.LIB_PATH)
    exe = tmp_path / "use_im"
    subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I",
                           os.path.join(ROOT, "include"), str(src), "-L", lib_dir, "-limx",
                           f"-Wl,-rpath,{lib_dir}", "-o", str(exe)])
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, (out.returncode, out.stdout, out.stderr)

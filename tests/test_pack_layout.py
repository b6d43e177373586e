"""LDS layout of the packed propagation kernel (csrc/pack_layout.h), checked on
the host for every configuration the launch code can form: maxJ a multiple of
64 in [64, 4096], pack sizes 1, 2 and 4 KiB, with and without the instrumented
sector masks, every wave of the workgroup.  The header is compiled with the
host C++ compiler; the offsets it produces are re-checked here:
  - each wave's rows and dirty bytes start on 16 bytes (uint4 LDS accesses);
  - the 64-bit sector masks start on 8 bytes (64-bit LDS atomics; a
    misaligned one faults);
  - the pack counter word lies inside the table area, after X and the bucket
    table;
  - a workgroup fits in one CU's 160 KiB of LDS."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2410_14047_amd", "csrc")

PROG = r"""
#include <cstdio>
#include "pack_layout.h"
using namespace imx;
int main() {
    std::printf("ok %d\n", pack_layouts_ok() ? 1 : 0);
    for (int J = 64; J <= 4096; J += 64)
        for (int pb = 1024; pb <= 4096; pb *= 2)
            for (int s = 0; s < 2; ++s)
                for (int w = 0; w < kPackWaves; ++w)
                    std::printf("%d %d %d %d %d %d %d %d %d\n", J, pb, s, w, pack_table_words(J),
                                pack_wave_base(J, pb, s, w), pack_row_words(J, pb), pack_esec_word(J, pb, s, w),
                                pack_lds_words(J, pb, s));
    return 0;
}
"""


def test_pack_layout_alignment(tmp_path):
    src = tmp_path / "layout.cpp"
    exe = tmp_path / "layout"
    src.write_text(PROG)
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-I", CSRC, "-o", str(exe), str(src)])
    out = subprocess.check_output([str(exe)], text=True).splitlines()
    assert out[0] == "ok 1"
    rows = [tuple(int(x) for x in line.split()) for line in out[1:]]
    assert len(rows) == 64 * 3 * 2 * 8
    for J, pb, s, w, table, base, rw, esec, total in rows:
        assert table >= J + 1024 + 2, (J, "no counter word after the bucket table")
        assert (4 * base) % 16 == 0, (J, pb, s, w, "rows not 16-byte aligned")
        assert (4 * (base + rw)) % 16 == 0, (J, pb, s, w, "dirty bytes not 16-byte aligned")
        assert (4 * esec) % 8 == 0, (J, pb, s, w, "sector masks not 8-byte aligned")
        assert rw * 4 >= max(J, pb), (J, pb, "rows area smaller than a pack")
        assert 4 * total <= 160 * 1024, (J, pb, s, "workgroup LDS above 160 KiB")

// LDS layout of the packed propagation kernel (k_propagate_pack), as plain
// constexpr arithmetic with no HIP dependency, so that the kernel, its launch
// code and a host-only check share one definition.
//
// One workgroup of kPackWaves waves holds, in 32-bit words:
//   [0, table_words(maxJ))        the sorted simulation values X (J words), the
//                                 bucket table (kBuckets + 1 words), a padding
//                                 word (the workgroup's pack counter), rounded
//                                 up to whole 16-byte chunks;
//   then per wave w, wave_words(maxJ, pb, stats) words at
//   table_words + w * wave_words:
//     rows      row_words      the pack's register rows (16-byte chunks)
//     dirty     dirty_words    one byte per row word (cleared in 16-byte chunks)
//     arcs      kPackArcWords  per-arc operands of one 64-arc chunk
//     tasks     kPackTaskWords per-task records of the pack
//     esec      2 x 64         64-bit sector masks (instrumented variant only;
//                              64-bit LDS atomics need 8-byte alignment)
//     list      kPackBufCap    staging of the changed in-task list
#pragma once

namespace imx {

constexpr int kBuckets = 1024;    // bucket table over the top bits of the 31-bit X values
constexpr int kBucketShift = 21;  // X >> 21 selects the bucket
// Words of the bucket table area (kBuckets + 1 entries and at least one
// padding word), padded to 16 bytes so that the areas after it keep 8- and
// 16-byte alignment.
constexpr int kTableWords = ((kBuckets + 1 + 1 + 3) / 4) * 4;

constexpr int kPackMax = 16;    // tasks per pack, at most
constexpr int kPackWaves = 8;   // waves per workgroup of the packed kernel
constexpr int kPackWG = 64 * kPackWaves;
constexpr int kPackArcWords = 6 * 64;              // ev, eh, eW, edl, est, ek
constexpr int kPackTaskWords = 10 * kPackMax + 16;  // u, e0 lo/hi, prefix (+1), split, touched, active, changed, in0, inc
constexpr int kPackBufCap = 128;                    // staging entries per wave for the changed in-task list
constexpr int kLdsBytesPerCU = 160 * 1024;          // gfx950

constexpr int pack_row_words(int maxJ, int pb) { return (maxJ > pb) ? maxJ / 4 : pb / 4; }
constexpr int pack_dirty_words(int maxJ, int pb) { return pack_row_words(maxJ, pb) / 4; }  // a byte per row word
constexpr int pack_wave_words(int maxJ, int pb, bool stats)
{
    return pack_row_words(maxJ, pb) + pack_dirty_words(maxJ, pb) + kPackArcWords + kPackTaskWords + (stats ? 2 * 64 : 0) +
           kPackBufCap;
}
constexpr int pack_table_words(int maxJ) { return ((maxJ + kTableWords) + 3) & ~3; }
constexpr int pack_wave_base(int maxJ, int pb, bool stats, int wave)
{
    return pack_table_words(maxJ) + wave * pack_wave_words(maxJ, pb, stats);
}
constexpr int pack_esec_word(int maxJ, int pb, bool stats, int wave)
{
    return pack_wave_base(maxJ, pb, stats, wave) + pack_row_words(maxJ, pb) + pack_dirty_words(maxJ, pb) + kPackArcWords +
           kPackTaskWords;
}
constexpr int pack_lds_words(int maxJ, int pb, bool stats)
{
    return pack_table_words(maxJ) + kPackWaves * pack_wave_words(maxJ, pb, stats);
}

// The alignments the kernel relies on, for one configuration: rows and dirty
// bytes on 16 bytes (uint4 accesses), the sector masks on 8 bytes (64-bit LDS
// atomics), the counter word inside the table area, and the workgroup within
// one CU's LDS.  (The dynamic LDS base itself is 16-byte aligned.)
constexpr bool pack_layout_ok(int maxJ, int pb, bool stats)
{
    if (maxJ + kBuckets + 1 >= pack_table_words(maxJ)) return false;  // no room for the counter word
    for (int w = 0; w < kPackWaves; ++w) {
        const int base = pack_wave_base(maxJ, pb, stats, w);
        if (base % 4 != 0) return false;
        if ((base + pack_row_words(maxJ, pb)) % 4 != 0) return false;
        if (pack_esec_word(maxJ, pb, stats, w) % 2 != 0) return false;
    }
    return 4 * pack_lds_words(maxJ, pb, stats) <= kLdsBytesPerCU;
}

// Every configuration the launch code can form: maxJ a multiple of 64 in
// [64, 4096], pack sizes of 1, 2 and 4 KiB, with and without the sector masks.
constexpr bool pack_layouts_ok()
{
    for (int maxJ = 64; maxJ <= 4096; maxJ += 64)
        for (int pb = 1024; pb <= 4096; pb *= 2)
            for (int s = 0; s < 2; ++s)
                if (!pack_layout_ok(maxJ, pb, s != 0)) return false;
    return true;
}

}  // namespace imx

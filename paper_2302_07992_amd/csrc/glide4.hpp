// The recovery glide (Sec. III-A decoding) on four pixels per word.
//
// A pixel labelled 0 takes the replaceable bits of the nearest pixel to its
// left labelled 1.  Inside one 4-pixel word with label pattern m (bit j:
// pixel j labelled 1), pixel j therefore copies pixel h, the highest i <= j
// with bit i of m set, or, when there is none, the value carried in from the
// left.  With the word as operand a of v_perm_b32 and the previous word's
// result (whose byte 3 is that carried value) as operand b, the copy is one
// permute with selector byte j = 4 + h, or 3 for the carry:
//   fill = vperm(word, previous fill, fill_sel[m]),
// and the replaceable bits of the output come from fill, the rest from word.
#pragma once
#include <cstdint>

namespace rdhei {
namespace glide4 {

struct Tables {
    uint32_t fill_sel[16];
};

constexpr Tables make_tables() {
    Tables t{};
    for (uint32_t m = 0; m < 16; ++m) {
        uint32_t sel = 0, cur = 3;
        for (uint32_t j = 0; j < 4; ++j) {
            if ((m >> j) & 1u) cur = 4 + j;
            sel |= cur << (8 * j);
        }
        t.fill_sel[m] = sel;
    }
    return t;
}

constexpr Tables kTables = make_tables();
constexpr int kWords = 16;

}  // namespace glide4
}  // namespace rdhei

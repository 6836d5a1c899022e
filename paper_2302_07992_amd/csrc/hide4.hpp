// Four pixels per word for data hiding and extraction.
//
// A redundant pixel holds `rep` payload bits in its replaceable bits (top bit
// first), and payload bits fill redundant pixels in raster order, so the
// redundant pixels of one 4-pixel word take one contiguous run of the
// payload: `rep` bits per redundant pixel, in pixel order.  With m the word's
// redundancy pattern (bit j: pixel j is redundant), one byte permute moves the
// per-pixel fields between their pixels and a packed order:
//   compact[m]: byte 3 - i of the result = field of the i-th redundant pixel
//               (bytes of missing pixels are zero);
//   expand[m]:  the inverse, byte j = byte 3 - i when pixel j is the i-th
//               redundant pixel, else zero;
//   bytes[m]:   0xFF in the bytes of the redundant pixels.
// In packed order the fields are f0..f3 from byte 3 down to byte 0, so the run
// is f0 f1 f2 f3 read from the top: (f0 << 3 rep) | (f1 << 2 rep) | ...
#pragma once
#include <cstdint>

namespace rdhei {
namespace hide4 {

struct Tables {
    uint32_t compact[16];
    uint32_t expand[16];
    uint32_t bytes[16];
};

constexpr Tables make_tables() {
    Tables t{};
    for (uint32_t m = 0; m < 16; ++m) {
        uint32_t c = 0x0C0C0C0Cu, e = 0, b = 0, i = 0;
        for (uint32_t j = 0; j < 4; ++j) {
            uint32_t esel = 0x0Cu;
            if ((m >> j) & 1u) {
                const uint32_t slot = 3u - i;                         // packed byte of the i-th field
                c = (c & ~(0xFFu << (8 * slot))) | (j << (8 * slot));
                esel = slot;
                b |= 0xFFu << (8 * j);
                ++i;
            }
            e |= esel << (8 * j);
        }
        t.compact[m] = c;
        t.expand[m] = e;
        t.bytes[m] = b;
    }
    return t;
}

constexpr Tables kTables = make_tables();
constexpr int kWords = (int)(sizeof(Tables) / sizeof(uint32_t));   // 48

}  // namespace hide4
}  // namespace rdhei

// Host check of the glide fill selectors: for every label pattern, carried
// value and word, the one-permute fill must give each pixel the value of the
// nearest pixel labelled 1 at or to its left, or the carried value.
#include <cstdio>
#include <cstdint>
#include "../../paper_2302_07992_amd/csrc/glide4.hpp"

using namespace rdhei::glide4;

static uint32_t vperm(uint32_t a, uint32_t b, uint32_t sel) {
    const uint64_t v = ((uint64_t)a << 32) | b;
    uint32_t out = 0;
    for (int i = 0; i < 4; ++i) {
        const uint32_t s = (sel >> (8 * i)) & 0xFFu;
        if (s >= 8) return 0xDEADBEEFu;   // only byte selectors are generated
        out |= (uint32_t)((v >> (8 * s)) & 0xFFu) << (8 * i);
    }
    return out;
}

int main() {
    int bad = 0, cases = 0;
    uint32_t x = 0x9E3779B9u;
    for (uint32_t m = 0; m < 16; ++m)
        for (int trial = 0; trial < 64; ++trial) {
            x = x * 1664525u + 1013904223u;
            const uint32_t word = x;
            x = x * 1664525u + 1013904223u;
            const uint32_t prev = x;
            const uint32_t fill = vperm(word, prev, kTables.fill_sel[m]);
            uint32_t carry = prev >> 24;
            for (int j = 0; j < 4; ++j) {
                if ((m >> j) & 1u) carry = (word >> (8 * j)) & 0xFFu;
                if (((fill >> (8 * j)) & 0xFFu) != carry) ++bad;
            }
            ++cases;
        }
    printf("cases %d mismatches %d\n", cases, bad);
    return bad ? 1 : 0;
}

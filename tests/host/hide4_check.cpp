// Host check of the 4-pixel hiding tables: packing the fields of a word's
// redundant pixels through compact[] and unpacking a payload run through
// expand[] (with a CPU model of the byte permute) must agree with placing
// rep bits per redundant pixel one pixel at a time, for every pattern and
// every rep in 1..7, with the fields at the top of the byte (EMR) or just
// below bit 7 (LMR).
#include <cstdio>
#include <cstdint>
#include <random>
#include "../../paper_2302_07992_amd/csrc/hide4.hpp"

using namespace rdhei::hide4;

static uint32_t vperm(uint32_t a, uint32_t b, uint32_t sel) {
    const uint64_t v = ((uint64_t)a << 32) | b;
    uint32_t out = 0;
    for (int i = 0; i < 4; ++i) {
        const uint32_t s = (sel >> (8 * i)) & 0xFFu;
        uint32_t byte = 0;
        if (s < 8) byte = (uint32_t)(v >> (8 * s)) & 0xFFu;
        else if (s != 12) return 0xDEADBEEFu;
        out |= byte << (8 * i);
    }
    return out;
}

int main() {
    std::mt19937 rng(7);
    int bad = 0, cases = 0;
    for (uint32_t rep = 1; rep <= 7; ++rep)
      for (uint32_t shift = 7 - rep; shift <= 8 - rep; ++shift) {   // LMR (below bit 7) and EMR (top bits)
        const uint32_t low = (1u << rep) - 1u;
        for (uint32_t m = 0; m < 16; ++m)
            for (int trial = 0; trial < 50; ++trial) {
                const uint32_t x = rng(), run = rng();
                const uint32_t k = __builtin_popcount(m);
                // reference: pixel j (redundant, i-th) takes run bits [i rep, (i+1) rep) at its top
                uint32_t ref_embed = x, ref_run = 0, i = 0;
                for (uint32_t j = 0; j < 4; ++j) {
                    if (!((m >> j) & 1u)) continue;
                    const uint32_t f = (run >> (32 - (i + 1) * rep)) & low;
                    ref_embed = (ref_embed & ~(low << (8 * j + shift))) | (f << (8 * j + shift));
                    const uint32_t g = (x >> (8 * j + shift)) & low;
                    ref_run |= g << (32 - (i + 1) * rep);
                    ++i;
                }
                // packed: extraction
                const uint32_t fields = (x >> shift) & (low * 0x01010101u);
                const uint32_t c = vperm(0, fields, kTables.compact[m]);
                const uint32_t s = (((c >> 24) << (3 * rep)) | (((c >> 16) & 0xFFu) << (2 * rep)) |
                                    (((c >> 8) & 0xFFu) << rep) | (c & 0xFFu)) << (32 - 4 * rep);
                // packed: embedding
                const uint32_t F01 = run >> (32 - 2 * rep), F23 = (run >> (32 - 4 * rep)) & ((1u << (2 * rep)) - 1u);
                const uint32_t t = (F01 << 16) | F23;
                const uint32_t L = low * 0x00010001u;
                const uint32_t cp = (t & L) | (((t >> rep) & L) << 8);
                const uint32_t e = vperm(0, cp, kTables.expand[m]) << shift;
                const uint32_t K = kTables.bytes[m] & ((low << shift) * 0x01010101u);
                const uint32_t emb = (x & ~K) | (e & K);
                const uint32_t used = k ? ~0u << (32 - k * rep) : 0u;
                if (emb != ref_embed) ++bad;
                if ((s & used) != ref_run || (s & ~used) != 0) ++bad;
                ++cases;
            }
    }
    printf("cases %d mismatches %d\n", cases, bad);
    return bad ? 1 : 0;
}

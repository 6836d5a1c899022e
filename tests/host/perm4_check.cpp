// Host check of the 4x4 block permute selectors: a CPU model of v_perm_b32
// applied with the tables must move every pixel where the bit-pair turn rule
// sends it, for every R1 and every set of four level-1 codes, and the inverse
// sequence must restore the block, both as two steps and as the composed
// one-step selectors.
#include <cstdio>
#include <cstdint>
#include "../../paper_2302_07992_amd/csrc/perm4.hpp"

using namespace rdhei::perm4;

static uint32_t vperm(uint32_t a, uint32_t b, uint32_t sel) {
    const uint64_t v = ((uint64_t)a << 32) | b;
    uint32_t out = 0;
    for (int i = 0; i < 4; ++i) {
        const uint32_t s = (sel >> (8 * i)) & 0xFFu;
        uint32_t byte = 0;
        if (s < 8) byte = (uint32_t)(v >> (8 * s)) & 0xFFu;
        else if (s == 12) byte = 0;
        else return 0xDEADBEEFu;   // other selector values are never generated
        out |= byte << (8 * i);
    }
    return out;
}

static void forward(const uint32_t w[4], uint32_t R1, const uint32_t c[4], uint32_t out[4]) {
    const Tables &T = kTables;
    uint32_t t[4];
    for (int h = 0; h < 2; ++h) {
        const uint32_t k = c[2 * h] + 4 * c[2 * h + 1];
        t[2 * h] = vperm(w[2 * h + 1], w[2 * h], T.sub[k][0]);
        t[2 * h + 1] = vperm(w[2 * h + 1], w[2 * h], T.sub[k][1]);
    }
    for (int I = 0; I < 4; ++I)
        out[I] = vperm(t[1], t[0], T.whole[R1][2 * I]) | vperm(t[3], t[2], T.whole[R1][2 * I + 1]);
}

static void inverse(const uint32_t w[4], uint32_t R1, const uint32_t c[4], uint32_t out[4]) {
    const Tables &T = kTables;
    uint32_t t[4];
    const uint32_t r = (4 - R1) & 3u;
    for (int I = 0; I < 4; ++I)
        t[I] = vperm(w[1], w[0], T.whole[r][2 * I]) | vperm(w[3], w[2], T.whole[r][2 * I + 1]);
    for (int h = 0; h < 2; ++h) {
        const uint32_t k = c[2 * h] + 4 * c[2 * h + 1];
        out[2 * h] = vperm(t[2 * h + 1], t[2 * h], T.sub_inv[k][0]);
        out[2 * h + 1] = vperm(t[2 * h + 1], t[2 * h], T.sub_inv[k][1]);
    }
}

int main() {
    int bad = 0, cases = 0;
    uint32_t w[4];
    for (int i = 0; i < 4; ++i) w[i] = 0x03020100u + 0x04040404u * (uint32_t)i + 0x10101010u;
    for (uint32_t R1 = 0; R1 < 4; ++R1)
        for (uint32_t k = 0; k < 256; ++k) {
            const uint32_t c[4] = {k & 3u, (k >> 2) & 3u, (k >> 4) & 3u, (k >> 6) & 3u};
            uint32_t out[4], back[4];
            forward(w, R1, c, out);
            // brute force: pixel (i, j) goes to (I, J) by the bit-pair rule
            for (uint32_t i = 0; i < 4; ++i)
                for (uint32_t j = 0; j < 4; ++j) {
                    uint32_t Y1, X1, Y0, X0;
                    turn1(R1, i >> 1, j >> 1, Y1, X1);
                    turn1(R1 + c[2 * (i >> 1) + (j >> 1)], i & 1u, j & 1u, Y0, X0);
                    const uint32_t I = 2 * Y1 + Y0, J = 2 * X1 + X0;
                    const uint32_t got = (out[I] >> (8 * J)) & 0xFFu;
                    const uint32_t want = (w[i] >> (8 * j)) & 0xFFu;
                    if (got != want) ++bad;
                }
            inverse(out, R1, c, back);
            for (int i = 0; i < 4; ++i)
                if (back[i] != w[i]) ++bad;
            for (int h = 0; h < 2; ++h) {
                const uint32_t kk = c[2 * h] + 4 * c[2 * h + 1];
                for (int Y = 0; Y < 2; ++Y) {
                    const uint32_t cs = kInvTables.inv[R1][h][kk][2 * Y], ds = kInvTables.inv[R1][h][kk][2 * Y + 1];
                    for (int J = 0; J < 4; ++J) {   // exactly one of the two selectors picks each byte
                        const bool cz = ((cs >> (8 * J)) & 0xFFu) == 0x0Cu, dz = ((ds >> (8 * J)) & 0xFFu) == 0x0Cu;
                        if (cz == dz) ++bad;
                    }
                    const uint32_t row = vperm(out[1], out[0], cs) | vperm(out[3], out[2], ds);
                    if (row != w[2 * h + Y]) ++bad;
                }
            }
            ++cases;
        }
    printf("cases %d mismatches %d\n", cases, bad);
    return bad ? 1 : 0;
}

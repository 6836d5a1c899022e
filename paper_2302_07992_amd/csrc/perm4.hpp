// Quarter turns of a 4x4 pixel block held in four row words (byte j of word i
// is pixel (row i, column j)), done with byte permutes (v_perm_b32).
//
// The composed block rotation (Sec. III-A) turns the coordinate bit pair 1
// of a pixel inside its 4x4 block by R1 (the codes of the levels >= 2 that
// contain it, plus the turns of everything above) and bit pair 0 by
// R1 + c, with c the level-1 code of its 2x2 sub-block.  That is the same as
//   1. turning each 2x2 sub-block in place by its own level-1 code, then
//   2. turning the whole 4x4 block by R1,
// since quarter turns of a bit pair add.  Step 1 is one permute per row of a
// row pair (selectors `sub`), step 2 two permutes and an OR per output row
// (selectors `whole`, one from rows 0-1 and one from rows 2-3).  The inverse
// applies step 2 with -R1, then step 1 with the negated codes.
//
// Selector bytes follow v_perm_b32 with operands (a, b): 0..3 pick bytes of
// b, 4..7 bytes of a, 0x0C gives zero.  The tables are generated at compile
// time from the bit-pair turn rule; a host test checks them against a
// brute-force rotation.
#pragma once
#include <cstdint>

namespace rdhei {
namespace perm4 {

// Quarter turns of one bit pair: r = 0 (y, x); 1 (!x, y); 2 (!y, !x); 3 (x, !y).
constexpr void turn1(uint32_t r, uint32_t y, uint32_t x, uint32_t &oy, uint32_t &ox) {
    r &= 3u;
    oy = r == 0 ? y : r == 1 ? (x ^ 1u) : r == 2 ? (y ^ 1u) : x;
    ox = r == 0 ? x : r == 1 ? y : r == 2 ? (x ^ 1u) : (y ^ 1u);
}

struct Tables {
    // sub[cl + 4 cr][Y]: row Y (0/1) of a row pair after turning its left
    // sub-block by cl and its right one by cr; operands (upper row, lower row)
    uint32_t sub[16][2];
    // whole[r][2 I + h]: row I of the block turned by r, from rows 2h, 2h+1
    uint32_t whole[4][8];
    // sub_inv[k] = sub[k with both codes negated]: undoes sub[k]
    uint32_t sub_inv[16][2];
};

constexpr Tables make_tables() {
    Tables t{};
    for (uint32_t cl = 0; cl < 4; ++cl)
        for (uint32_t cr = 0; cr < 4; ++cr)
            for (uint32_t Y = 0; Y < 2; ++Y) {
                uint32_t sel = 0;
                for (uint32_t J = 0; J < 4; ++J) {
                    const uint32_t x1 = J >> 1, X = J & 1u, c = x1 ? cr : cl;
                    uint32_t s = 0x0Cu;
                    for (uint32_t y0 = 0; y0 < 2; ++y0)
                        for (uint32_t x0 = 0; x0 < 2; ++x0) {
                            uint32_t oy = 0, ox = 0;
                            turn1(c, y0, x0, oy, ox);
                            if (oy == Y && ox == X) s = 4u * y0 + 2u * x1 + x0;
                        }
                    sel |= s << (8 * J);
                }
                t.sub[cl + 4 * cr][Y] = sel;
            }
    for (uint32_t r = 0; r < 4; ++r)
        for (uint32_t I = 0; I < 4; ++I) {
            uint32_t lo = 0, hi = 0;
            for (uint32_t J = 0; J < 4; ++J) {
                uint32_t src_i = 0, src_j = 0;
                for (uint32_t i = 0; i < 4; ++i)
                    for (uint32_t j = 0; j < 4; ++j) {
                        uint32_t Y1 = 0, X1 = 0, Y0 = 0, X0 = 0;
                        turn1(r, i >> 1, j >> 1, Y1, X1);
                        turn1(r, i & 1u, j & 1u, Y0, X0);
                        if (2 * Y1 + Y0 == I && 2 * X1 + X0 == J) { src_i = i; src_j = j; }
                    }
                const uint32_t a = src_i < 2 ? 4u * src_i + src_j : 0x0Cu;
                const uint32_t b = src_i < 2 ? 0x0Cu : 4u * (src_i - 2) + src_j;
                lo |= a << (8 * J);
                hi |= b << (8 * J);
            }
            t.whole[r][2 * I] = lo;
            t.whole[r][2 * I + 1] = hi;
        }
    for (uint32_t k = 0; k < 16; ++k) {
        const uint32_t n = ((4u - (k & 3u)) & 3u) + 4u * ((4u - (k >> 2)) & 3u);
        t.sub_inv[k][0] = t.sub[n][0];
        t.sub_inv[k][1] = t.sub[n][1];
    }
    return t;
}

constexpr Tables kTables = make_tables();
constexpr int kWords = (int)(sizeof(Tables) / sizeof(uint32_t));   // 96

// The inverse as one step: the whole-block turn by -R1 and the negated
// level-1 turns composed, so that row 2h + Y of the source block is
//   vperm(w1, w0, c) | vperm(w3, w2, d),  (c, d) = inv[R1][h][k][2Y], [2Y + 1],
// with k the level-1 codes (left + 4 right) of row pair h.  Every selector
// byte of c or d is either a byte of the composed move or 0x0C, and exactly
// one of the two is not 0x0C.
struct InvTables {
    uint32_t inv[4][2][16][4];
};

constexpr InvTables make_inv_tables() {
    const Tables t = make_tables();
    InvTables f{};
    for (uint32_t R1 = 0; R1 < 4; ++R1) {
        const uint32_t r = (4u - R1) & 3u;
        for (uint32_t h = 0; h < 2; ++h)
            for (uint32_t k = 0; k < 16; ++k)
                for (uint32_t Y = 0; Y < 2; ++Y) {
                    const uint32_t s = t.sub_inv[k][Y];
                    uint32_t c = 0, d = 0;
                    for (uint32_t J = 0; J < 4; ++J) {
                        const uint32_t sj = (s >> (8 * J)) & 0xFFu;      // byte of t[2h] (0..3) or t[2h+1] (4..7)
                        const uint32_t I = 2 * h + (sj >> 2), jj = sj & 3u;
                        const uint32_t a = (t.whole[r][2 * I] >> (8 * jj)) & 0xFFu;
                        const uint32_t b = (t.whole[r][2 * I + 1] >> (8 * jj)) & 0xFFu;
                        c |= a << (8 * J);
                        d |= b << (8 * J);
                    }
                    f.inv[R1][h][k][2 * Y] = c;
                    f.inv[R1][h][k][2 * Y + 1] = d;
                }
    }
    return f;
}

constexpr InvTables kInvTables = make_inv_tables();
constexpr int kInvWords = (int)(sizeof(InvTables) / sizeof(uint32_t));   // 512

}  // namespace perm4
}  // namespace rdhei

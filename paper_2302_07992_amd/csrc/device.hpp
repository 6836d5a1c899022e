// Device helpers for gfx950: keystream, job lookup, the closed form of the
// composed block rotation.
#pragma once
#include "internal.hpp"
#include "perm4.hpp"

namespace rdhei {

// ---- Global-memory access ------------------------------------------------------
// Loads and stores through address-space-1 pointers compile to global_* (not
// flat_*) instructions, whose completion is counted on vmcnt only; flat
// accesses also hold up every wait on scalar and LDS results.
template <typename T>
__device__ __forceinline__ T gload(const void *p) {
    return *(const __attribute__((address_space(1))) T *)(p);
}
template <typename T>
__device__ __forceinline__ void gstore(void *p, T v) {
    *(__attribute__((address_space(1))) T *)(p) = v;
}
typedef uint32_t v4u32 __attribute__((ext_vector_type(4)));
template <>
__device__ __forceinline__ uint4 gload<uint4>(const void *p) {
    const v4u32 v = *(const __attribute__((address_space(1))) v4u32 *)(p);
    return make_uint4(v.x, v.y, v.z, v.w);
}
template <>
__device__ __forceinline__ void gstore<uint4>(void *p, uint4 v) {
    const v4u32 w = {v.x, v.y, v.z, v.w};
    *(__attribute__((address_space(1))) v4u32 *)(p) = w;
}

// ---- Keystream ---------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32x32->64
// multiplies, key bumped by the Weyl constants between rounds.  The paper only
// asks for a secure stream cipher (Sec. III-A, secret key generation); a
// counter-based generator lets every 16-byte piece of the stream be produced
// independently, which is what a data-parallel kernel needs.
struct U4 { uint32_t x, y, z, w; };

__device__ __forceinline__ U4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                     uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)c0 * 0xD2511F53u;
        const uint64_t p1 = (uint64_t)c2 * 0xCD9E8D57u;
        // three-input XOR in one instruction (truth table 0x96)
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return U4{c0, c1, c2, c3};
}

// ChaCha20 (Bernstein 2008, in the IETF layout: four constant words, eight
// key words, a 32-bit block counter, three nonce words; ten double rounds of
// four column and four diagonal quarter rounds, then the input added back).
// It is the cryptographically secure stream cipher Sec. III-A asks for, and it
// is counter-based too, so any 64-byte block comes on its own.
__device__ __forceinline__ void chacha_qr(uint32_t &a, uint32_t &b, uint32_t &c, uint32_t &d) {
    a += b; d = __builtin_rotateleft32(d ^ a, 16);
    c += d; b = __builtin_rotateleft32(b ^ c, 12);
    a += b; d = __builtin_rotateleft32(d ^ a, 8);
    c += d; b = __builtin_rotateleft32(b ^ c, 7);
}

// Words 4q..4q+3 of the ChaCha20 block with key (k0, k1, 0, ..., 0), counter
// ctr and nonce (n0, n1, n2).
__device__ __forceinline__ U4 chacha20_quarter(uint32_t k0, uint32_t k1, uint32_t ctr, uint32_t n0, uint32_t n1,
                                               uint32_t n2, uint32_t q) {
    const uint32_t c0 = 0x61707865u, c1 = 0x3320646eu, c2 = 0x79622d32u, c3 = 0x6b206574u;
    uint32_t x0 = c0, x1 = c1, x2 = c2, x3 = c3;
    uint32_t x4 = k0, x5 = k1, x6 = 0, x7 = 0, x8 = 0, x9 = 0, x10 = 0, x11 = 0;
    uint32_t x12 = ctr, x13 = n0, x14 = n1, x15 = n2;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        chacha_qr(x0, x4, x8, x12);
        chacha_qr(x1, x5, x9, x13);
        chacha_qr(x2, x6, x10, x14);
        chacha_qr(x3, x7, x11, x15);
        chacha_qr(x0, x5, x10, x15);
        chacha_qr(x1, x6, x11, x12);
        chacha_qr(x2, x7, x8, x13);
        chacha_qr(x3, x4, x9, x14);
    }
    U4 o;
    o.x = q == 0 ? x0 + c0 : q == 1 ? x4 + k0 : q == 2 ? x8 : x12 + ctr;
    o.y = q == 0 ? x1 + c1 : q == 1 ? x5 + k1 : q == 2 ? x9 : x13 + n0;
    o.z = q == 0 ? x2 + c2 : q == 1 ? x6 : q == 2 ? x10 : x14 + n1;
    o.w = q == 0 ? x3 + c3 : q == 1 ? x7 : q == 2 ? x11 : x15 + n2;
    return o;
}

// DPP quad_perm: lane i of each group of four lanes reads lane sel_i, CTRL =
// sel_0 | sel_1 << 2 | sel_2 << 4 | sel_3 << 6.
template <int CTRL>
__device__ __forceinline__ uint32_t qperm(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, CTRL, 0xF, 0xF, false);
}

template <int CTRL>
__device__ __forceinline__ uint32_t chacha_row(uint32_t a, uint32_t b, uint32_t c, uint32_t d, uint32_t g) {
    const uint32_t ra = qperm<CTRL>(a), rb = qperm<CTRL>(b), rc = qperm<CTRL>(c), rd = qperm<CTRL>(d);
    return g == 0 ? ra : g == 1 ? rb : g == 2 ? rc : rd;
}

// One ChaCha20 block computed by the four lanes of a lane quad together (same
// key, counter and nonce in all four): lane g = lane id mod 4 holds column g of
// the state (words g, 4+g, 8+g, 12+g) and runs its quarter round; for the
// diagonal rounds rows 1, 2 and 3 are first turned by one, two and three lanes
// (lane g then holds words 4+(g+1)%4, 8+(g+2)%4, 12+(g+3)%4, which is diagonal
// g) and turned back afterwards.  A transpose inside the quad leaves lane g
// with words 4g..4g+3.  A quarter of the full block's work per lane; every lane
// of each quad must be active.
__device__ __forceinline__ U4 chacha20_quad(uint32_t k0, uint32_t k1, uint32_t ctr, uint32_t n0, uint32_t n1,
                                            uint32_t n2) {
    const uint32_t g = __lane_id() & 3u;
    const uint32_t cst = g == 0 ? 0x61707865u : g == 1 ? 0x3320646eu : g == 2 ? 0x79622d32u : 0x6b206574u;
    const uint32_t key = g == 0 ? k0 : g == 1 ? k1 : 0u;
    const uint32_t ctl = g == 0 ? ctr : g == 1 ? n0 : g == 2 ? n1 : n2;
    uint32_t a = cst, b = key, c = 0u, d = ctl;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        chacha_qr(a, b, c, d);
        b = qperm<0x39>(b);     // from lane (g + 1) % 4
        c = qperm<0x4E>(c);     // from lane (g + 2) % 4
        d = qperm<0x93>(d);     // from lane (g + 3) % 4
        chacha_qr(a, b, c, d);
        b = qperm<0x93>(b);
        c = qperm<0x4E>(c);
        d = qperm<0x39>(d);
    }
    a += cst;
    b += key;
    d += ctl;
    // word 4g + j is row g of column j: register g of lane j (every lane reads
    // all four registers of lane j, then keeps its own row)
    U4 o;
    o.x = chacha_row<0x00>(a, b, c, d, g);
    o.y = chacha_row<0x55>(a, b, c, d, g);
    o.z = chacha_row<0xAA>(a, b, c, d, g);
    o.w = chacha_row<0xFF>(a, b, c, d, g);
    return o;
}

constexpr uint32_t kDomainImage = 1;
constexpr uint32_t kDomainMessage = 2;

// The 16 stream bytes [16*blk, 16*blk+16) of the stream (key, nonce, domain)
// as four little-endian words (streams stay below 2^36 bytes: images of at
// most 2^31 pixels, messages of at most 7 bits per pixel).  Philox: one block
// per 16 bytes, counter (blk, nonce high word, domain, nonce low word).
// ChaCha20: the 64-byte block blk/4 with the 64-bit key in key words 0-1,
// block counter blk/4 and nonce (domain, nonce low word, nonce high word), so
// the stream is ChaCha20's own byte stream for that key and 96-bit nonce.
template <int KS>
__device__ __forceinline__ U4 stream_block(uint64_t key, uint64_t nonce, uint32_t domain, uint64_t blk) {
    if constexpr (KS == kKsChaCha20)
        return chacha20_quarter((uint32_t)key, (uint32_t)(key >> 32), (uint32_t)(blk >> 2), domain, (uint32_t)nonce,
                                (uint32_t)(nonce >> 32), (uint32_t)blk & 3u);
    else
        return philox((uint32_t)blk, (uint32_t)(nonce >> 32), domain, (uint32_t)nonce, (uint32_t)key,
                      (uint32_t)(key >> 32));
}

// stream_block for call sites where the four lanes of every lane quad ask,
// together, for the four 16-byte pieces of one 64-byte-aligned stream block,
// lane l for piece l % 4 (the tiled kernels: lanes 4k..4k+3 cover one 64-byte
// tile row, and tile rows start on multiples of 64 because M and N are).
// ChaCha20 then shares one block among the four lanes.
template <int KS>
__device__ __forceinline__ U4 stream_block_quad(uint64_t key, uint64_t nonce, uint32_t domain, uint64_t blk) {
    if constexpr (KS == kKsChaCha20)
        return chacha20_quad((uint32_t)key, (uint32_t)(key >> 32), (uint32_t)(blk >> 2), domain, (uint32_t)nonce,
                             (uint32_t)(nonce >> 32));
    else
        return stream_block<KS>(key, nonce, domain, blk);
}

template <int KS>
__device__ __forceinline__ uint32_t stream_byte(uint64_t key, uint64_t nonce, uint32_t domain, uint64_t idx) {
    U4 v = stream_block<KS>(key, nonce, domain, idx >> 4);
    uint32_t w = ((idx >> 2) & 3) == 0 ? v.x : ((idx >> 2) & 3) == 1 ? v.y : ((idx >> 2) & 3) == 2 ? v.z : v.w;
    return (w >> (8 * (idx & 3))) & 0xFFu;
}

// Values that decide whether a workgroup reaches a barrier are made
// wave-uniform (readfirstlane), so the compiler keeps that control flow scalar
// instead of building exec-mask loops around the barriers.
__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t uni64(uint64_t v) {
    return ((uint64_t)uni((uint32_t)(v >> 32)) << 32) | uni((uint32_t)v);
}

// Inclusive sum over the 64 lanes of a wave.
__device__ __forceinline__ uint32_t wave_scan_incl(uint32_t x) {
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, true);    // row_shr:1
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, true);    // row_shr:2
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, true);    // row_shr:4
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, true);    // row_shr:8
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xA, 0xF, false);   // row_bcast:15
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xC, 0xF, false);   // row_bcast:31
    return x;
}

// Lane l + N of the same row of 16 lanes (DPP row_shl), 0 past the row's end.
template <int N>
__device__ __forceinline__ uint32_t row_shl(uint32_t x) {
    static_assert(N >= 1 && N <= 15, "row_shl takes 1..15");
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x100 + N, 0xF, 0xF, true);
}

// ---- Batches -----------------------------------------------------------------
// Index of the job owning work unit u of a kind: one load from the per-unit
// table when the launch has one, else a search over the ascending bases.
template <int KIND>
__device__ __forceinline__ int find_job(const Job *jobs, int njobs, uint32_t u, const uint32_t *ujob) {
    if (ujob) return (int)ujob[u];
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].ubase[KIND] <= u) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Per-image keystream nonce: the content owner's choice at encryption (in the
// job table), read back from the public meta record by the other roles.
__device__ __forceinline__ uint64_t job_nonce(const Job &J) {
    return J.nonce_meta ? uni64(gload<uint64_t>(&J.meta->nonce)) : J.nonce;
}

// ---- Rotation ------------------------------------------------------------------
// A quarter turn counter-clockwise of a 2^m block maps local (y, x) to
// (2^m-1-x, y): per coordinate bit, (y_j, x_j) -> (!x_j, y_j).  Because a block
// turn at level m acts on every bit below m the same way, and the block index
// used at every level is a function of the untouched high bits, the composed
// map of all levels turns bit pair j by R_j = sum of the codes of the blocks
// (levels m > j, full blocks only) containing the pixel.
__device__ __forceinline__ void turn_bits(uint32_t r, uint32_t &y, uint32_t &x, uint32_t mask) {
    // r = 0: (y, x); 1: (!x, y); 2: (!y, !x); 3: (x, !y), on the bits in mask.
    const uint32_t sw = r & 1u;
    const uint32_t ny = sw ? x : y;
    const uint32_t nx = sw ? y : x;
    const uint32_t fy = (r == 1u || r == 2u) ? mask : 0u;
    const uint32_t fx = (r >= 2u) ? mask : 0u;
    y = (ny ^ fy) & mask;
    x = (nx ^ fx) & mask;
}

// Code (2 bits) of block (by, bx) of tile-level m from a packed record in LDS.
__device__ __forceinline__ uint32_t tile_code(const uint8_t *rec, int m, uint32_t by, uint32_t bx) {
    const uint32_t q = by * (uint32_t)(kTile >> m) + bx;
    return (rec[code_off(m) + (q >> 2)] >> (2 * (q & 3))) & 3u;
}

// Byte offset of level m (> kTileLog) of the upper pyramid, whose level
// kTileLog is the tiles_y x tiles_x array of tile sums.
__device__ __host__ inline uint64_t pyr_off(int M, int N, int m) {
    uint64_t off = 0;
    for (int k = kTileLog; k < m; ++k) off += (uint64_t)(M >> k) * (uint64_t)(N >> k);
    return off;
}

// Where a whole tile goes: levels above the tile move the tile rigidly.  Walks
// levels ascending on tile coordinates; returns the destination tile and the
// number of quarter turns the tile's content receives.
__device__ __forceinline__ void upper_walk(const Job &J, const uint8_t *pyr, int ty, int tx,
                                           int &dy, int &dx, uint32_t &turns) {
    uint32_t cy = (uint32_t)ty, cx = (uint32_t)tx, o = 0;
    const int lo = J.min_level > kTileLog + 1 ? J.min_level : kTileLog + 1;
    for (int m = lo; m <= J.max_level; ++m) {
        const int sh = m - kTileLog;
        const uint32_t BY = (uint32_t)ty >> sh, BX = (uint32_t)tx >> sh;
        const uint32_t gy = (uint32_t)(J.M >> m), gx = (uint32_t)(J.N >> m);
        if (BY < gy && BX < gx) {
            const uint32_t r = pyr[pyr_off(J.M, J.N, m) + BY * gx + BX] & 3u;
            o += r;
            const uint32_t mask = (1u << sh) - 1u;
            uint32_t ly = cy & mask, lx = cx & mask;
            turn_bits(r, ly, lx, mask);
            cy = (cy & ~mask) | ly;
            cx = (cx & ~mask) | lx;
        }
    }
    dy = (int)cy;
    dx = (int)cx;
    turns = o & 3u;
}

// Tile-map entry: destination tile row (bits 0..13), column (bits 14..27) and
// quarter turns of the content (bits 28..29); the host sends images with more
// than kTmapMaxTiles tiles along a side to the per-pixel path.
__device__ __forceinline__ uint32_t tmap_pack(int dy, int dx, uint32_t turns) {
    return (uint32_t)dy | ((uint32_t)dx << 14) | (turns << 28);
}
__device__ __forceinline__ void tmap_unpack(uint32_t v, int &dy, int &dx, uint32_t &turns) {
    dy = (int)(v & 0x3FFFu);
    dx = (int)((v >> 14) & 0x3FFFu);
    turns = (v >> 28) & 3u;
}

// Destinations inside the tile of the 16 pixels of 4x4 block (by, bx), given
// the tile's code record and the turns added by the levels above the tile.
// dst[k] = (row << 8) | col for pixel k = 4*u + v of the block.
__device__ __forceinline__ void block_map(const uint8_t *rec, int min_level, uint32_t up_turns,
                                          uint32_t by, uint32_t bx, uint32_t dst[16]) {
    // turns per pixel bit j >= 2 (block bit j - 2), accumulated from the top
    uint32_t acc = up_turns;
    uint32_t ny = 0, nx = 0;
#pragma unroll
    for (int m = kTileLog; m >= 3; --m) {
        if (m >= min_level) acc += tile_code(rec, m, by >> (m - 2), bx >> (m - 2));
        const int j = m - 3;             // block bit j carries pixel bit m - 1
        uint32_t yb = (by >> j) & 1u, xb = (bx >> j) & 1u;
        turn_bits(acc & 3u, yb, xb, 1u);
        ny |= yb << j;
        nx |= xb << j;
    }
    const uint32_t r1 = (acc + (2 >= min_level ? tile_code(rec, 2, by, bx) : 0u)) & 3u;
#pragma unroll
    for (int su = 0; su < 2; ++su) {
#pragma unroll
        for (int sv = 0; sv < 2; ++sv) {
            uint32_t y1 = (uint32_t)su, x1 = (uint32_t)sv;
            turn_bits(r1, y1, x1, 1u);
            const uint32_t r0 = (r1 + (1 >= min_level ? tile_code(rec, 1, 2 * by + su, 2 * bx + sv) : 0u)) & 3u;
#pragma unroll
            for (int pu = 0; pu < 2; ++pu) {
#pragma unroll
                for (int pv = 0; pv < 2; ++pv) {
                    uint32_t y0 = (uint32_t)pu, x0 = (uint32_t)pv;
                    turn_bits(r0, y0, x0, 1u);
                    const uint32_t row = (ny << 2) | (y1 << 1) | y0;
                    const uint32_t col = (nx << 2) | (x1 << 1) | x0;
                    dst[(2 * su + pu) * 4 + (2 * sv + pv)] = (row << 8) | col;
                }
            }
        }
    }
}

// Destination of 4x4 block (by, bx) inside the tile, and the turns of its
// content: R1 (levels >= 2 and the turns from above the tile) and the level-1
// codes of its 2x2 sub-blocks packed per row pair (left + 4 * right); levels
// below min_level contribute nothing.
__device__ __forceinline__ void block_turns(const uint8_t *rec, int min_level, uint32_t up_turns, uint32_t by,
                                            uint32_t bx, uint32_t &ny, uint32_t &nx, uint32_t &R1, uint32_t &k0,
                                            uint32_t &k1) {
    uint32_t acc = up_turns;
    ny = 0;
    nx = 0;
#pragma unroll
    for (int m = kTileLog; m >= 3; --m) {
        if (m >= min_level) acc += tile_code(rec, m, by >> (m - 2), bx >> (m - 2));
        const int j = m - 3;
        uint32_t yb = (by >> j) & 1u, xb = (bx >> j) & 1u;
        turn_bits(acc & 3u, yb, xb, 1u);
        ny |= yb << j;
        nx |= xb << j;
    }
    R1 = (acc + (2 >= min_level ? tile_code(rec, 2, by, bx) : 0u)) & 3u;
    if (min_level <= 1) {
        const uint32_t q0 = (2u * by) * (uint32_t)(kTile >> 1) + 2u * bx;
        const uint32_t q1 = q0 + (uint32_t)(kTile >> 1);
        k0 = (rec[code_off(1) + (q0 >> 2)] >> (2 * (q0 & 3u))) & 0xFu;
        k1 = (rec[code_off(1) + (q1 >> 2)] >> (2 * (q1 & 3u))) & 0xFu;
    } else {
        k0 = 0;
        k1 = 0;
    }
}

// Quarter turns of one coordinate bit pair as a 32-bit table: entry r*4 + y*2 + x
// (2 bits) holds (y', x') as y'*2 + x' for r = 0 (y, x), 1 (!x, y), 2 (!y, !x),
// 3 (x, !y).
constexpr uint32_t turn_lut() {
    uint32_t t = 0;
    for (uint32_t r = 0; r < 4; ++r)
        for (uint32_t y = 0; y < 2; ++y)
            for (uint32_t x = 0; x < 2; ++x) {
                const uint32_t oy = r == 0 ? y : r == 1 ? (x ^ 1u) : r == 2 ? (y ^ 1u) : x;
                const uint32_t ox = r == 0 ? x : r == 1 ? y : r == 2 ? (x ^ 1u) : (y ^ 1u);
                t |= (oy * 2 + ox) << (2 * (r * 4 + y * 2 + x));
            }
    return t;
}
constexpr uint32_t kTurnLut = turn_lut();
__device__ __forceinline__ uint32_t turn2(uint32_t r, uint32_t y, uint32_t x) {   // -> y' * 2 + x'
    return (kTurnLut >> (2 * (((r & 3u) << 2) | (y << 1) | x))) & 3u;
}

// block_turns for the four blocks (by, 4c..4c+3) of one lane's 4x16 strip:
// the codes of levels 4..6 and the upper bits are shared, and the level-1,
// 2 and 3 codes of the four blocks come from a few record bytes.
__device__ __forceinline__ void block_turns4(const uint8_t *rec, int min_level, uint32_t up, uint32_t by, uint32_t c,
                                             uint32_t ny[4], uint32_t nx[4], uint32_t R1[4], uint32_t k0[4],
                                             uint32_t k1[4]) {
    // levels 6 and 5 turn block bits 3 and 2, shared by the four blocks (bx = 4c + k)
    uint32_t acc = up;
    if (6 >= min_level) acc += rec[code_off(6)] & 3u;
    const uint32_t t6 = turn2(acc, (by >> 3) & 1u, (c >> 1) & 1u);
    if (5 >= min_level) acc += tile_code(rec, 5, by >> 3, c >> 1);
    const uint32_t t5 = turn2(acc, (by >> 2) & 1u, c & 1u);
    if (4 >= min_level) acc += tile_code(rec, 4, by >> 2, c);
    const uint32_t hy = ((t6 >> 1) << 3) | ((t5 >> 1) << 2), hx = ((t6 & 1u) << 3) | ((t5 & 1u) << 2);
    // level 3: two codes (bx >> 1 = 2c, 2c + 1) in one byte; level 2: four codes in one byte
    const uint32_t q3 = (by >> 1) * 8u + 2u * c;
    const uint32_t c3b = 3 >= min_level ? (uint32_t)rec[code_off(3) + (q3 >> 2)] >> (2 * (q3 & 3u)) : 0u;
    const uint32_t c2b = 2 >= min_level ? (uint32_t)rec[code_off(2) + by * 4u + c] : 0u;
    // level 1: per row pair of sub-blocks, 16 bits = the four blocks' nibbles
    uint32_t l1a = 0, l1b = 0;
    if (min_level <= 1) {
        l1a = *reinterpret_cast<const uint16_t *>(rec + code_off(1) + (2u * by) * 8u + 2u * c);
        l1b = *reinterpret_cast<const uint16_t *>(rec + code_off(1) + (2u * by + 1u) * 8u + 2u * c);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t t4 = turn2(acc, (by >> 1) & 1u, (uint32_t)(k >> 1));
        const uint32_t a3 = acc + ((c3b >> (2 * (k >> 1))) & 3u);
        const uint32_t t3 = turn2(a3, by & 1u, (uint32_t)(k & 1));
        ny[k] = hy | ((t4 >> 1) << 1) | (t3 >> 1);
        nx[k] = hx | ((t4 & 1u) << 1) | (t3 & 1u);
        R1[k] = (a3 + ((c2b >> (2 * k)) & 3u)) & 3u;
        k0[k] = (l1a >> (4 * k)) & 0xFu;
        k1[k] = (l1b >> (4 * k)) & 0xFu;
    }
}

// ---- 4x4 block permutes (selector tables staged in LDS) -------------------------
static __constant__ perm4::Tables kPermTables = perm4::kTables;
constexpr int kPermSub = 0, kPermWhole = 32, kPermSubInv = 64;

__device__ __forceinline__ void stage_perm_tables(uint32_t *lds, int tid) {
    if (tid < perm4::kWords) lds[tid] = reinterpret_cast<const uint32_t *>(&kPermTables)[tid];
}

__device__ __forceinline__ uint32_t vperm(uint32_t a, uint32_t b, uint32_t sel) {
    return __builtin_amdgcn_perm(a, b, sel);
}

// Rows w of a source block -> rows o of the block at its destination.
__device__ __forceinline__ void block_forward(const uint32_t *T, uint32_t R1, uint32_t k0, uint32_t k1,
                                              const uint32_t w[4], uint32_t o[4]) {
    const uint2 s0 = *reinterpret_cast<const uint2 *>(T + kPermSub + 2 * k0);
    const uint2 s1 = *reinterpret_cast<const uint2 *>(T + kPermSub + 2 * k1);
    const uint32_t t0 = vperm(w[1], w[0], s0.x), t1 = vperm(w[1], w[0], s0.y);
    const uint32_t t2 = vperm(w[3], w[2], s1.x), t3 = vperm(w[3], w[2], s1.y);
    const uint4 a = *reinterpret_cast<const uint4 *>(T + kPermWhole + 8 * R1);
    const uint4 b = *reinterpret_cast<const uint4 *>(T + kPermWhole + 8 * R1 + 4);
    o[0] = vperm(t1, t0, a.x) | vperm(t3, t2, a.y);
    o[1] = vperm(t1, t0, a.z) | vperm(t3, t2, a.w);
    o[2] = vperm(t1, t0, b.x) | vperm(t3, t2, b.y);
    o[3] = vperm(t1, t0, b.z) | vperm(t3, t2, b.w);
}

// Rows w of a block at its destination -> rows o of the source block.  The
// selectors are shared by the two planes the recovery moves.
struct InvSel {
    uint4 a, b;
    uint2 s0, s1;
};
__device__ __forceinline__ InvSel inverse_selectors(const uint32_t *T, uint32_t R1, uint32_t k0, uint32_t k1) {
    const uint32_t r = (4u - R1) & 3u;
    InvSel S;
    S.a = *reinterpret_cast<const uint4 *>(T + kPermWhole + 8 * r);
    S.b = *reinterpret_cast<const uint4 *>(T + kPermWhole + 8 * r + 4);
    S.s0 = *reinterpret_cast<const uint2 *>(T + kPermSubInv + 2 * k0);
    S.s1 = *reinterpret_cast<const uint2 *>(T + kPermSubInv + 2 * k1);
    return S;
}
__device__ __forceinline__ void block_inverse(const InvSel &S, const uint32_t w[4], uint32_t o[4]) {
    const uint32_t t0 = vperm(w[1], w[0], S.a.x) | vperm(w[3], w[2], S.a.y);
    const uint32_t t1 = vperm(w[1], w[0], S.a.z) | vperm(w[3], w[2], S.a.w);
    const uint32_t t2 = vperm(w[1], w[0], S.b.x) | vperm(w[3], w[2], S.b.y);
    const uint32_t t3 = vperm(w[1], w[0], S.b.z) | vperm(w[3], w[2], S.b.w);
    o[0] = vperm(t1, t0, S.s0.x);
    o[1] = vperm(t1, t0, S.s0.y);
    o[2] = vperm(t3, t2, S.s1.x);
    o[3] = vperm(t3, t2, S.s1.y);
}

}  // namespace rdhei

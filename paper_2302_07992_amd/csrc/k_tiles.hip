// Tiled fast path (M, N multiples of 64): keystream code pyramid + label
// statistics, per-image finalisation (optimal b, upper rotation levels), the
// permuting encryption, and the recovery (EMR by 2x2 tile quads, LMR by bands).
//
// The tile kernels are persistent: each workgroup owns a contiguous range of
// work units (tiles of one image stay on one workgroup, hence on one XCD and
// its L2) and loads the next unit's inputs before working on the current one.
#include <mutex>
#include <type_traits>
#include <unordered_map>

#include "device.hpp"
#include "glide4.hpp"

namespace rdhei {

// Byte offset of 4x4 block (by, bx) in a wave's tile of blocks: 16 bytes per
// block, 16 blocks per block row, columns swizzled so that the writes of
// lanes (q, g) and (q + 1, g) fall in different banks.
__device__ __forceinline__ uint32_t blk_addr(uint32_t by, uint32_t bx) {
    const uint32_t sw = (((bx >> 3) & 1u) << 1) ^ (by & 1u);
    return by * 256u + ((bx ^ sw) << 4);
}

// Contiguous unit range [u0, u1) of this workgroup, its length rounded up to
// a multiple of `align` (the last workgroups may get less, or nothing).
__device__ __forceinline__ void unit_range(uint32_t units, uint32_t &u0, uint32_t &u1, uint32_t align = 1) {
    const uint64_t per = (((uint64_t)units + gridDim.x - 1) / gridDim.x + align - 1) / align * align;
    const uint64_t a = (uint64_t)blockIdx.x * per, b = a + per;
    u0 = (uint32_t)(a < units ? a : units);
    u1 = (uint32_t)(b < units ? b : units);
}

// ----------------------------------------------------------------------------
// Per-tile building blocks shared by the staged kernels (k_tile_prep,
// k_encrypt_quad) and the one-workgroup-per-image encryption (k_encrypt_image).
// Lane (q, g) of the wave that owns a tile holds rows 4q..4q+3, columns
// 16g..16g+15 of it.
// ----------------------------------------------------------------------------

// Rotation codes of tile t (levels 1..6 inside the tile, Sec. III-A rotation
// equation: block code = (sum of s over the block) mod 4) into the tile's code
// record, and the tile's own code (level 6) into the pyramid.
template <int KS>
__device__ __forceinline__ void tile_codes(const Job &J, uint64_t nz, uint32_t t, int ty, int tx, int q, int g, int lane,
                                           uint8_t *__restrict__ ws) {
    const uint64_t idx0 = (uint64_t)(ty * kTile + 4 * q) * (uint64_t)J.N + (uint64_t)(tx * kTile + 16 * g);

    // level 1 (2x2) pair sums: h[pp][k] bytes 0 and 2, rows 4q+2pp..+1, columns 16g+4k..+3
    uint32_t h[2][4];
#pragma unroll
    for (int pp = 0; pp < 2; ++pp) {
        const U4 sa = stream_block_quad<KS>(J.key, nz, kDomainImage, (idx0 + (uint64_t)(2 * pp) * J.N) >> 4);
        const U4 sb = stream_block_quad<KS>(J.key, nz, kDomainImage, (idx0 + (uint64_t)(2 * pp + 1) * J.N) >> 4);
        const uint32_t wa[4] = {sa.x, sa.y, sa.z, sa.w}, wb[4] = {sb.x, sb.y, sb.z, sb.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t a = (wa[k] & 0x03030303u) + (wb[k] & 0x03030303u);   // <= 6 per byte
            h[pp][k] = a + (a >> 8);                                            // bytes 0, 2: <= 12
        }
    }
    // level-1 codes: code row 4q/2 + pp, code columns 8g..8g+7 -> 16 bits
    uint8_t *rec = ws + J.ws_codes + (uint64_t)t * kCodeRecord;
#pragma unroll
    for (int pp = 0; pp < 2; ++pp) {
        const uint32_t c = vperm(h[pp][1], h[pp][0], 0x06040200u) & 0x03030303u;
        const uint32_t d = vperm(h[pp][3], h[pp][2], 0x06040200u) & 0x03030303u;
        const uint32_t c8 = (c | (c >> 6) | (c >> 12) | (c >> 18)) & 0xFFu;
        const uint32_t d8 = (d | (d >> 6) | (d >> 12) | (d >> 18)) & 0xFFu;
        gstore<uint16_t>(rec + code_off(1) + (2 * q + pp) * 8 + 2 * g, (uint16_t)(c8 | (d8 << 8)));
    }
    // level 2 (4x4): block (q, 4g + k)
    uint32_t L2[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t v = h[0][k] + h[1][k];
        L2[k] = (v + (v >> 16)) & 0xFFu;                    // <= 48
    }
    gstore<uint8_t>(rec + code_off(2) + q * 4 + g,
                    (uint8_t)((L2[0] & 3u) | ((L2[1] & 3u) << 2) | ((L2[2] & 3u) << 4) | ((L2[3] & 3u) << 6)));
    // level 3 (8x8): block (q/2, 2g + jj) for even q, from lanes q and q+1
    const uint32_t hs = (L2[0] + L2[1]) | ((L2[2] + L2[3]) << 16);
    // (lanes of a row of 16 are q = 4r..4r+3, so these partners stay in the row)
    const uint32_t L3 = hs + row_shl<4>(hs);                // halves: columns 2g, 2g+1
    const uint32_t nib = (L3 & 3u) | ((L3 >> 14) & 0xCu);
    const uint32_t nib_hi = row_shl<1>(nib);
    if ((q & 1) == 0 && (g & 1) == 0)
        gstore<uint8_t>(rec + code_off(3) + (q >> 1) * 2 + (g >> 1), (uint8_t)(nib | (nib_hi << 4)));
    // level 4 (16x16): block (q/4, g) for q % 4 == 0, from lanes q, q+2
    const uint32_t l3s = (L3 & 0xFFFFu) + (L3 >> 16);
    const uint32_t L4 = l3s + row_shl<8>(l3s);
    const uint32_t c4 = L4 & 3u;
    const uint32_t c4row = c4 | (row_shl<1>(c4) << 2) | (row_shl<2>(c4) << 4) | (row_shl<3>(c4) << 6);
    if ((q & 3) == 0 && g == 0) gstore<uint8_t>(rec + code_off(4) + (q >> 2), (uint8_t)c4row);
    // level 5 (32x32): the sums of 16x16 column pairs sit in lanes 0, 2 (rows 0..15),
    // 16, 18 (16..31), 32, 34, 48, 50; level 6 (the tile) follows, on the scalar unit
    const uint32_t l4h = L4 + row_shl<1>(L4);
    auto at = [&](int l) { return (uint32_t)__builtin_amdgcn_readlane((int)l4h, l); };
    const uint32_t c5a = (at(0) + at(16)) & 3u, c5b = (at(2) + at(18)) & 3u;
    const uint32_t c5c = (at(32) + at(48)) & 3u, c5d = (at(34) + at(50)) & 3u;
    if (lane == 0) {
        const uint32_t c6 = (c5a + c5b + c5c + c5d) & 3u;
        gstore<uint8_t>(rec + code_off(5), (uint8_t)(c5a | (c5b << 2) | (c5c << 4) | (c5d << 6)));
        gstore<uint8_t>(rec + code_off(6), (uint8_t)c6);
        ws[J.ws_pyr + t] = (uint8_t)c6;
    }
}

// The lane's pixels of tile (ty, tx), and the byte left of each of its four
// rows (meaningful in lanes g = 0 of tiles past column 0).
__device__ __forceinline__ void tile_load(const Job &J, int ty, int tx, int q, int g, uint4 p[4], uint32_t &left) {
    const uint8_t *row = J.in + (uint64_t)(ty * kTile + 4 * q) * (uint64_t)J.N + (uint64_t)(tx * kTile + 16 * g);
    uint32_t lb = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        p[i] = gload<uint4>(row + (uint64_t)i * J.N);
        lb |= (uint32_t)gload<uint8_t>(row + (uint64_t)i * J.N - ((g == 0 && tx > 0) ? 1 : 0)) << (8 * i);
    }
    left = lb;
}

// Per lane, the thermometer codes of its pixels (bit k of a byte: x >= 2^k,
// x = pixel XOR left neighbour) are summed bit-sliced: a carry-save tree over
// the 16 words of a tile (ones, twos, fours, eights: weights 1..8) and a ripple
// counter of the tree's sixteens across tiles (hi[p]: weight 16 * 2^p).  Z_b =
// pixels - (pixels with x >= 2^(8-b)); the counters are emptied after at most
// kHeldMax tiles (before hi can overflow).
constexpr int kHiPlanes = 6;
constexpr uint32_t kHeldMax = (1u << kHiPlanes) - 1u;
struct Thermo {
    uint32_t ones, twos, fours, eights, hi[kHiPlanes];
};
__device__ __forceinline__ void thermo_clear(Thermo &C) {
    C.ones = C.twos = C.fours = C.eights = 0;
#pragma unroll
    for (int p = 0; p < kHiPlanes; ++p) C.hi[p] = 0;
}
// carry-save adder: h:l = a + b + c, bitwise
__device__ __forceinline__ void csa(uint32_t &h, uint32_t &l, uint32_t a, uint32_t b, uint32_t c) {
    h = __builtin_amdgcn_bitop3_b32(a, b, c, 0xE8);   // majority
    l = __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);   // parity
}
// lambda >= b exactly when x = pixel XOR left neighbour is below 2^(8-b): y
// smears each byte of x down, so bit k of y says x >= 2^k.  left: the byte left
// of each of the lane's four rows (lanes g = 0); column 0 counts as differing.
__device__ __forceinline__ void tile_thermo(const uint4 p[4], uint32_t left, int tx, int g, uint32_t y[16]) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint32_t w[4] = {p[i].x, p[i].y, p[i].z, p[i].w};
        // byte left of the lane's 16 pixels: lane g-1 of the row, or the previous tile for g = 0
        uint32_t lb = (uint32_t)__builtin_amdgcn_mov_dpp((int)(p[i].w >> 24), 0x90, 0xF, 0xF, false);
        if (g == 0) lb = (left >> (8 * i)) & 0xFFu;
        uint32_t x[4];
        x[0] = w[0] ^ ((w[0] << 8) | lb);
        x[1] = w[1] ^ __builtin_amdgcn_alignbit(w[1], w[0], 24);
        x[2] = w[2] ^ __builtin_amdgcn_alignbit(w[2], w[1], 24);
        x[3] = w[3] ^ __builtin_amdgcn_alignbit(w[3], w[2], 24);
        if (tx == 0 && g == 0) x[0] |= 0xFFu;     // column 0 has no left neighbour
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            uint32_t t = x[k];                                                // t | (t >> s) & mask
            t = __builtin_amdgcn_bitop3_b32(t, t >> 1, 0x7F7F7F7Fu, 0xF8);
            t = __builtin_amdgcn_bitop3_b32(t, t >> 2, 0x3F3F3F3Fu, 0xF8);
            t = __builtin_amdgcn_bitop3_b32(t, t >> 4, 0x0F0F0F0Fu, 0xF8);
            y[4 * i + k] = t;
        }
    }
}
// One tile's 16 thermometer words into the counters: ones, twos, fours,
// eights, and the word of sixteens rippled into hi.
__device__ __forceinline__ void thermo_add(Thermo &C, const uint32_t y[16]) {
    uint32_t tA, tB, fA, fB, eA, eB, sx;
    csa(tA, C.ones, C.ones, y[0], y[1]);
    csa(tB, C.ones, C.ones, y[2], y[3]);
    csa(fA, C.twos, C.twos, tA, tB);
    csa(tA, C.ones, C.ones, y[4], y[5]);
    csa(tB, C.ones, C.ones, y[6], y[7]);
    csa(fB, C.twos, C.twos, tA, tB);
    csa(eA, C.fours, C.fours, fA, fB);
    csa(tA, C.ones, C.ones, y[8], y[9]);
    csa(tB, C.ones, C.ones, y[10], y[11]);
    csa(fA, C.twos, C.twos, tA, tB);
    csa(tA, C.ones, C.ones, y[12], y[13]);
    csa(tB, C.ones, C.ones, y[14], y[15]);
    csa(fB, C.twos, C.twos, tA, tB);
    csa(eB, C.fours, C.fours, fA, fB);
    csa(sx, C.eights, C.eights, eA, eB);
#pragma unroll
    for (int p = 0; p < kHiPlanes; ++p) {
        const uint32_t c = C.hi[p] & sx;
        C.hi[p] ^= sx;
        sx = c;
    }
}
// This lane's pixels with x >= 2^(8-b) in the counters (planes: hi planes in use).
__device__ __forceinline__ uint32_t thermo_ge(const Thermo &C, int b, int planes) {
    const uint32_t m = 0x01010101u << (8 - b);
    uint32_t h = 0;
#pragma unroll
    for (int p = 0; p < kHiPlanes; ++p)
        if (p < planes) h += (uint32_t)__popc(C.hi[p] & m) << p;
    return (uint32_t)__popc(C.ones & m) + 2u * (uint32_t)__popc(C.twos & m) + 4u * (uint32_t)__popc(C.fours & m) +
           8u * (uint32_t)__popc(C.eights & m) + 16u * h;
}
// Dynamic b: the b_t of the one tile in the counters (the first b in 2..7
// reaching the largest b * Z_b(t)), its Z_{b_t}(t) and b_t * Z_{b_t}(t);
// wave-uniform.
__device__ __forceinline__ void thermo_tile_b(const Thermo &C, uint32_t &best_b, uint32_t &best_z, uint32_t &best_s) {
    best_b = 2;
    best_z = 0;
    best_s = 0;
#pragma unroll
    for (int b = 2; b <= 7; ++b) {
        const uint32_t z = uni((uint32_t)__builtin_amdgcn_readlane((int)wave_scan_incl(64u - thermo_ge(C, b, 1)), 63));
        if (b == 2 || (uint32_t)b * z > best_s) {
            best_b = (uint32_t)b;
            best_z = z;
            best_s = (uint32_t)b * z;
        }
    }
}

// ----------------------------------------------------------------------------
// Keystream code pyramid of one tile (Sec. III-A rotation equation: block code
// = (sum of s over the block) mod 4 at every level 2^1..2^6 inside the tile)
// and, for encryption, the counts Z_b of pixels whose leading-shared-bit count
// lambda with their left neighbour is at least b (Sec. III-A location map; the
// Omega glide labels a pixel redundant for b exactly when lambda >= b).
//
// One wave per tile, no workgroup barriers: lane (q, g) holds rows 4q..4q+3,
// columns 16g..16g+15 (four keystream blocks), so levels 1 and 2 sum inside
// the lane, and levels 3..6 take a few lane shuffles.  Only the low two bits
// of every keystream byte matter for the codes.
// lambda >= b means x = pixel XOR left neighbour is below 2^(8-b); the
// thresholds are nested, so each byte of x is smeared into a thermometer code
// (bit k set when x >= 2^k) and the codes are summed bit-sliced, all seven
// thresholds at once.  Counts stay in registers across the tiles of one image
// and go to one of the image's counter slots with one atomic add per wave.
// ----------------------------------------------------------------------------
// DYN (dynamic b, RDHEI_DEMR): every tile's counts give the tile's own b_t,
// the first b in 2..7 reaching the largest b * Z_b(t); b_t goes to the
// image's tile table (original order) and Z_{b_t}(t), b_t * Z_{b_t}(t) are
// added to the image's totals.
template <bool STATS, int KS, bool DYN = false>
__global__ __launch_bounds__(kThreads) void k_tile_prep(const Job *__restrict__ jobs, int njobs,
                                                         uint8_t *__restrict__ ws, uint32_t units,
                                                         const uint32_t *__restrict__ ujob) {
    constexpr uint32_t kW = kThreads / 64;
    const int lane = threadIdx.x & 63, wave = (int)uni(threadIdx.x >> 6);   // wave-uniform
    const int q = lane >> 2, g = lane & 3;
    // the workgroup's contiguous tile range, dealt to its waves in turn so
    // that neighbouring tiles (which share 128-byte lines) are read together;
    // ranges start at multiples of kW tiles, so the two tiles of a line pair
    // (and the byte left of an even tile) fall in one iteration or the one
    // before, never in another workgroup
    uint32_t r0, r1;
    unit_range(units, r0, r1, kW);
    const uint32_t u0 = r0 + (uint32_t)wave, gw = blockIdx.x * kW + (uint32_t)wave;

    // next tile's pixels (STATS): rows 4q..4q+3, and for g = 0 the byte left of each row
    uint4 p_n[4];
    uint32_t left_n = 0;
    auto fetch = [&](uint32_t u) {
        if (!STATS) return;
        const Job &J = jobs[uni((uint32_t)find_job<UNIT_TILE>(jobs, njobs, u, ujob))];
        const uint32_t t = u - J.ubase[UNIT_TILE];
        const int ty = (int)(t / (uint32_t)J.tiles_x), tx = (int)(t % (uint32_t)J.tiles_x);
        tile_load(J, ty, tx, q, g, p_n, left_n);
    };
    if (STATS && u0 < r1) fetch(u0);

    Thermo C;
    thermo_clear(C);
    uint32_t held = 0;   // tiles in the counters (wave-uniform)
    int cur_j = -1;
    auto flush = [&](int jj) {                  // wave sums into one of the image's counter slots
        if (!STATS || jj < 0) return;
        const Job &Jf = jobs[jj];
        const uint32_t slot = gw % stat_slots(Jf);
        uint32_t *st = reinterpret_cast<uint32_t *>(ws + Jf.ws_stats) + slot * kStatWords;
        const uint32_t px = 64u * held;         // this lane's pixels
#pragma unroll
        for (int b = 2; b <= 8; ++b) {
            const uint32_t v = wave_scan_incl(px - thermo_ge(C, b, kHiPlanes));   // lane 63: the wave's Z_b
            if (lane == 63 && v) atomicAdd(&st[b - 2], v);
        }
        thermo_clear(C);
        held = 0;
    };

    // STATS: one barrier per iteration keeps the waves of a workgroup on the
    // same four tiles, so both halves of each 128-byte line are requested
    // close together (waves that drift apart make the L2 fetch lines twice)
    const uint32_t nit = r1 > r0 ? (r1 - r0 + kW - 1) / kW : 0u;   // uniform in the workgroup
    for (uint32_t it = 0; it < nit; ++it) {
        const uint32_t u = r0 + it * kW + (uint32_t)wave;
        if (STATS) __syncthreads();
        if (u >= r1) continue;                 // the tail of the last range
        uint4 p[4];
        uint32_t left = 0;
        if (STATS) {
#pragma unroll
            for (int i = 0; i < 4; ++i) p[i] = p_n[i];
            left = left_n;
            fetch(u + kW < r1 ? u + kW : u);    // the last tile reloads itself: loads always issued
        }
        const int j = (int)uni((uint32_t)find_job<UNIT_TILE>(jobs, njobs, u, ujob));
        const Job &J = jobs[j];
        const uint64_t nz = job_nonce(J);
        const uint32_t t = u - J.ubase[UNIT_TILE];
        const int ty = (int)(t / (uint32_t)J.tiles_x), tx = (int)(t % (uint32_t)J.tiles_x);
        tile_codes<KS>(J, nz, t, ty, tx, q, g, lane, ws);

        if (STATS) {
            if (!DYN && (j != cur_j || held == kHeldMax)) {
                flush(cur_j);
                cur_j = j;
            }
            uint32_t y[16];
            tile_thermo(p, left, tx, g, y);
            thermo_add(C, y);
            ++held;
            if (DYN) {
                // this tile's Z_b, b = 2..7 (64 pixels per lane), its b_t and capacity
                uint32_t best_b, best_z, best_s;
                thermo_tile_b(C, best_b, best_z, best_s);
                if (lane == 0) {
                    ws[J.ws_btab + t] = (uint8_t)best_b;
                    unsigned long long *acc = reinterpret_cast<unsigned long long *>(ws + stat_dyn_acc(J));
                    if (best_z) {
                        atomicAdd(acc, (unsigned long long)best_z);
                        atomicAdd(acc + 1, (unsigned long long)best_s);
                    }
                }
                thermo_clear(C);
                held = 0;
            }
        }
    }
    if (!DYN) flush(cur_j);
}

// Clears the statistics record of every tiled image before k_tile_prep<true>
// adds into it (images on the per-pixel path clear their own).
// Thread (j, y) clears slots y, y + gridDim.y, ... of image j (two 16-byte
// stores per slot).
__global__ void k_stats_zero(const Job *__restrict__ jobs, int njobs, uint8_t *__restrict__ ws) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= njobs || !jobs[j].fast) return;
    uint4 *st = reinterpret_cast<uint4 *>(ws + jobs[j].ws_stats);
    const uint32_t ns = stat_slots(jobs[j]);
    for (uint32_t q = blockIdx.y; q < ns; q += gridDim.y) {
        st[2 * q] = make_uint4(0, 0, 0, 0);
        st[2 * q + 1] = make_uint4(0, 0, 0, 0);
    }
    if (jobs[j].method == RDHEI_DEMR && blockIdx.y == 0)
        *reinterpret_cast<uint4 *>(ws + stat_dyn_acc(jobs[j])) = make_uint4(0, 0, 0, 0);
}

// ----------------------------------------------------------------------------
// One workgroup per image: sums the label histogram, picks the optimal b
// (Sec. III-A optimal-b equation: argmax of b*Z_b, smallest b on ties), writes
// the public meta record, and builds the rotation codes of the levels above
// the tile from the tile sums (a level-m block code is the sum of its four
// children mod 4 because block sums nest).
// ----------------------------------------------------------------------------
// Optimal b (Sec. III-A: argmax of b*Z_b, smallest b on ties) and the public
// meta record from an image's statistics record (words 0..6: Z_b for b =
// 2..8, the pixels with lambda >= b); Z also stays in the workspace as 64-bit
// values for the host (LMR candidates).
// Called by the 64 lanes of one wave: lane q reads counter slot q (at most 64
// slots), a shuffle tree adds the slots up, lane 0 writes the results.
__device__ void finish_stats(const Job &J, uint8_t *ws) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t *st = reinterpret_cast<const uint32_t *>(ws + J.ws_stats);
    const uint32_t ns = stat_slots(J);
    unsigned long long v[7];
#pragma unroll
    for (int k = 0; k < 7; ++k) v[k] = lane < ns ? st[lane * kStatWords + (uint32_t)k] : 0ull;
#pragma unroll
    for (int k = 0; k < 7; ++k)
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_down(v[k], off, 64);
    if (lane != 0) return;
    int64_t Z[9];
    for (int b = 2; b <= 8; ++b) Z[b] = (int64_t)v[b - 2];
    int64_t *zout = reinterpret_cast<int64_t *>(ws + stat_z_offset(J));
    for (int b = 2; b <= 8; ++b) zout[b - 2] = Z[b];
    if (J.method == RDHEI_DEMR) {
        const unsigned long long *acc = reinterpret_cast<const unsigned long long *>(ws + stat_dyn_acc(J));
        rdhei_meta m;
        m.height = J.M; m.width = J.N; m.method = RDHEI_DEMR; m.b = 0;
        m.min_level = J.min_level; m.max_level = J.max_level;
        m.redundant = (int64_t)acc[0]; m.capacity_bits = (int64_t)acc[1];
        m.map_bits = 0; m.status = RDHEI_OK;
        m.reserved = 0;
        m.nonce = J.nonce;
        *J.meta = m;
    } else if (J.method == RDHEI_EMR) {
        int best = 2;
        for (int b = 3; b <= 7; ++b)
            if ((int64_t)b * Z[b] > (int64_t)best * Z[best]) best = b;
        rdhei_meta m;
        m.height = J.M; m.width = J.N; m.method = RDHEI_EMR; m.b = best;
        m.min_level = J.min_level; m.max_level = J.max_level;
        m.redundant = Z[best]; m.capacity_bits = (int64_t)best * Z[best];
        m.map_bits = 0; m.status = RDHEI_OK;
        m.reserved = 0;
        m.nonce = J.nonce;
        *J.meta = m;
    }
}

// Upper pyramid levels lo..max_level, level by level, by one workgroup of NT
// threads.
template <int NT = kThreads>
__device__ void upper_levels(const Job &J, uint8_t *pyr, int lo) {
    const int tid = threadIdx.x;
    for (int m = lo; m <= J.max_level; ++m) {
        __syncthreads();
        const uint32_t gy = (uint32_t)(J.M >> m), gx = (uint32_t)(J.N >> m);
        const uint32_t cx = (uint32_t)(J.N >> (m - 1));
        const uint8_t *child = pyr + pyr_off(J.M, J.N, m - 1);
        uint8_t *cur = pyr + pyr_off(J.M, J.N, m);
        for (uint32_t q = tid; q < gy * gx; q += NT) {
            const uint32_t Y = q / gx, X = q % gx;
            const uint8_t *a = child + (2 * Y) * cx + 2 * X;
            cur[q] = (uint8_t)((a[0] + a[1] + a[cx] + a[cx + 1]) & 3);
        }
    }
    __syncthreads();
}

// Upper pyramid levels and tile map of image J by one workgroup of NT threads
// (the per-image kernels; the tile sums are in the pyramid); ends with a
// barrier.
template <int NT>
__device__ void image_pyramid_tmap(const Job &J, uint8_t *ws) {
    uint8_t *pyr = ws + J.ws_pyr;
    upper_levels<NT>(J, pyr, kTileLog + 1);
    uint32_t *tmap = reinterpret_cast<uint32_t *>(ws + J.ws_tmap);
    const uint32_t tiles_x = (uint32_t)J.tiles_x, ntiles = tiles_x * (uint32_t)J.tiles_y;
    for (uint32_t t = threadIdx.x; t < ntiles; t += NT) {
        int dy, dx;
        uint32_t turns;
        upper_walk(J, pyr, (int)(t / tiles_x), (int)(t % tiles_x), dy, dx, turns);
        tmap[t] = tmap_pack(dy, dx, turns);
    }
    __syncthreads();
}

// ----------------------------------------------------------------------------
// One workgroup per image: picks the optimal b from the image's counts,
// writes the public meta record, and builds the rotation codes of the levels
// above the tile from the tile sums (a level-m block code is the sum of its
// four children mod 4 because block sums nest), then the tile map.  Images of
// kBigTiles tiles or more are finalised across many workgroups instead
// (k_fin_blocks, k_fin_top, k_fin_tmap).
// ----------------------------------------------------------------------------
template <bool STATS>
__global__ __launch_bounds__(kThreads) void k_finalize(const Job *__restrict__ jobs, int njobs,
                                                        uint8_t *__restrict__ ws) {
    const int tid = threadIdx.x;
    for (int j = blockIdx.x; j < njobs; j += gridDim.x) {
        const Job &J = jobs[j];
        if (J.fast && (uint32_t)(J.tiles_x * J.tiles_y) >= kBigTiles) continue;   // uniform per workgroup
        if (STATS && tid < 64) finish_stats(J, ws);                            // wave 0
        if (J.fast) {
            uint8_t *pyr = ws + J.ws_pyr;
            upper_levels(J, pyr, kTileLog + 1);     // level kTileLog holds the tile sums
            // where every tile goes (levels above the tile move tiles rigidly)
            uint32_t *tmap = reinterpret_cast<uint32_t *>(ws + J.ws_tmap);
            const uint32_t ntiles = (uint32_t)(J.tiles_x * J.tiles_y);
            for (uint32_t q = tid; q < ntiles; q += kThreads) {
                int dy, dx;
                uint32_t turns;
                upper_walk(J, pyr, (int)(q / (uint32_t)J.tiles_x), (int)(q % (uint32_t)J.tiles_x), dy, dx, turns);
                tmap[q] = tmap_pack(dy, dx, turns);
            }
        }
        __syncthreads();
    }
}

// Large image, step 1: one workgroup per 16 x 16 block of tiles builds
// pyramid levels kTileLog+1..kTileLog+4 inside the block.
__global__ __launch_bounds__(kThreads) void k_fin_blocks(const Job *__restrict__ jobs, int j, uint8_t *__restrict__ ws) {
    __shared__ uint8_t lv[2][kFinBlock * kFinBlock];
    const Job &J = jobs[j];
    const int tid = threadIdx.x;
    const uint32_t nbx = (uint32_t)(J.tiles_x + kFinBlock - 1) / kFinBlock;
    const uint32_t BY = blockIdx.x / nbx, BX = blockIdx.x % nbx;
    const uint32_t ty = BY * kFinBlock + (uint32_t)(tid / kFinBlock), tx = BX * kFinBlock + (uint32_t)(tid % kFinBlock);
    const bool in = ty < (uint32_t)J.tiles_y && tx < (uint32_t)J.tiles_x;
    uint8_t *pyr = ws + J.ws_pyr;
    lv[0][tid] = in ? pyr[ty * (uint32_t)J.tiles_x + tx] : (uint8_t)0;
    int cur = 0;
    uint32_t side = kFinBlock;
    for (int m = kTileLog + 1; m <= kTileLog + 4; ++m) {
        __syncthreads();
        if (m > J.max_level) break;                  // uniform
        side >>= 1;
        const uint32_t gy = (uint32_t)(J.M >> m), gx = (uint32_t)(J.N >> m);
        if ((uint32_t)tid < side * side) {
            const uint32_t y = (uint32_t)tid / side, x = (uint32_t)tid % side;
            const uint8_t *a = lv[cur] + (2 * y) * (2 * side) + 2 * x;
            const uint8_t v = (uint8_t)((a[0] + a[1] + a[2 * side] + a[2 * side + 1]) & 3);
            lv[cur ^ 1][y * side + x] = v;
            const uint32_t Y = BY * side + y, X = BX * side + x;
            if (Y < gy && X < gx) pyr[pyr_off(J.M, J.N, m) + (uint64_t)Y * gx + X] = v;
        }
        cur ^= 1;
    }
}

// Large image, step 2 (one workgroup): the optimal b and meta, and the
// pyramid levels above kTileLog+4.
template <bool STATS>
__global__ __launch_bounds__(kThreads) void k_fin_top(const Job *__restrict__ jobs, int j, uint8_t *__restrict__ ws) {
    const Job &J = jobs[j];
    if (STATS && threadIdx.x < 64) finish_stats(J, ws);                        // wave 0
    upper_levels(J, ws + J.ws_pyr, kTileLog + 5);
}

// Large image, step 3: the tile map, one thread per tile.
__global__ __launch_bounds__(kThreads) void k_fin_tmap(const Job *__restrict__ jobs, int j, uint8_t *__restrict__ ws) {
    const Job &J = jobs[j];
    const uint32_t q = blockIdx.x * kThreads + threadIdx.x;
    const uint32_t ntiles = (uint32_t)(J.tiles_x * J.tiles_y);
    if (q >= ntiles) return;
    int dy, dx;
    uint32_t turns;
    upper_walk(J, ws + J.ws_pyr, (int)(q / (uint32_t)J.tiles_x), (int)(q % (uint32_t)J.tiles_x), dy, dx, turns);
    reinterpret_cast<uint32_t *>(ws + J.ws_tmap)[q] = tmap_pack(dy, dx, turns);
}

// Encryption of one tile by its wave (Sec. III-A encoding): label each pixel
// (l = 1 unless its b MSBs match its left neighbour's; column 0 always 1), move
// its 4x4 block whole to the block's rotated position (tile map entry tm, the
// tile's code record rc), XOR with the keystream at the destination and put l
// in the LSB.  LMR: full-byte XOR, then bit 7 of raster pixel p takes stream
// bit p; LMR_MAPS: the rotated location map and first-MSB map as bit planes.
// halo: the byte left of each of the lane's four rows (lanes g = 0); rec, dst:
// the wave's LDS record and tile buffers.
template <int MODE, int KS>
__device__ __forceinline__ void encrypt_tile(const Job &J, uint64_t nz, const uint4 p[4], uint32_t halo, int b, uint32_t tm,
                                             uint4 rc, int tx, uint8_t *rec, uint8_t *dst, const uint32_t *ptab, int q,
                                             int g, int lane) {
    constexpr bool kEmrLike = MODE == ENC_EMR || MODE == ENC_DEMR;      // the map in the LSB plane
    int dy, dx;
    uint32_t up;
    tmap_unpack(tm, dy, dx, up);
    // dynamic b: the tile's b into the table, at the tile's encrypted position
    if (MODE == ENC_DEMR && lane == 0) gstore<uint8_t>(J.btab + dy * J.tiles_x + dx, (uint8_t)b);

    // labels (Sec. III-A location map): l = 1 unless the b MSBs equal the left neighbour's
    uint32_t o[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint32_t w[4] = {p[i].x, p[i].y, p[i].z, p[i].w};
        const uint32_t from_left = (uint32_t)__builtin_amdgcn_mov_dpp((int)(p[i].w >> 24), 0x90, 0xF, 0xF, false);
        if (MODE == ENC_LMR) {
#pragma unroll
            for (int k = 0; k < 4; ++k) o[i][k] = w[k];
            continue;
        }
        const uint32_t left = g > 0 ? from_left : (halo >> (8 * i)) & 0xFFu;
        // the b MSBs of a byte below bit 7 (b >= 1, so bit 7 is always among them)
        const uint32_t topm7 = ((0x7Fu << (8 - b)) & 0x7Fu) * 0x01010101u;
        const uint32_t lw[4] = {(w[0] << 8) | left, __builtin_amdgcn_alignbit(w[1], w[0], 24),
                                __builtin_amdgcn_alignbit(w[2], w[1], 24), __builtin_amdgcn_alignbit(w[3], w[2], 24)};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            // x = pixel XOR left neighbour; per byte, r = its b MSBs below bit 7:
            // r + 0x7F reaches bit 7 exactly when r != 0 and never carries into
            // the next byte, so bit 7 of t says the b MSBs differ
            const uint32_t x = w[k] ^ lw[k];
            const uint32_t t = ((x & topm7) + 0x7F7F7F7Fu) | x;
            uint32_t lbl = (t >> 7) & 0x01010101u;                                        // l per byte
            if (k == 0 && tx == 0 && g == 0) lbl |= 1u;                                  // column 0
            if (kEmrLike) o[i][k] = (w[k] & 0xFEFEFEFEu) | lbl;
            else o[i][k] = (lbl << 1) | ((w[k] >> 7) & 0x01010101u);                     // l<<1 | eta
        }
    }
    if (lane < kCodeRecord / 16) reinterpret_cast<uint4 *>(rec)[lane] = rc;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    // this lane's four 4x4 blocks (row q, columns 4g..4g+3) go whole to their destinations
    uint32_t ny[4], nx[4], R1[4], k0[4], k1[4];
    block_turns4(rec, J.min_level, up, (uint32_t)q, (uint32_t)g, ny, nx, R1, k0, k1);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t w[4] = {o[0][k], o[1][k], o[2][k], o[3][k]};
        uint32_t ob[4];
        block_forward(ptab, R1[k], k0[k], k1[k], w, ob);
        *reinterpret_cast<uint4 *>(dst + blk_addr(ny[k], nx[k])) = make_uint4(ob[0], ob[1], ob[2], ob[3]);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    // the lane's destination blocks (q, 4g + k): row i of the strip is row i of each
    uint4 db[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) db[k] = *reinterpret_cast<const uint4 *>(dst + blk_addr((uint32_t)q, (uint32_t)(4 * g + k)));
    const uint32_t rows[4][4] = {{db[0].x, db[1].x, db[2].x, db[3].x}, {db[0].y, db[1].y, db[2].y, db[3].y},
                                 {db[0].z, db[1].z, db[2].z, db[3].z}, {db[0].w, db[1].w, db[2].w, db[3].w}};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint4 qv = make_uint4(rows[i][0], rows[i][1], rows[i][2], rows[i][3]);
        const uint64_t didx = (uint64_t)(dy * kTile + 4 * q + i) * (uint64_t)J.N + (uint64_t)(dx * kTile + 16 * g);
        if (MODE == ENC_LMR_MAPS) {
            // bit planes, MSB-first: pixel didx+k -> byte (didx+k)/8, bit 7-(k%8)
            const uint32_t qq[4] = {qv.x, qv.y, qv.z, qv.w};
            uint32_t lb = 0, eb = 0;
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const uint32_t v = (qq[k >> 2] >> (8 * (k & 3))) & 3u;
                const int pos = (k < 8) ? (7 - k) : (23 - k);   // little-endian u16 of two MSB-first bytes
                lb |= ((v >> 1) & 1u) << pos;
                eb |= (v & 1u) << pos;
            }
            gstore<uint16_t>(J.out + (didx >> 3), (uint16_t)lb);
            gstore<uint16_t>(J.msg + (didx >> 3), (uint16_t)eb);
        } else {
            const U4 sk = stream_block_quad<KS>(J.key, nz, kDomainImage, didx >> 4);
            uint4 e;
            if (kEmrLike) {
                e = make_uint4(qv.x ^ (sk.x & 0xFEFEFEFEu), qv.y ^ (sk.y & 0xFEFEFEFEu),
                               qv.z ^ (sk.z & 0xFEFEFEFEu), qv.w ^ (sk.w & 0xFEFEFEFEu));
            } else {
                e = make_uint4(qv.x ^ sk.x, qv.y ^ sk.y, qv.z ^ sk.z, qv.w ^ sk.w);
                if ((int64_t)didx < J.stream_bits) {
                    // 16 stream bits for pixels didx..didx+15 (didx is a multiple of 16)
                    const uint32_t sb = ((uint32_t)J.stream[didx >> 3] << 8) | J.stream[(didx >> 3) + 1];
                    uint32_t ew[4] = {e.x, e.y, e.z, e.w};
#pragma unroll
                    for (int k = 0; k < 16; ++k) {
                        if ((int64_t)didx + k < J.stream_bits) {
                            const uint32_t bit = (sb >> (15 - k)) & 1u;
                            ew[k >> 2] = (ew[k >> 2] & ~(0x80u << (8 * (k & 3)))) | (bit << (8 * (k & 3) + 7));
                        }
                    }
                    e = make_uint4(ew[0], ew[1], ew[2], ew[3]);
                }
            }
            gstore<uint4>(J.out + didx, e);
        }
    }
}

// Work unit u of a quad launch: quads c0 .. c0 + nc - 1 of band pair p (tile
// rows 2p, 2p + 1) of image j; band pairs are cut into ns segments of at most
// J.qseg quads, s is this one.  Wave-uniform.
struct QSeg {
    int j, p, c0, nc, s, ns;
};
__device__ __forceinline__ QSeg qseg_of(const Job *jobs, int njobs, const uint32_t *ujob, uint32_t u) {
    QSeg r;
    r.j = (int)uni((uint32_t)find_job<UNIT_QROW>(jobs, njobs, u, ujob));
    const Job &J = jobs[r.j];
    const uint32_t qs = (uint32_t)J.qseg;
    const uint32_t nq = (uint32_t)((J.tiles_x + 1) >> 1), ns = (nq + qs - 1) / qs;
    const uint32_t v = u - J.ubase[UNIT_QROW];
    r.p = (int)(v / ns);
    r.s = (int)(v % ns);
    r.ns = (int)ns;
    r.c0 = r.s * (int)qs;
    r.nc = (int)(nq - (uint32_t)r.c0 < qs ? nq - (uint32_t)r.c0 : qs);
    return r;
}

// ----------------------------------------------------------------------------
// Encryption (Sec. III-A encoding): label each pixel (l = 1 unless its b MSBs
// match its left neighbour's; column 0 always 1), move it to its rotated
// position (closed form of the level-by-level block turns), XOR with the
// keystream at the destination, and put l in the LSB.
// LMR: full-byte XOR, then bit 7 of raster pixel p takes stream bit p.
// LMR_MAPS: instead of the image, write the rotated location map and
// first-MSB map as bit planes (for the host coder).
//
// Work goes by 2x2 tile quads of a band pair (tile rows 2p, 2p + 1), left to
// right, one wave per tile.  The four tiles of a full quad form a level-7
// block, which moves whole: its four destination tiles form one 128 x 128
// block, so the quad's reads and writes both cover whole 128-byte lines.  The
// byte left of each tile row comes from the wave holding the left tile, by
// LDS (same quad, or the right tile of the previous quad).
// ----------------------------------------------------------------------------
template <int MODE, int KS>
__global__ __launch_bounds__(kThreads) void k_encrypt_quad(const Job *__restrict__ jobs, int njobs,
                                                            uint8_t *__restrict__ ws, uint32_t units,
                                                            const uint32_t *__restrict__ ujob) {
    constexpr int kW = kThreads / 64;
    __shared__ __align__(16) uint8_t dsts[kW][kTile * kTile];   // per wave: the destination tile, 4x4 blocks
    __shared__ __align__(16) uint8_t recs[kW][kCodeRecord];     // per wave: the tile's code record
    __shared__ __align__(16) uint32_t ptab[perm4::kWords];
    __shared__ __align__(16) uint32_t edge[2][kW][kTile / 4];   // per tile: column 63, four rows per word
    const int lane = threadIdx.x & 63, wave = (int)uni(threadIdx.x >> 6);   // wave-uniform
    const int q = lane >> 2, g = lane & 3;                       // rows 4q..4q+3, columns 16g..16g+15
    const int side = wave & 1, half = wave >> 1;                 // this wave's tile in the quad
    uint8_t *dst = dsts[wave];
    uint8_t *rec = recs[wave];
    stage_perm_tables(ptab, (int)threadIdx.x);
    __syncthreads();

    uint32_t r0, r1;
    unit_range(units, r0, r1);
    auto seg_of = [&](uint32_t u) { return qseg_of(jobs, njobs, ujob, u); };
    uint4 p_n[4], rc_n = make_uint4(0, 0, 0, 0);
    uint32_t b_n = 0, st_n = 0, tm_n = 0, halo_n = 0;
    // loads of this wave's tile of quad c of segment S; a tile outside the image
    // loads the nearest one inside instead (unused): no branch, no register copies
    auto fetch = [&](const QSeg &S, int c) {
        const Job &J = jobs[S.j];
        const int ty = min(2 * S.p + half, J.tiles_y - 1), tx = min(2 * (S.c0 + c) + side, J.tiles_x - 1);
        const uint32_t t = (uint32_t)(ty * J.tiles_x + tx);
        const uint8_t *row = J.in + (uint64_t)(ty * kTile + 4 * q) * (uint64_t)J.N + (uint64_t)(tx * kTile + 16 * g);
#pragma unroll
        for (int i = 0; i < 4; ++i) p_n[i] = gload<uint4>(row + (uint64_t)i * J.N);
        if (side == 0 && c == 0 && tx > 0 && g == 0) {   // left column of the segment, from memory
            uint32_t hb = 0;
#pragma unroll
            for (int i = 0; i < 4; ++i) hb |= (uint32_t)gload<uint8_t>(row + (uint64_t)i * J.N - 1) << (8 * i);
            halo_n = hb;
        }
        rc_n = gload<uint4>(ws + J.ws_codes + (uint64_t)t * kCodeRecord + 16 * (lane % (kCodeRecord / 16)));
        b_n = MODE == ENC_DEMR ? (uint32_t)gload<uint8_t>(ws + J.ws_btab + t) : (uint32_t)gload<int32_t>(&J.meta->b);
        st_n = (uint32_t)gload<int32_t>(&J.meta->status);
        tm_n = gload<uint32_t>(ws + J.ws_tmap + 4 * (uint64_t)t);
    };

    uint32_t u = r0;
    int c = 0;
    QSeg S{0, 0, 0, 1, 0, 1};
    if (u < r1) {
        S = seg_of(u);
        fetch(S, c);
    }
    for (uint32_t it = 0; u < r1; ++it) {
        uint32_t u1 = u;
        int c1 = c + 1;
        QSeg S1 = S;
        if (c1 >= S.nc) {
            ++u1;
            c1 = 0;
            if (u1 < r1) S1 = seg_of(u1);
        }
        uint4 p[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) p[i] = p_n[i];
        const uint4 rc = rc_n;
        const uint32_t b_cur = uni(b_n), st_cur = uni(st_n), tm = uni(tm_n), halo_mem = halo_n;
        const Job &J = jobs[S.j];
        const uint64_t nz = job_nonce(J);
        const int ty = 2 * S.p + half, tx = 2 * (S.c0 + c) + side;
        const bool have = ty < J.tiles_y && tx < J.tiles_x;   // wave-uniform
        const bool first = c == 0;
        const uint32_t slot = it & 1u;
        // column 63 of the previous quad's right tile, read before this barrier: it
        // was written before the last one, and its wave writes that slot again
        // right after this one
        const uint32_t edge_prev = side ? 0u : edge[slot ^ 1u][wave + 1][q];
        // column 63 of this tile for the wave of the tile to its right
        if (have && g == 3)
            edge[slot][wave][q] = (p[0].w >> 24) | ((p[1].w >> 24) << 8) | ((p[2].w >> 24) << 16) | (p[3].w & 0xFF000000u);
        __syncthreads();
        if (u1 < r1) fetch(S1, c1);
        u = u1;
        c = c1;
        S = S1;
        if (!have) continue;                                              // uniform per wave
        constexpr bool kEmrLike = MODE == ENC_EMR || MODE == ENC_DEMR;      // the map in the LSB plane
        if (kEmrLike && st_cur != (uint32_t)RDHEI_OK) continue;           // uniform per wave
        const int b = J.fixed_b > 0 ? J.fixed_b : (int)b_cur;
        // the byte left of rows 4q..4q+3 of this tile (column 0 of the image has none)
        const uint32_t halo = side ? edge[slot][wave - 1][q]
                                   : (tx == 0 ? 0u : (first ? halo_mem : edge_prev));
        encrypt_tile<MODE, KS>(J, nz, p, halo, b, tm, rc, tx, rec, dst, ptab, q, g, lane);
    }
}

// ----------------------------------------------------------------------------
// Encryption of whole small images, one workgroup of NW waves per image: the
// same arithmetic as k_tile_prep<true> -> k_finalize<true> -> k_encrypt_quad
// (Sec. III-A encoding), in three phases separated by workgroup barriers.
//  1. Tiles are dealt to the waves in turn: rotation codes and label counts
//     (the counts meet in LDS instead of global counter slots); the waves
//     run free until the phase ends.
//  2. Optimal b and the meta record, the upper pyramid levels, the tile map.
//  3. NW/4 band pairs side by side, four waves (one 2x2 quad) each, walking
//     their quads left to right; the byte left of each tile row passes through
//     LDS as in k_encrypt_quad.
// Phase 3 reads the image a second time soon after phase 1 read it (past L2,
// so from the device's last-level cache or HBM), and one launch replaces
// four.  The phases of the workgroups on a CU interleave, so vector-bound code
// and count work overlaps memory-bound encryption.  Images must be on the tiled path with at
// most kImageWgMaxTiles tiles, method EMR or DEMR.
// ----------------------------------------------------------------------------
template <int MODE, int KS, int NW>
__global__ __launch_bounds__(NW * 64) void k_encrypt_image(const Job *__restrict__ jobs, int njobs,
                                                           uint8_t *__restrict__ ws) {
    static_assert(NW % 4 == 0, "four waves per quad");
    static_assert(MODE == ENC_EMR || MODE == ENC_DEMR, "EMR-style encryption only");
    constexpr bool DYN = MODE == ENC_DEMR;
    constexpr int kG = NW / 4;                                    // band pairs side by side
    __shared__ __align__(16) uint8_t dsts[NW][kTile * kTile];    // per wave: the destination tile
    __shared__ __align__(16) uint8_t recs[NW][kCodeRecord];      // per wave: the tile's code record
    __shared__ __align__(16) uint32_t ptab[perm4::kWords];
    __shared__ __align__(16) uint32_t edge[2][NW][kTile / 4];    // per tile: column 63, four rows per word
    __shared__ uint32_t zc[8];                                    // Z_b, b = 2..8
    __shared__ unsigned long long dacc[2];                        // DEMR: redundant pixels, capacity
    __shared__ int32_t sb;                                        // the image's b
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = (int)uni((uint32_t)tid >> 6);   // wave-uniform
    const int q = lane >> 2, g = lane & 3;
    stage_perm_tables(ptab, tid);
    uint8_t *dst = dsts[wave];
    uint8_t *rec = recs[wave];

    for (int j = blockIdx.x; j < njobs; j += gridDim.x) {
        const Job &J = jobs[j];
        const uint64_t nz = job_nonce(J);
        const uint32_t tiles_x = (uint32_t)J.tiles_x, ntiles = tiles_x * (uint32_t)J.tiles_y;
        if (tid < 8) zc[tid] = 0;
        if (tid < 2) dacc[tid] = 0;

        // ---- 1. codes and counts: tile t = it * NW + wave
        Thermo C;
        thermo_clear(C);
        uint32_t held = 0;
        auto flush = [&]() {
#pragma unroll
            for (int b = 2; b <= 8; ++b) {
                const uint32_t v = wave_scan_incl(64u * held - thermo_ge(C, b, kHiPlanes));
                if (lane == 63 && v) atomicAdd(&zc[b - 2], v);
            }
            thermo_clear(C);
            held = 0;
        };
        // no barrier per iteration (unlike k_tile_prep): the image is read
        // again in phase 3 anyway, and free-running waves measured faster.
        // No prefetch either: the tile's loads are issued first and the
        // keystream codes, which do not need them, run while they are in
        // flight (measured faster than carrying the next tile in registers)
        const uint32_t nit = (ntiles + NW - 1) / NW;
        __syncthreads();                                              // the counters are cleared
        for (uint32_t it = 0; it < nit; ++it) {
            const uint32_t t = it * NW + (uint32_t)wave;
            if (t >= ntiles) continue;
            const int ty = (int)(t / tiles_x), tx = (int)(t % tiles_x);
            uint4 p[4];
            uint32_t left;
            tile_load(J, ty, tx, q, g, p, left);
            tile_codes<KS>(J, nz, t, ty, tx, q, g, lane, ws);
            if (!DYN && held == kHeldMax) flush();
            uint32_t y[16];
            tile_thermo(p, left, tx, g, y);
            thermo_add(C, y);
            ++held;
            if (DYN) {
                uint32_t best_b, best_z, best_s;
                thermo_tile_b(C, best_b, best_z, best_s);
                if (lane == 0) {
                    ws[J.ws_btab + t] = (uint8_t)best_b;
                    if (best_z) {
                        atomicAdd(&dacc[0], (unsigned long long)best_z);
                        atomicAdd(&dacc[1], (unsigned long long)best_s);
                    }
                }
                thermo_clear(C);
                held = 0;
            }
        }
        if (!DYN && held) flush();
        __syncthreads();

        // ---- 2. optimal b (Sec. III-A: argmax of b*Z_b, smallest b on ties), meta, upper levels, tile map
        if (tid == 0) {
            int64_t *zout = reinterpret_cast<int64_t *>(ws + stat_z_offset(J));
            for (int b = 2; b <= 8; ++b) zout[b - 2] = (int64_t)zc[b - 2];
            rdhei_meta m;
            m.height = J.M; m.width = J.N; m.method = J.method;
            m.min_level = J.min_level; m.max_level = J.max_level;
            m.map_bits = 0; m.status = RDHEI_OK;
            m.reserved = 0;
            m.nonce = J.nonce;
            if (DYN) {
                m.b = 0;
                m.redundant = (int64_t)dacc[0];
                m.capacity_bits = (int64_t)dacc[1];
                sb = 0;
            } else {
                int best = 2;
                for (int b = 3; b <= 7; ++b)
                    if ((int64_t)b * zc[b - 2] > (int64_t)best * zc[best - 2]) best = b;
                m.b = best;
                m.redundant = (int64_t)zc[best - 2];
                m.capacity_bits = (int64_t)best * zc[best - 2];
                sb = J.fixed_b > 0 ? J.fixed_b : best;
            }
            *J.meta = m;
        }
        image_pyramid_tmap<NW * 64>(J, ws);
        const uint32_t *tmap = reinterpret_cast<const uint32_t *>(ws + J.ws_tmap);

        // ---- 3. encryption: group gq takes band pairs gq, gq + kG, ..., their quads left to right
        const int gq = wave >> 2, side = wave & 1, half = (wave >> 1) & 1;   // this wave's tile in the quad
        const uint32_t npairs = ((uint32_t)J.tiles_y + 1) / 2, nq = (tiles_x + 1) / 2;
        const uint32_t nit3 = (npairs + kG - 1) / kG * nq;                  // uniform in the workgroup
        const int b_img = sb;
        uint4 p_n[4], rc_n = make_uint4(0, 0, 0, 0);
        uint32_t tm_n = 0, bt_n = 0;
        auto fetch3 = [&](uint32_t it) {
            // a tile outside the image loads the nearest one inside instead (its
            // values go unused): loads without a branch need no register copies
            const uint32_t pr = it / nq * kG + (uint32_t)gq, c = it % nq;
            const int ty = min((int)(2 * pr) + half, J.tiles_y - 1), tx = min((int)(2 * c) + side, J.tiles_x - 1);
            const uint32_t t = (uint32_t)ty * tiles_x + (uint32_t)tx;
            uint32_t unused;
            tile_load(J, ty, tx, q, g, p_n, unused);
            rc_n = gload<uint4>(ws + J.ws_codes + (uint64_t)t * kCodeRecord + 16 * (lane % (kCodeRecord / 16)));
            tm_n = tmap[t];
            if (DYN) bt_n = ws[J.ws_btab + t];
        };
        if (nit3) fetch3(0);
        for (uint32_t it = 0; it < nit3; ++it) {
            uint4 p[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) p[i] = p_n[i];
            const uint4 rc = rc_n;
            const uint32_t tm = uni(tm_n), bt = uni(bt_n);
            const uint32_t pr = it / nq * kG + (uint32_t)gq, c = it % nq;
            const int ty = (int)(2 * pr) + half, tx = (int)(2 * c) + side;
            const bool have = ty < J.tiles_y && tx < J.tiles_x;              // wave-uniform
            const uint32_t slot = it & 1u;
            // column 63 of the previous quad's right tile, read before this barrier
            const uint32_t edge_prev = side ? 0u : edge[slot ^ 1u][wave + 1][q];
            if (have && g == 3)
                edge[slot][wave][q] = (p[0].w >> 24) | ((p[1].w >> 24) << 8) | ((p[2].w >> 24) << 16) | (p[3].w & 0xFF000000u);
            __syncthreads();
            if (it + 1 < nit3) fetch3(it + 1);
            if (!have) continue;                                              // uniform per wave
            const int b = DYN ? (int)bt : b_img;
            // the byte left of rows 4q..4q+3 (a band pair starts at column 0, which has none)
            const uint32_t halo = side ? edge[slot][wave - 1][q] : (tx == 0 ? 0u : edge_prev);
            encrypt_tile<MODE, KS>(J, nz, p, halo, b, tm, rc, tx, rec, dst, ptab, q, g, lane);
        }
        __syncthreads();                                                      // LDS is reused by the next image
    }
}

// ----------------------------------------------------------------------------
// LMR recovery of row bands of tiles, left to right (Sec. III-B decoding with
// K1): gather each original-domain tile from its rotated position, decrypt
// with the keystream at the encrypted position, read l from the decompressed
// location map and bit 7 from the first-MSB map, then the recovery glide
// along each row: a pixel labelled 0 takes the replaceable bits of the
// nearest pixel labelled 1 to its left.  Rows carry that value across tiles.
// ----------------------------------------------------------------------------
template <int KS>
__global__ __launch_bounds__(kThreads) void k_recover_band_lmr(const Job *__restrict__ jobs, int njobs,
                                                            uint8_t *__restrict__ ws, uint32_t units,
                                                            const uint32_t *__restrict__ ujob) {
    constexpr int kRow2 = 2 * kTile + 32;   // u16 per pixel: value | l << 8
    __shared__ __align__(16) uint8_t src[kTile * kRow2];
    __shared__ __align__(16) uint8_t dst[kTile * kRow2];
    __shared__ __align__(16) uint8_t rec[kCodeRecord];
    const int tid = threadIdx.x;
    const int r = tid >> 2, g = tid & 3;
    const int by = tid >> 4, bx = tid & 15;
    const int lane = tid & 63;
    uint32_t u0, u1;
    unit_range(units, u0, u1);

    // prefetched inputs of the next (band, tile) step
    uint4 e_n = make_uint4(0, 0, 0, 0), rc_n = make_uint4(0, 0, 0, 0);
    uint32_t lb_n = 0, eb_n = 0, b_n = 0;
    auto fetch = [&](uint32_t u, int tx) {
        const Job &J = jobs[uni((uint32_t)find_job<UNIT_BAND>(jobs, njobs, u, ujob))];
        const int ty = (int)(u - J.ubase[UNIT_BAND]);
        const uint32_t t = (uint32_t)(ty * J.tiles_x + tx);
        int ey, ex;
        uint32_t up;
        tmap_unpack(reinterpret_cast<const uint32_t *>(ws + J.ws_tmap)[t], ey, ex, up);
        const uint64_t eidx = (uint64_t)(ey * kTile + r) * (uint64_t)J.N + (uint64_t)(ex * kTile + 16 * g);
        e_n = gload<uint4>(J.in + eidx);
        lb_n = __builtin_bswap16(gload<uint16_t>(J.lbits + (eidx >> 3)));
        eb_n = __builtin_bswap16(gload<uint16_t>(J.etabits + (eidx >> 3)));
        rc_n = gload<uint4>(ws + J.ws_codes + (uint64_t)t * kCodeRecord + 16 * (tid % (kCodeRecord / 16)));
        b_n = (uint32_t)gload<int32_t>(&J.meta->b);
    };
    if (u0 < u1) fetch(u0, 0);

    for (uint32_t u = u0; u < u1; ++u) {
        const Job &J = jobs[uni((uint32_t)find_job<UNIT_BAND>(jobs, njobs, u, ujob))];
        const uint64_t nz = job_nonce(J);
        const int ty = (int)(u - J.ubase[UNIT_BAND]);
        const int b = (int)uni(b_n);
        const uint32_t mask = (0xFFu << (8 - b)) & 0x7Fu;   // bits 6..8-b (bit 7 comes from the eta map)
        uint32_t carry = 0;   // replaceable bits of the last marker in this row

        for (int tx = 0; tx < J.tiles_x; ++tx) {
            const uint4 e = e_n, rc = rc_n;
            const uint32_t lbv = lb_n, ebv = eb_n;
            // next step: the next tile of this band, else the first tile of the next band
            // (the last step reloads itself, so the loads are always issued)
            const bool more = tx + 1 < J.tiles_x;
            fetch(more ? u : (u + 1 < u1 ? u + 1 : u), more ? tx + 1 : (u + 1 < u1 ? 0 : tx));
            int ey, ex;
            uint32_t up;
            tmap_unpack(reinterpret_cast<const uint32_t *>(ws + J.ws_tmap)[ty * J.tiles_x + tx], ey, ex, up);
            const uint64_t eidx = (uint64_t)(ey * kTile + r) * (uint64_t)J.N + (uint64_t)(ex * kTile + 16 * g);
            const U4 s = stream_block_quad<KS>(J.key, nz, kDomainImage, eidx >> 4);
            uint32_t D[4] = {e.x ^ s.x, e.y ^ s.y, e.z ^ s.z, e.w ^ s.w};
            uint32_t Lw[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                uint32_t lw = 0, ew = 0;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    lw |= ((lbv >> (15 - (4 * k + q))) & 1u) << (8 * q);
                    ew |= ((ebv >> (15 - (4 * k + q))) & 1u) << (8 * q + 7);
                }
                Lw[k] = lw;
                D[k] = (D[k] & 0x7F7F7F7Fu) | ew;
            }
            uint32_t il[8];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                il[2 * k] = __builtin_amdgcn_perm(Lw[k], D[k], 0x05010400u);
                il[2 * k + 1] = __builtin_amdgcn_perm(Lw[k], D[k], 0x07030602u);
            }
            uint4 *sp = reinterpret_cast<uint4 *>(src + r * kRow2 + 32 * g);
            sp[0] = make_uint4(il[0], il[1], il[2], il[3]);
            sp[1] = make_uint4(il[4], il[5], il[6], il[7]);
            if (tid < kCodeRecord / 16) reinterpret_cast<uint4 *>(rec)[tid] = rc;
            __syncthreads();

            uint32_t dmap[16];
            block_map(rec, J.min_level, up, (uint32_t)by, (uint32_t)bx, dmap);
#pragma unroll
            for (int uu = 0; uu < 4; ++uu) {
                uint32_t vals[4];
#pragma unroll
                for (int vv = 0; vv < 4; ++vv) {
                    const uint32_t d = dmap[4 * uu + vv];
                    vals[vv] = *reinterpret_cast<const uint16_t *>(src + (d >> 8) * kRow2 + 2 * (d & 0xFFu));
                }
                *reinterpret_cast<uint2 *>(dst + (4 * by + uu) * kRow2 + 8 * bx) =
                    make_uint2(vals[0] | (vals[1] << 16), vals[2] | (vals[3] << 16));
            }
            __syncthreads();

            const uint4 *rp = reinterpret_cast<const uint4 *>(dst + r * kRow2 + 32 * g);
            const uint4 a0 = rp[0], a1 = rp[1];
            const uint32_t pk[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
            // segment summary: does it hold a marker, and the last marker's bits
            uint32_t has = 0, last = 0;
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const uint32_t v = (pk[k >> 1] >> (16 * (k & 1))) & 0xFFFFu;
                const bool marker = ((v >> 8) & 1u) || (tx == 0 && g == 0 && k == 0);
                if (marker) { has = 1; last = v & mask; }
            }
            // carry-in from the nearest segment to the left in this row
            uint32_t cin = carry, found = 0;
#pragma unroll
            for (int d = 1; d <= 3; ++d) {
                const uint32_t h2 = __shfl(has, (lane - d) & 63, 64);
                const uint32_t l2 = __shfl(last, (lane - d) & 63, 64);
                if (!found && d <= g && h2) { cin = l2; found = 1; }
            }
            // new row carry: last marker of the whole row so far
            uint32_t rc2 = carry;
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                const uint32_t h2 = __shfl(has, (lane & ~3) | d, 64);
                const uint32_t l2 = __shfl(last, (lane & ~3) | d, 64);
                if (h2) rc2 = l2;
            }
            carry = rc2;
            uint32_t outw[4] = {0, 0, 0, 0};
            uint32_t cur = cin;
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const uint32_t v = (pk[k >> 1] >> (16 * (k & 1))) & 0xFFFFu;
                const bool marker = ((v >> 8) & 1u) || (tx == 0 && g == 0 && k == 0);
                uint32_t px = v & 0xFFu;
                if (marker) cur = px & mask;
                else px = (px & ~mask) | cur;
                outw[k >> 2] |= px << (8 * (k & 3));
            }
            const uint64_t oidx = (uint64_t)(ty * kTile + r) * (uint64_t)J.N + (uint64_t)(tx * kTile + 16 * g);
            gstore<uint4>(J.out + oidx, make_uint4(outw[0], outw[1], outw[2], outw[3]));
        }
    }
}

// ----------------------------------------------------------------------------
// EMR recovery by quads: the 2x2 tiles of tile rows 2p, 2p+1 and tile columns
// 2c, 2c+1, one wave per tile, quads of a band pair left to right.  The four
// tiles of a full quad form a level-7 block, so their encrypted data is one
// 128 x 128 block (whole 128-byte lines), read by the four waves together.
//
// Each wave decrypts its encrypted tile (keystream at the encrypted position)
// into LDS as 4x4 blocks (pixels and labels l = LSB), then each lane gathers
// its own four original blocks and turns them back with one composed permute
// per row.  The glide (a pixel labelled 0 takes the replaceable bits of the
// nearest pixel labelled 1 to its left) is one permute per 4-pixel word,
// selected by the word's label pattern; values cross lanes by a quad scan
// and cross tiles through LDS (left tile of a row -> right tile -> next quad),
// with one workgroup barrier per quad.
// ----------------------------------------------------------------------------

static __constant__ perm4::InvTables kInvTables = perm4::kInvTables;
static __constant__ glide4::Tables kGlideTables = glide4::kTables;

// DYN (dynamic b, RDHEI_DEMR): each tile has its own b (from the tile table,
// at the tile's encrypted position) and a pixel labelled 0 takes the top b
// bits of its restored left neighbour, so what crosses a tile border is the
// restored last pixel of the row (last labelled value in the tile's replaceable
// bits, decrypted bits below), not the last labelled value.
// IMG: one workgroup per image (grid-stride over the images): the keystream
// code pyramid of its tiles (as k_tile_prep<false>), the upper levels and
// tile map (as k_finalize<false>), then its quads as below; every band pair
// is one segment (Job::qseg covers it), so no row fix-up follows.  The
// workgroups on a CU are in different phases, so the vector-bound pyramid of
// some images overlaps the memory-bound recovery of others.
// (At most 128 VGPRs: four waves per SIMD, which is what the LDS allows.)
template <int KS, bool DYN = false, bool IMG = false>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_recover_quad_emr(
    const Job *__restrict__ jobs, int njobs, uint8_t *__restrict__ ws, uint32_t units, const uint32_t *__restrict__ ujob) {
    constexpr int kW = kThreads / 64;
    __shared__ __align__(16) uint8_t dts[kW][kTile * kTile];   // per wave: decrypted tile, 4x4 blocks
    __shared__ __align__(16) uint8_t lbs[kW][kTile * kTile];   // per wave: labels, same layout
    __shared__ __align__(16) uint8_t recs[kW][kCodeRecord];    // per wave: the tile's code record
    __shared__ __align__(16) uint32_t itab[perm4::kInvWords];
    __shared__ __align__(16) uint32_t gtab[glide4::kWords];
    // per tile row: last labelled value | 0x100 (0: none), and in bits 9..15
    // the column of its first labelled pixel (64: none; segmented images only)
    __shared__ __align__(8) uint16_t sums[2][kW][kTile];
    __shared__ __align__(8) uint16_t carry[2][2][kTile];       // per band half: carry into the next quad
    __shared__ __align__(4) uint8_t lastpx[DYN ? 2 : 1][kW][kTile];   // DYN: decrypted column 63 of each tile row
    __shared__ uint32_t tileb[DYN ? 2 : 1][kW];                       // DYN: each wave's tile b
    const int lane = threadIdx.x & 63, wave = (int)uni(threadIdx.x >> 6);   // wave-uniform
    const int q = lane >> 2, g = lane & 3;                      // rows 4q..4q+3, columns 16g..16g+15
    const int side = wave & 1, half = wave >> 1;                // this wave's tile in the quad
    uint8_t *dt = dts[wave];
    uint8_t *lb = lbs[wave];
    uint8_t *rec = recs[wave];
    for (int i = (int)threadIdx.x; i < perm4::kInvWords; i += kThreads)
        itab[i] = reinterpret_cast<const uint32_t *>(&kInvTables)[i];
    if (threadIdx.x < glide4::kWords) gtab[threadIdx.x] = kGlideTables.fill_sel[threadIdx.x];
    __syncthreads();

    uint32_t r0 = 0, r1 = 0;
    if (!IMG) unit_range(units, r0, r1);
    // quad positions (unit u, quad c of its segment S), wave-uniform
    struct Pos {
        uint32_t u;
        int c;
        QSeg S;
    };
    auto advance = [&](const Pos &P) {
        Pos n = P;
        if (n.u >= r1) return n;
        if (++n.c >= n.S.nc) {
            ++n.u;
            n.c = 0;
            if (n.u < r1) n.S = qseg_of(jobs, njobs, ujob, n.u);
        }
        return n;
    };
    // this wave's tile of a quad; false when it lies outside the image
    auto tile_of = [&](const Pos &P, int &ty, int &tx) {
        if (P.u >= r1) return false;
        const Job &J = jobs[P.S.j];
        ty = 2 * P.S.p + half;
        tx = 2 * (P.S.c0 + P.c) + side;
        return ty < J.tiles_y && tx < J.tiles_x;
    };
    // tile-map entry and b of a quad's tile (loaded an iteration before the pixels)
    auto load_tm = [&](const Pos &P, uint32_t &tm, uint32_t &bb) {
        int ty = 0, tx = 0;
        if (!tile_of(P, ty, tx)) return;
        const Job &J = jobs[P.S.j];
        tm = gload<uint32_t>(ws + J.ws_tmap + 4 * (uint64_t)(ty * J.tiles_x + tx));
        if (DYN) {
            int ey, ex;
            uint32_t up;
            tmap_unpack(uni(tm), ey, ex, up);
            bb = (uint32_t)gload<uint8_t>(J.btab + ey * J.tiles_x + ex);
        } else {
            bb = (uint32_t)gload<int32_t>(&J.meta->b);
        }
    };
    uint4 e_n[4], rc_n = make_uint4(0, 0, 0, 0);
    // Loads the pixels and code record of P's tile.  Inside the quad loop a
    // position past the range keeps the last segment, so its image is tiled:
    // a tile outside that image, and a stale tile-map entry, are clamped onto
    // the image and loaded unused, so the loads need no branch (and no
    // register copies); before the loop (CLAMP false) a missing tile loads nothing.
    auto fetch = [&](const Pos &P, uint32_t tm, auto clamp) {
        constexpr bool CLAMP = decltype(clamp)::value;
        int ty = 0, tx = 0;
        if (!CLAMP && !tile_of(P, ty, tx)) return;
        const Job &J = jobs[P.S.j];
        if (CLAMP) {
            ty = min(2 * P.S.p + half, J.tiles_y - 1);
            tx = min(2 * (P.S.c0 + P.c) + side, J.tiles_x - 1);
        }
        int ey, ex;
        uint32_t up;
        tmap_unpack(uni(tm), ey, ex, up);
        if (CLAMP) {
            ey = min(ey, J.tiles_y - 1);
            ex = min(ex, J.tiles_x - 1);
        }
        const uint8_t *src = J.in + (uint64_t)(ey * kTile + 4 * q) * (uint64_t)J.N + (uint64_t)(ex * kTile + 16 * g);
#pragma unroll
        for (int i = 0; i < 4; ++i) e_n[i] = gload<uint4>(src + (uint64_t)i * J.N);
        rc_n = gload<uint4>(ws + J.ws_codes + (uint64_t)(ty * J.tiles_x + tx) * kCodeRecord + 16 * (lane % (kCodeRecord / 16)));
    };

    // IMG: the images of this workgroup in turn, each one's quads as the units
    for (int j_img = IMG ? (int)blockIdx.x : 0;; j_img += (int)gridDim.x) {
    if (IMG) {
        if (j_img >= njobs) break;
        const Job &J = jobs[j_img];
        const uint64_t nz = job_nonce(J);
        const uint32_t tiles_x = (uint32_t)J.tiles_x, ntiles = tiles_x * (uint32_t)J.tiles_y;
        for (uint32_t t = (uint32_t)wave; t < ntiles; t += kW)
            tile_codes<KS>(J, nz, t, (int)(t / tiles_x), (int)(t % tiles_x), q, g, lane, ws);
        __syncthreads();
        image_pyramid_tmap<kThreads>(J, ws);
        r0 = J.ubase[UNIT_QROW];
        r1 = r0 + J.ucount[UNIT_QROW];
    }
    Pos cur{r0, 0, QSeg{0, 0, 0, 1, 0, 1}};
    if (r0 < r1) cur.S = qseg_of(jobs, njobs, ujob, r0);
    Pos nxt = advance(cur);
    uint32_t tm = 0, b_cur = 0, tm1 = 0, b1 = 0;
    load_tm(cur, tm, b_cur);
    fetch(cur, tm, std::false_type{});
    load_tm(nxt, tm1, b1);
    uint32_t lead[4] = {0, 0, 0, 0}, open[4] = {1, 1, 1, 1};   // left waves of segmented images

    for (uint32_t it = 0; cur.u < r1; ++it) {
        uint4 e[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) e[i] = e_n[i];
        const uint4 rc = rc_n;
        const uint32_t tm_cur = uni(tm), bq = uni(b_cur);
        // pipeline: pixels of the next quad, tile map of the one after
        fetch(nxt, tm1, std::true_type{});
        const Pos nn = advance(nxt);
        tm = tm1;
        b_cur = b1;
        load_tm(nn, tm1, b1);

        int ty = 0, tx = 0;
        const bool have = tile_of(cur, ty, tx);   // wave-uniform
        const Job &J = jobs[cur.S.j];
        const uint64_t nz = job_nonce(J);
        const bool first = cur.c == 0, last = cur.c == cur.S.nc - 1;
        const bool segd = !IMG && cur.S.ns > 1;   // rows continue in other segments (fixed up afterwards)
        const bool right_in = 2 * (cur.S.c0 + cur.c) + 1 < J.tiles_x;
        const uint32_t slot = it & 1u;
        uint32_t Do[4][4], sel[4][4], excl[4], tsum[4], fcol[4];
        if (have) {
            int ey, ex;
            uint32_t up;
            tmap_unpack(tm_cur, ey, ex, up);
            // decrypt at the encrypted position; blocks (q, 4g + k) of the encrypted tile
            const uint64_t e0 = (uint64_t)(ey * kTile + 4 * q) * (uint64_t)J.N + (uint64_t)(ex * kTile + 16 * g);
            uint32_t dw[4][4], lw[4][4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const U4 s = stream_block_quad<KS>(J.key, nz, kDomainImage, (e0 + (uint64_t)i * J.N) >> 4);
                const uint32_t ew[4] = {e[i].x, e[i].y, e[i].z, e[i].w}, sw[4] = {s.x, s.y, s.z, s.w};
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    dw[i][k] = ew[k] ^ sw[k];
                    lw[i][k] = ew[k] & 0x01010101u;
                }
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint32_t a = blk_addr((uint32_t)q, (uint32_t)(4 * g + k));
                *reinterpret_cast<uint4 *>(dt + a) = make_uint4(dw[0][k], dw[1][k], dw[2][k], dw[3][k]);
                *reinterpret_cast<uint4 *>(lb + a) = make_uint4(lw[0][k], lw[1][k], lw[2][k], lw[3][k]);
            }
            if (lane < kCodeRecord / 16) reinterpret_cast<uint4 *>(rec)[lane] = rc;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

            // this lane's original blocks (q, 4g + k), gathered and turned back
            uint32_t ny[4], nx[4], R1[4], k0[4], k1[4];
            block_turns4(rec, J.min_level, up, (uint32_t)q, (uint32_t)g, ny, nx, R1, k0, k1);
            uint32_t m[4][4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint32_t a = blk_addr(ny[k], nx[k]);
                const uint4 wd = *reinterpret_cast<const uint4 *>(dt + a);
                const uint4 wl = *reinterpret_cast<const uint4 *>(lb + a);
                const uint4 f0 = *reinterpret_cast<const uint4 *>(itab + ((R1[k] * 2u) * 16u + k0[k]) * 4u);
                const uint4 f1 = *reinterpret_cast<const uint4 *>(itab + ((R1[k] * 2u + 1u) * 16u + k1[k]) * 4u);
                const uint32_t fs[8] = {f0.x, f0.y, f0.z, f0.w, f1.x, f1.y, f1.z, f1.w};
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    Do[i][k] = vperm(wd.y, wd.x, fs[2 * i]) | vperm(wd.w, wd.z, fs[2 * i + 1]);
                    const uint32_t l = vperm(wl.y, wl.x, fs[2 * i]) | vperm(wl.w, wl.z, fs[2 * i + 1]);
                    m[i][k] = __builtin_amdgcn_udot4(l, 0x08040201u, 0u, false);   // label pattern
                }
            }
            if (tx == 0 && g == 0) {
#pragma unroll
                for (int i = 0; i < 4; ++i) m[i][0] |= 1u;   // column 0 has no left neighbour
            }
            // per row: the lane's last labelled value, then a scan over the four lanes of the row
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                uint32_t f = 0;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    sel[i][k] = gtab[m[i][k]];
                    f = vperm(Do[i][k], f, sel[i][k]);
                }
                const uint32_t any = m[i][0] | m[i][1] | m[i][2] | m[i][3];
                uint32_t v = any ? ((f >> 24) | 0x100u) : 0u;
                uint32_t p = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x90, 0xF, 0xF, false);   // lane g-1 (0: itself)
                v = v ? v : p;
                p = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x44, 0xF, 0xF, false);            // lane g-2 (0, 1: themselves)
                v = v ? v : p;
                const uint32_t x = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x90, 0xF, 0xF, false);
                excl[i] = g == 0 ? 0u : x;
                tsum[i] = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xFF, 0xF, 0xF, false);      // lane 3
                fcol[i] = 64u;
            }
            if (segd) {
                // column of the first labelled pixel of each tile row (minimum over the row's lanes)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const uint32_t m16 = m[i][0] | (m[i][1] << 4) | (m[i][2] << 8) | (m[i][3] << 12);
                    uint32_t f = m16 ? 16u * (uint32_t)g + (uint32_t)__builtin_ctz(m16) : 64u;
                    uint32_t o = (uint32_t)__builtin_amdgcn_mov_dpp((int)f, 0xB1, 0xF, 0xF, false);   // lane g ^ 1
                    f = f < o ? f : o;
                    o = (uint32_t)__builtin_amdgcn_mov_dpp((int)f, 0x4E, 0xF, 0xF, false);            // lane g ^ 2
                    fcol[i] = f < o ? f : o;
                }
            }
            if (g == 0)
                *reinterpret_cast<uint2 *>(&sums[slot][wave][4 * q]) =
                    make_uint2((tsum[0] | (fcol[0] << 9)) | ((tsum[1] | (fcol[1] << 9)) << 16),
                               (tsum[2] | (fcol[2] << 9)) | ((tsum[3] | (fcol[3] << 9)) << 16));
            if (DYN && g == 3)
                *reinterpret_cast<uint32_t *>(&lastpx[DYN ? slot : 0][wave][4 * q]) =
                    (Do[0][3] >> 24) | ((Do[1][3] >> 24) << 8) | ((Do[2][3] >> 24) << 16) | (Do[3][3] & 0xFF000000u);
            if (DYN && lane == 0) tileb[DYN ? slot : 0][wave] = bq;
        }
        __syncthreads();
        if (have) {
            const int b = J.fixed_b > 0 ? J.fixed_b : (int)bq;
            const uint32_t mrep = ((0xFFu << (8 - b)) & 0xFFu) * 0x01010101u;   // replaceable bits, every byte
            const uint2 cw = *reinterpret_cast<const uint2 *>(&carry[slot][half][4 * q]);
            const uint32_t cr[4] = {cw.x & 0xFFFFu, cw.x >> 16, cw.y & 0xFFFFu, cw.y >> 16};
            uint32_t lf[4] = {0, 0, 0, 0}, rf[4] = {64, 64, 64, 64};
            if (side) {
                const uint2 lw2 = *reinterpret_cast<const uint2 *>(&sums[slot][wave - 1][4 * q]);
                lf[0] = lw2.x & 0x1FFu;
                lf[1] = (lw2.x >> 16) & 0x1FFu;
                lf[2] = lw2.y & 0x1FFu;
                lf[3] = (lw2.y >> 16) & 0x1FFu;
            } else if (segd && right_in) {
                const uint2 rw2 = *reinterpret_cast<const uint2 *>(&sums[slot][wave + 1][4 * q]);
                rf[0] = (rw2.x >> 9) & 0x7Fu;
                rf[1] = (rw2.x >> 25) & 0x7Fu;
                rf[2] = (rw2.y >> 9) & 0x7Fu;
                rf[3] = (rw2.y >> 25) & 0x7Fu;
            }
            uint32_t nc[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const uint32_t from_left = first ? 0u : cr[i];           // into the quad (none at a segment start)
                uint32_t tin = lf[i] ? lf[i] : from_left;                // into this tile
                if (DYN) {
                    // the restored last pixel of the row of the tile to the left
                    tin = from_left;
                    if (side) {
                        const uint32_t src = lf[i] ? lf[i] : from_left;
                        const uint32_t bl = tileb[DYN ? slot : 0][wave - 1];
                        const uint32_t ml = (0xFFu << (8 - bl)) & 0xFFu;
                        const uint32_t dl = lastpx[DYN ? slot : 0][wave - 1][4 * q + i];
                        tin = src ? ((src & ml) | (dl & ~ml & 0xFFu) | 0x100u) : 0u;
                    }
                }
                const uint32_t cin = excl[i] ? excl[i] : tin;            // into this lane
                nc[i] = tsum[i] ? tsum[i] : tin;                         // out of this tile
                if (DYN) {
                    const uint32_t dl = qperm<0xFF>(Do[i][3] >> 24);     // this row's column 63 (lane 3 of the row)
                    const uint32_t mt = mrep & 0xFFu;
                    nc[i] = nc[i] ? ((nc[i] & mt) | (dl & ~mt & 0xFFu) | 0x100u) : 0u;
                }
                uint32_t f = (cin & 0xFFu) << 24;
                uint32_t o[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    f = vperm(Do[i][k], f, sel[i][k]);
                    o[k] = (f & mrep) | (Do[i][k] & ~mrep);
                }
                const uint64_t oidx = (uint64_t)(ty * kTile + 4 * q + i) * (uint64_t)J.N + (uint64_t)(tx * kTile + 16 * g);
                gstore<uint4>(J.out + oidx, make_uint4(o[0], o[1], o[2], o[3]));
            }
            if (side && g == 0)
                *reinterpret_cast<uint2 *>(&carry[slot ^ 1u][half][4 * q]) =
                    make_uint2(nc[0] | (nc[1] << 16), nc[2] | (nc[3] << 16));
            if (segd) {
                // per image row and segment: leading pixels still waiting for a carry (left
                // wave) and the last labelled value (wave with the segment's last tile)
                const uint32_t ns = (uint32_t)cur.S.ns, sg = (uint32_t)cur.S.s;
                const uint64_t R0 = (uint64_t)(128 * cur.S.p + 64 * half + 4 * q);
                uint16_t *fix_lead = reinterpret_cast<uint16_t *>(ws + J.ws_fix);
                uint16_t *fix_sum = fix_lead + (uint64_t)J.M * ns;
                if (!side) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        if (first) {
                            lead[i] = 0;
                            open[i] = 1;
                        }
                        if (open[i]) {
                            if (fcol[i] < 64u) {
                                lead[i] += fcol[i];
                                open[i] = 0;
                            } else if (rf[i] < 64u) {
                                lead[i] += 64u + rf[i];
                                open[i] = 0;
                            } else {
                                lead[i] += right_in ? 128u : 64u;
                            }
                        }
                    }
                    if (last && g == 0) {
#pragma unroll
                        for (int i = 0; i < 4; ++i) fix_lead[(uint64_t)sg * J.M + R0 + i] = (uint16_t)lead[i];
                    }
                }
                if (last && g == 0 && (side || !right_in)) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) fix_sum[(uint64_t)sg * J.M + R0 + i] = (uint16_t)nc[i];
                }
            }
        }
        cur = nxt;
        nxt = nn;
    }
    if (!IMG) break;
    __syncthreads();                              // LDS is reused by the next image
    }
}

// Rows of images whose band pairs were cut into segments: a segment started
// without the value carried in from its left, so the pixels before its first
// labelled pixel (per row) still lack their replaceable bits.  One thread per
// image row and segment s >= 1 (blockIdx.y + 1) finds the nearest segment to
// the left with a labelled pixel in that row (column 0 always is one) and
// completes those pixels, kFixPiece bytes at a time (all loads of a piece
// before its stores).  Records are segment-major: [s][row].  Image blockIdx.z.
constexpr uint32_t kFixPiece = 64;

// Dynamic b: a pixel labelled 0 takes the top b bits (b of its tile) of its
// restored left neighbour, so the value entering segment sg is the restored
// last pixel of the row before it: from the nearest segment to the left whose
// row end is known (fix_sum flag 0x100; segment 0 always is), carried through
// the tiles of the segments between (none labelled in this row, so each
// tile's restored last pixel is the carry in its b bits and its decrypted
// value below them, as the quad kernel left it), then spread over the lead
// tile by tile.
__device__ void recover_fix_dyn(const Job &J, const uint8_t *ws, uint32_t R, uint32_t sg, uint32_t qs, uint32_t ns,
                                uint32_t lead, const uint16_t *fix_sum) {
    const uint32_t *tmap = reinterpret_cast<const uint32_t *>(ws + J.ws_tmap);
    const uint32_t ty = R >> kTileLog;
    auto mask_of = [&](uint32_t tx) {           // replaceable bits of tile (ty, tx)
        int ey, ex;
        uint32_t up;
        tmap_unpack(tmap[ty * (uint32_t)J.tiles_x + tx], ey, ex, up);
        const uint32_t b = J.btab[ey * J.tiles_x + ex];
        return (0xFFu << (8 - b)) & 0xFFu;
    };
    uint8_t *row = J.out + (uint64_t)R * (uint64_t)J.N;
    uint32_t k = sg;
    uint32_t carry = 0;
    while (k-- > 0) {
        const uint32_t sum = fix_sum[(uint64_t)k * J.M + R];
        if (sum & 0x100u) {
            carry = sum & 0xFFu;
            break;
        }
    }
    const uint32_t seg_px = qs * 2u * (uint32_t)kTile;
    for (uint32_t x = (k + 1) * seg_px; x < sg * seg_px; x += kTile) {   // unlabelled segments between
        const uint32_t m = mask_of(x >> kTileLog);
        carry = (carry & m) | (row[x + kTile - 1] & ~m & 0xFFu);
    }
    const uint32_t x0 = sg * seg_px;
    const uint32_t n = lead < (uint32_t)J.N - x0 ? lead : (uint32_t)J.N - x0;
    for (uint32_t t0 = 0; t0 < n; t0 += kTile) {                         // the lead, one tile at a time
        const uint32_t m = mask_of((x0 + t0) >> kTileLog);
        const uint32_t cv = (carry & m) * 0x01010101u, mb = m * 0x01010101u;
        const uint32_t e = n - t0 < (uint32_t)kTile ? n - t0 : (uint32_t)kTile;
#pragma unroll
        for (int q = 0; q < kTile / 16; ++q) {
            const uint32_t k16 = 16u * (uint32_t)q;
            if (k16 >= e) continue;
            uint4 v = *reinterpret_cast<const uint4 *>(row + x0 + t0 + k16);
            uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const uint32_t lo = k16 + 4u * (uint32_t)j;
                const uint32_t take = lo >= e ? 0u : (e - lo >= 4u ? 4u : e - lo);
                const uint32_t bm = take == 4u ? 0xFFFFFFFFu : ((1u << (8u * take)) - 1u);
                const uint32_t pm = bm & mb;
                w[j] = (w[j] & ~pm) | (cv & pm);
            }
            *reinterpret_cast<uint4 *>(row + x0 + t0 + k16) = make_uint4(w[0], w[1], w[2], w[3]);
        }
        if (e == (uint32_t)kTile) carry = (carry & m) | (row[x0 + t0 + kTile - 1] & ~m & 0xFFu);
    }
}

__global__ void k_recover_fix(const Job *__restrict__ jobs, const uint8_t *__restrict__ ws) {
    const Job &J = jobs[blockIdx.z];
    if (!J.fast || J.method == RDHEI_LMR) return;
    const uint32_t qs = (uint32_t)J.qseg;
    const uint32_t nq = (uint32_t)((J.tiles_x + 1) >> 1), ns = (nq + qs - 1) / qs;
    const uint32_t sg = blockIdx.y + 1u;
    if (sg >= ns) return;
    const uint32_t R = blockIdx.x * blockDim.x + threadIdx.x;
    if (R >= (uint32_t)J.M) return;
    const uint16_t *fix_lead = reinterpret_cast<const uint16_t *>(ws + J.ws_fix);
    const uint16_t *fix_sum = fix_lead + (uint64_t)J.M * ns;
    const uint32_t lead = fix_lead[(uint64_t)sg * J.M + R];
    if (!lead) return;
    if (J.method == RDHEI_DEMR) {
        recover_fix_dyn(J, ws, R, sg, qs, ns, lead, fix_sum);
        return;
    }
    uint32_t carry = 0;
    for (uint32_t t = sg; t-- > 0;) {
        const uint32_t sum = fix_sum[(uint64_t)t * J.M + R];
        if (sum & 0x100u) {
            carry = sum & 0xFFu;
            break;
        }
    }
    const int b = J.fixed_b > 0 ? J.fixed_b : J.meta->b;
    const uint32_t mrep = ((0xFFu << (8 - b)) & 0xFFu) * 0x01010101u;   // replaceable bits, every byte
    const uint32_t cv = carry * 0x01010101u;
    const uint32_t x0 = sg * qs * 2u * (uint32_t)kTile;
    const uint32_t n = lead < (uint32_t)J.N - x0 ? lead : (uint32_t)J.N - x0;
    // rows and segments start on 64-byte boundaries; the bytes of the last
    // block past the lead keep their values
    uint8_t *row = J.out + (uint64_t)R * (uint64_t)J.N + x0;
    constexpr int kB = (int)(kFixPiece / 16);
    for (uint32_t k0 = 0; k0 < n; k0 += kFixPiece) {
        uint4 v[kB];
#pragma unroll
        for (int q = 0; q < kB; ++q)
            if (k0 + 16u * (uint32_t)q < n) v[q] = *reinterpret_cast<const uint4 *>(row + k0 + 16u * (uint32_t)q);
#pragma unroll
        for (int q = 0; q < kB; ++q) {
            const uint32_t k = k0 + 16u * (uint32_t)q;
            if (k >= n) continue;
            uint32_t w[4] = {v[q].x, v[q].y, v[q].z, v[q].w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const uint32_t lo = k + 4u * (uint32_t)j;
                const uint32_t take = lo >= n ? 0u : (n - lo >= 4u ? 4u : n - lo);   // bytes of this word in the lead
                const uint32_t bm = take == 4u ? 0xFFFFFFFFu : ((1u << (8u * take)) - 1u);
                const uint32_t pm = bm & mrep;
                w[j] = (w[j] & ~pm) | (cv & pm);
            }
            *reinterpret_cast<uint4 *>(row + k) = make_uint4(w[0], w[1], w[2], w[3]);
        }
    }
}

// ---- launchers ---------------------------------------------------------------
// Workgroups of a persistent launch: what fits on the device at once (or the
// caller's cap), never more than there are units.
// The resident count of each kernel is asked of the runtime once and kept.
static int resident_per_cu(const void *kernel) {
    static std::mutex mu;
    static std::unordered_map<const void *, int> cache;
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(kernel);
    if (it != cache.end()) return it->second;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kThreads, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    cache[kernel] = per_cu;
    return per_cu;
}

template <typename K>
static unsigned persistent_grid(const Launch &L, K kernel, uint32_t units) {
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (cus <= 0) cus = 1;
    }
    const int per_cu = resident_per_cu(reinterpret_cast<const void *>(kernel));
    uint32_t g = (uint32_t)cus * (uint32_t)per_cu;
    if (L.max_grid > 0) g = (uint32_t)L.max_grid;
    if (g > units) g = units;
    return g ? g : 1;
}

static inline unsigned grid_for(const Launch &L, uint32_t units) {
    uint32_t g = units;
    if (L.max_grid > 0 && g > (uint32_t)L.max_grid) g = (uint32_t)L.max_grid;
    return g ? g : 1;
}

void launch_tile_prep(const Launch &L, uint32_t units, bool stats) {
    if (!units) return;
    const uint32_t *UJ = L.ujob[UNIT_TILE];
    if (stats) {
        hipLaunchKernelGGL(k_stats_zero, dim3((L.njobs + 255) / 256, L.njobs > 64 ? 1 : 8), dim3(256), 0, L.stream,
                           L.jobs, L.njobs, L.ws);
    }
    with_keystream(L.keystream, [&](auto K) {
        constexpr int KS = decltype(K)::value;
        if (stats && L.dyn)
            hipLaunchKernelGGL((k_tile_prep<true, KS, true>), dim3(persistent_grid(L, k_tile_prep<true, KS, true>, units)),
                               dim3(kThreads), 0, L.stream, L.jobs, L.njobs, L.ws, units, UJ);
        else if (stats)
            hipLaunchKernelGGL((k_tile_prep<true, KS>), dim3(persistent_grid(L, k_tile_prep<true, KS>, units)),
                               dim3(kThreads), 0, L.stream, L.jobs, L.njobs, L.ws, units, UJ);
        else
            hipLaunchKernelGGL((k_tile_prep<false, KS>), dim3(persistent_grid(L, k_tile_prep<false, KS>, units)),
                               dim3(kThreads), 0, L.stream, L.jobs, L.njobs, L.ws, units, UJ);
    });
}

void launch_finalize(const Launch &L, bool stats, const std::vector<int> &big, const std::vector<Job> &hj) {
    if (!L.njobs) return;
    if (big.size() < (size_t)L.njobs) {
        const unsigned g = grid_for(L, (uint32_t)L.njobs);
        if (stats)
            hipLaunchKernelGGL(k_finalize<true>, dim3(g), dim3(kThreads), 0, L.stream, L.jobs, L.njobs, L.ws);
        else
            hipLaunchKernelGGL(k_finalize<false>, dim3(g), dim3(kThreads), 0, L.stream, L.jobs, L.njobs, L.ws);
    }
    for (int j : big) {
        const Job &J = hj[(size_t)j];
        const unsigned nb = (unsigned)(((J.tiles_y + kFinBlock - 1) / kFinBlock) * ((J.tiles_x + kFinBlock - 1) / kFinBlock));
        const unsigned nt = (unsigned)(((uint32_t)(J.tiles_x * J.tiles_y) + kThreads - 1) / kThreads);
        hipLaunchKernelGGL(k_fin_blocks, dim3(nb), dim3(kThreads), 0, L.stream, L.jobs, j, L.ws);
        if (stats) hipLaunchKernelGGL(k_fin_top<true>, dim3(1), dim3(kThreads), 0, L.stream, L.jobs, j, L.ws);
        else hipLaunchKernelGGL(k_fin_top<false>, dim3(1), dim3(kThreads), 0, L.stream, L.jobs, j, L.ws);
        hipLaunchKernelGGL(k_fin_tmap, dim3(nt), dim3(kThreads), 0, L.stream, L.jobs, j, L.ws);
    }
}

void launch_encrypt_tiles(const Launch &L, uint32_t units, int mode) {
    if (!units) return;
    const uint32_t *UJ = L.ujob[UNIT_QROW];
    const dim3 bl(kThreads);
    with_keystream(L.keystream, [&](auto K) {
        constexpr int KS = decltype(K)::value;
        if (mode == ENC_EMR)
            hipLaunchKernelGGL((k_encrypt_quad<ENC_EMR, KS>), dim3(persistent_grid(L, k_encrypt_quad<ENC_EMR, KS>, units)),
                               bl, 0, L.stream, L.jobs, L.njobs, L.ws, units, UJ);
        else if (mode == ENC_DEMR)
            hipLaunchKernelGGL((k_encrypt_quad<ENC_DEMR, KS>), dim3(persistent_grid(L, k_encrypt_quad<ENC_DEMR, KS>, units)),
                               bl, 0, L.stream, L.jobs, L.njobs, L.ws, units, UJ);
        else if (mode == ENC_LMR)
            hipLaunchKernelGGL((k_encrypt_quad<ENC_LMR, KS>), dim3(persistent_grid(L, k_encrypt_quad<ENC_LMR, KS>, units)),
                               bl, 0, L.stream, L.jobs, L.njobs, L.ws, units, UJ);
        else
            hipLaunchKernelGGL((k_encrypt_quad<ENC_LMR_MAPS, KS>),
                               dim3(persistent_grid(L, k_encrypt_quad<ENC_LMR_MAPS, KS>, units)), bl, 0, L.stream, L.jobs,
                               L.njobs, L.ws, units, UJ);
    });
}

// One workgroup per image by default (more than fit on the device at once:
// the hardware starts each as another ends, so the workgroups on a CU are in
// different phases), or the caller's cap with images dealt round-robin.
void launch_encrypt_images(const Launch &L) {
    if (!L.njobs) return;
    const unsigned grid = grid_for(L, (uint32_t)L.njobs);
    with_keystream(L.keystream, [&](auto K) {
        constexpr int KS = decltype(K)::value;
        auto go = [&](auto kernel) {
            hipLaunchKernelGGL(kernel, dim3(grid), dim3(kEncImageWaves * 64), 0, L.stream, L.jobs, L.njobs, L.ws);
        };
        if (L.dyn) go(k_encrypt_image<ENC_DEMR, KS, kEncImageWaves>);
        else go(k_encrypt_image<ENC_EMR, KS, kEncImageWaves>);
    });
}

void launch_recover_images(const Launch &L) {
    if (!L.njobs) return;
    const unsigned grid = grid_for(L, (uint32_t)L.njobs);
    with_keystream(L.keystream, [&](auto K) {
        constexpr int KS = decltype(K)::value;
        if (L.dyn)
            hipLaunchKernelGGL((k_recover_quad_emr<KS, true, true>), dim3(grid), dim3(kThreads), 0, L.stream, L.jobs,
                               L.njobs, L.ws, 0u, L.ujob[UNIT_QROW]);
        else
            hipLaunchKernelGGL((k_recover_quad_emr<KS, false, true>), dim3(grid), dim3(kThreads), 0, L.stream, L.jobs,
                               L.njobs, L.ws, 0u, L.ujob[UNIT_QROW]);
    });
}

void launch_recover_bands(const Launch &L, uint32_t units, int method, uint32_t fix_rows, uint32_t fix_segs) {
    if (!units) return;
    const uint32_t *UJ = L.ujob[UNIT_BAND];
    const dim3 bl(kThreads);
    if (method != RDHEI_LMR) {
        with_keystream(L.keystream, [&](auto K) {
            constexpr int KS = decltype(K)::value;
            if (L.dyn)
                hipLaunchKernelGGL((k_recover_quad_emr<KS, true>), dim3(persistent_grid(L, k_recover_quad_emr<KS, true>, units)),
                                   bl, 0, L.stream, L.jobs, L.njobs, L.ws, units, L.ujob[UNIT_QROW]);
            else
                hipLaunchKernelGGL((k_recover_quad_emr<KS>), dim3(persistent_grid(L, k_recover_quad_emr<KS>, units)), bl, 0,
                                   L.stream, L.jobs, L.njobs, L.ws, units, L.ujob[UNIT_QROW]);
        });
        if (fix_rows)
            hipLaunchKernelGGL(k_recover_fix, dim3((fix_rows + 255) / 256, fix_segs - 1, (unsigned)L.njobs), dim3(256),
                               0, L.stream, L.jobs, L.ws);
    }
    else
        with_keystream(L.keystream, [&](auto K) {
            constexpr int KS = decltype(K)::value;
            hipLaunchKernelGGL((k_recover_band_lmr<KS>), dim3(persistent_grid(L, k_recover_band_lmr<KS>, units)), bl, 0,
                               L.stream, L.jobs, L.njobs, L.ws, units, UJ);
        });
}

}  // namespace rdhei

// Data hiding and extraction (Sec. III-A/B data hiding phase, decoding with
// K2).  The rotated location map decides which pixels are redundant; payload
// bit t lands in redundant pixel floor(t / rep) of the raster order, bits
// top..top-rep+1 (rep = b for EMR, b-1 for LMR), so a pixel's bit offset is
// rep times the number of redundant pixels before it: a prefix sum.
//
// The work is cut into steps of 4096 raster pixels, one wave each.  Batches
// of small images walk each image with one wave, step after step, the rank
// carried in registers.  Otherwise (large images, small batches) the steps
// are spread over the device in three launches, none of which waits on
// another workgroup: count the redundant pixels of every step, turn each
// image's counts into exclusive prefix sums, then hide or extract every step
// at its rank.  On request the steps go in one pass instead, each taking its
// rank from the steps before it with a decoupled look-back.
#include <algorithm>

#include "device.hpp"
#include "hide4.hpp"

namespace rdhei {

// A step: four 16-byte loads per lane of a wave; lane l, load k covers
// pixels 1024 k + 16 l .. +15 of the step.
constexpr int kWLoads = 4;
constexpr uint64_t kWSegPx = 64ull * 16 * kWLoads;                   // 4096 pixels
// payload window of one step (at most 7 bits per pixel), in 32-bit words
constexpr int kWWinWords = (int)((kWSegPx * 7 + 127) / 128 + 1) * 4 + 8;
// images of at most this many pixels may be walked whole by one wave
constexpr uint64_t kWholeMaxPx = 1ull << 20;

struct HideParams {
    uint32_t rep, shift;      // replaceable bits per redundant pixel, position of the lowest
    int64_t nbits;            // bits requested (resolved against the capacity)
    uint64_t nonce;           // keystream nonce of the image (from the meta record)
    bool ok;
};

__device__ __forceinline__ HideParams hide_params(const Job &J) {
    const rdhei_meta *m = J.meta;
    HideParams h;
    const int b = m->b;
    h.rep = (uint32_t)(J.method == RDHEI_LMR ? b - 1 : b);
    h.shift = (uint32_t)(8 - b);
    const int64_t cap = m->capacity_bits;
    h.nbits = J.nbits < 0 ? cap : J.nbits;
    // dynamic b: the b of each tile comes from the tile table (meta.b is 0)
    h.ok = (m->status == RDHEI_OK) && h.nbits <= cap && (J.method == RDHEI_DEMR || (h.rep >= 1 && h.rep <= 7));
    h.rep = uni(h.rep);
    h.shift = uni(h.shift);
    h.nbits = (int64_t)uni64((uint64_t)h.nbits);
    h.nonce = uni64(m->nonce);
    h.ok = uni(h.ok ? 1u : 0u) != 0;
    return h;
}

// 16 pixels at raster index pos (multiple of 16) of an image of `total`
// pixels; pixels past the end read as 0x01 (never redundant).
__device__ __forceinline__ uint4 load16(const uint8_t *img, uint64_t pos, uint64_t total) {
    if (pos + 16 <= total) return gload<uint4>(img + pos);
    uint32_t w[4] = {0x01010101u, 0x01010101u, 0x01010101u, 0x01010101u};
    for (int k = 0; k < 16; ++k)
        if (pos + k < total) w[k >> 2] = (w[k >> 2] & ~(0xFFu << (8 * (k & 3)))) | ((uint32_t)img[pos + k] << (8 * (k & 3)));
    return make_uint4(w[0], w[1], w[2], w[3]);
}

__device__ __forceinline__ void store16(uint8_t *img, uint64_t pos, uint64_t total, uint4 v) {
    if (pos + 16 <= total) { gstore<uint4>(img + pos, v); return; }
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
    for (int k = 0; k < 16; ++k)
        if (pos + k < total) img[pos + k] = (uint8_t)(w[k >> 2] >> (8 * (k & 3)));
}

// Redundancy mask of 16 pixels: bit k set when pixel pos+k is labelled 0.
__device__ __forceinline__ uint32_t redundant16(const Job &J, uint4 px, uint64_t pos, uint64_t total) {
    uint32_t m = 0;
    if (pos >= total) return 0u;
    if (J.method != RDHEI_LMR) {
        // LSB 0 -> redundant: the inverted LSBs of the bytes, weighted by their
        // bit position with 4-byte dot products
        const uint32_t lo = __builtin_amdgcn_udot4(
            ~px.y & 0x01010101u, 0x80402010u, __builtin_amdgcn_udot4(~px.x & 0x01010101u, 0x08040201u, 0u, false), false);
        const uint32_t hi = __builtin_amdgcn_udot4(
            ~px.w & 0x01010101u, 0x80402010u, __builtin_amdgcn_udot4(~px.z & 0x01010101u, 0x08040201u, 0u, false), false);
        m = lo | (hi << 8);
    } else {
        const uint32_t be = ((uint32_t)J.lbits[pos >> 3] << 8) | (pos + 8 < total ? J.lbits[(pos >> 3) + 1] : 0xFFu);
#pragma unroll
        for (int k = 0; k < 16; ++k) m |= ((~(be >> (15 - k))) & 1u) << k;
    }
    if (pos + 16 > total) m &= (1u << (uint32_t)(total - pos)) - 1u;
    return m;
}

// ---- four pixels per word ---------------------------------------------------------
// Field permutes of hide4.hpp, staged once per workgroup in LDS: compact at 0,
// expand at 16, redundant-byte masks at 32.
static __constant__ hide4::Tables kHideTables = hide4::kTables;

__device__ __forceinline__ void stage_hide_tables(uint32_t *lds, int tid) {
    if (tid < hide4::kWords) lds[tid] = reinterpret_cast<const uint32_t *>(&kHideTables)[tid];
}

// Per-image constants of the word-wise field moves.
struct Hide4 {
    uint32_t rep, shift;
    uint32_t low_bytes;   // (2^rep - 1) in every byte
    uint32_t rep_bytes;   // the replaceable bits, in every byte
    uint32_t low_pairs;   // (2^rep - 1) in bytes 0 and 2
};

__device__ __forceinline__ Hide4 hide4_params(const HideParams &hp) {
    Hide4 h;
    h.rep = hp.rep;
    h.shift = hp.shift;
    const uint32_t low = (1u << hp.rep) - 1u;
    h.low_bytes = low * 0x01010101u;
    h.rep_bytes = (low << hp.shift) * 0x01010101u;
    h.low_pairs = low * 0x00010001u;
    return h;
}

// Dynamic b: the b of the tile holding raster pixel pos (16-pixel loads never
// straddle a tile: tiles are 64 wide).  The row comes from a double-precision
// product with 1/N and one integer correction (pos < 2^31, so the product is
// off by at most one).
__device__ __forceinline__ uint32_t tile_b_at(const Job &J, uint64_t pos, double inv_n) {
    uint32_t r = (uint32_t)((double)pos * inv_n);
    if ((uint64_t)(r + 1u) * (uint64_t)J.N <= pos) ++r;
    if ((uint64_t)r * (uint64_t)J.N > pos) --r;
    const uint32_t c = (uint32_t)(pos - (uint64_t)r * (uint64_t)J.N);
    return (uint32_t)gload<uint8_t>(J.btab + (uint64_t)(r >> kTileLog) * (uint64_t)J.tiles_x + (c >> kTileLog));
}

// Word-wise field moves for a b (EMR-style: the top b bits are replaced).
__device__ __forceinline__ Hide4 hide4_of_b(uint32_t b) {
    Hide4 h;
    h.rep = b;
    h.shift = 8u - b;
    const uint32_t low = (1u << b) - 1u;
    h.low_bytes = low * 0x01010101u;
    h.rep_bytes = (low << h.shift) * 0x01010101u;
    h.low_pairs = low * 0x00010001u;
    return h;
}

// 32 payload bits (top bit first) starting at bit p of a staged window whose
// word 0 is a guard, so p >= 32 and the bits lie in words (p-1)/32 and the next.
__device__ __forceinline__ uint32_t window_bits(const uint32_t *win, uint32_t p) {
    const uint32_t t = p - 1u;
    const uint32_t a = t >> 5;
    return __builtin_amdgcn_alignbit(win[a], win[a + 1], 31u - (t & 31u));
}

// OR a run of bits (top-aligned in s) into an extraction window at bit p.
__device__ __forceinline__ void window_or(uint32_t *win, uint32_t p, uint32_t s) {
    const uint32_t a = p >> 5, sb = p & 31u;
    atomicOr(&win[a], s >> sb);
    atomicOr(&win[a + 1], __builtin_amdgcn_alignbit(s, 0u, sb));
}

// Embedding into 16 pixels (four words w) with redundancy mask rm: the first
// redundant pixel takes the payload bits from window position rel (relative
// to the staged window, before its guard word); bits at rend and beyond are
// not part of the payload.  Whole words use the field permutes; the one word
// where the payload ends goes pixel by pixel.
// TAIL: the payload may end inside these pixels (the last step of an image
// hiding less than its capacity); otherwise every field lies inside it.
template <bool TAIL = true>
__device__ __forceinline__ void embed16(uint32_t w[4], uint32_t rm, uint32_t rel, uint32_t rend, const uint32_t *win,
                                        const Hide4 &hk, const uint32_t *T) {
    const uint32_t rep = hk.rep;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint32_t m = (rm >> (4 * q)) & 0xFu;
        const uint32_t pos = rel;
        rel += __umul24((uint32_t)__popc(m), rep);
        // whole word (every field inside the payload), computed unconditionally
        const uint32_t run = window_bits(win, pos + 32u);
        const uint32_t F01 = run >> (32u - 2u * rep);
        const uint32_t F23 = __builtin_amdgcn_ubfe(run, 32u - 4u * rep, 2u * rep);
        const uint32_t t = (F01 << 16) | F23;
        const uint32_t cp = (t & hk.low_pairs) | (((t >> rep) & hk.low_pairs) << 8);
        const uint32_t e = vperm(0u, cp, T[16 + m]) << hk.shift;
        const uint32_t K = T[32 + m] & hk.rep_bytes;
        const uint32_t x = w[q];
        if (!TAIL) {
            w[q] = (x & ~K) | (e & K);
            continue;
        }
        w[q] = rel <= rend ? ((x & ~K) | (e & K)) : x;
        if (__builtin_expect(rel > rend && pos < rend, 0)) {
            // the word where the payload ends: pixel by pixel
            const uint32_t top = hk.shift + rep - 1u;
            uint32_t p = pos, y = x;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (((m >> j) & 1u) && p < rend) {
                    const uint32_t val = window_bits(win, p + 32u) >> (32u - rep);
                    const uint32_t left = rend - p;
                    const uint32_t take = left < rep ? left : rep;
                    const uint32_t wmask = ((1u << take) - 1u) << (top + 1u - take);
                    y = (y & ~(wmask << (8 * j))) | (((val << hk.shift) & wmask) << (8 * j));
                    p += rep;
                }
            }
            w[q] = y;
        }
    }
}

// Extraction from 16 pixels: the payload bits of the redundant pixels are ORed
// into the window (word 0 = first window word) from position rel on; bits at
// rend and beyond are dropped.
template <bool TAIL = true>
__device__ __forceinline__ void extract16(const uint32_t w[4], uint32_t rm, uint32_t rel, uint32_t rend, uint32_t *win,
                                          const Hide4 &hk, const uint32_t *T) {
    const uint32_t rep = hk.rep;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint32_t m = (rm >> (4 * q)) & 0xFu;
        const uint32_t pos = rel;
        rel += __umul24((uint32_t)__popc(m), rep);
        if (!TAIL) {
            // every field inside the payload; an empty word ORs zeros
            const uint32_t c = vperm(0u, (w[q] >> hk.shift) & hk.low_bytes, T[m]);
            const uint32_t v = ((c >> 8) & 0x00FF00FFu) << rep | (c & 0x00FF00FFu);
            const uint32_t s = __builtin_amdgcn_alignbit(v >> 16, v << (32u - 2u * rep), 2u * rep);
            window_or(win, pos, s);
            continue;
        }
        if (m == 0 || pos >= rend) continue;
        if (__builtin_expect(rel <= rend, 1)) {
            // the fields of the word's redundant pixels, in order, then packed
            // pairwise: P = f0 f1 in bits 16.., Q = f2 f3 in bits 0..
            const uint32_t c = vperm(0u, (w[q] >> hk.shift) & hk.low_bytes, T[m]);
            const uint32_t v = ((c >> 8) & 0x00FF00FFu) << rep | (c & 0x00FF00FFu);
            // f0 f1 f2 f3 top-aligned: P on top, Q right below it
            const uint32_t s = __builtin_amdgcn_alignbit(v >> 16, v << (32u - 2u * rep), 2u * rep);
            window_or(win, pos, s);
        } else {
            uint32_t p = pos;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (((m >> j) & 1u) && p < rend) {
                    const uint32_t pv = (w[q] >> (8 * j)) & 0xFFu;
                    const uint32_t left = rend - p;
                    const uint32_t take = left < rep ? left : rep;
                    const uint32_t val = (pv >> (hk.shift + rep - take)) & ((1u << take) - 1u);
                    window_or(win, p, val << (32u - take));
                    p += take;
                }
            }
        }
    }
}

// ---- extraction -------------------------------------------------------------------
// Message words a step only partly owns (shared with a neighbouring step, or
// the message's last word) go to a side record; two small passes clear, then
// OR them into place.
struct PartWord {
    int64_t word;      // word index into the message (-1: none)
    uint32_t bits;     // already XORed with the keystream and masked to the owner's bits
    uint32_t job;
};

// mask of big-endian bits [lo, hi) of word w (stream bit 0 = bit 31 of word 0)
__device__ __forceinline__ uint32_t be_mask(int64_t w, int64_t lo, int64_t hi) {
    int64_t a = lo - 32 * w, b = hi - 32 * w;
    if (a < 0) a = 0;
    if (b > 32) b = 32;
    if (b <= a) return 0u;
    const uint32_t upto_b = b >= 32 ? 0xFFFFFFFFu : ~(0xFFFFFFFFu >> b);
    const uint32_t upto_a = a == 0 ? 0u : ~(0xFFFFFFFFu >> a);
    return upto_b & ~upto_a;
}

// Message keystream word w, big-endian bit order.
template <int KS>
__device__ __forceinline__ uint32_t ks_word(uint64_t key, uint64_t nonce, int64_t w) {
    const U4 ks = stream_block<KS>(key, nonce, kDomainMessage, (uint64_t)w >> 2);
    const uint32_t kw = (w & 3) == 0 ? ks.x : (w & 3) == 1 ? ks.y : (w & 3) == 2 ? ks.z : ks.w;
    return __builtin_bswap32(kw);
}

__global__ void k_extract_fix(const Job *__restrict__ jobs, const PartWord *__restrict__ part, uint32_t n, int phase) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const PartWord pw = part[i];
    if (pw.word < 0) return;
    uint32_t *dst = reinterpret_cast<uint32_t *>(jobs[pw.job].msg) + pw.word;
    if (phase == 0) *dst = 0u;
    else atomicOr(dst, pw.bits);
}


// ---- whole images, one wave each ----------------------------------------------
// Images of at most kWholeMaxPx pixels, in batches large enough to fill the
// device, are walked by one wave each, one step after the other: the rank
// carries over in registers, the next step's pixels (and, embedding, message
// blocks) are loaded while the current one is processed, ranks inside a step
// come from a wave scan (DPP), and nothing waits on another wave.

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Pixels of one step.  Whole-image hiding is used only for images whose
// pixel count is a multiple of 16, so every 16-byte piece is in or out.
__device__ __forceinline__ void wseg_load(const uint8_t *img, uint64_t s0, uint64_t s1, int lane, uint4 px[kWLoads]) {
#pragma unroll
    for (int k = 0; k < kWLoads; ++k) {
        const uint64_t pos = s0 + (uint64_t)k * 1024u + 16 * (uint64_t)lane;
        px[k] = pos < s1 ? gload<uint4>(img + pos) : make_uint4(0x01010101u, 0x01010101u, 0x01010101u, 0x01010101u);
    }
}

// Ranks of the step's redundant pixels: for each load k of the lane, the
// redundant pixels of the step before its first pixel; T = the step's total.
// cnt[k]: the lane's count for load k (redundant pixels, or with a b per tile
// their payload bits: at most 7 * 16 per lane, 7,168 per load of the wave).
__device__ __forceinline__ void step_ranks(const uint32_t cnt[kWLoads], uint32_t lr[kWLoads], uint32_t &T) {
    // counts of loads 0, 1 and 2, 3 in 16-bit halves (at most 7,168 each)
    const uint32_t c01 = cnt[0] | (cnt[1] << 16);
    const uint32_t c23 = cnt[2] | (cnt[3] << 16);
    const uint32_t i01 = wave_scan_incl(c01), i23 = wave_scan_incl(c23);
    const uint32_t t01 = uni((uint32_t)__builtin_amdgcn_readlane((int)i01, 63));
    const uint32_t t23 = uni((uint32_t)__builtin_amdgcn_readlane((int)i23, 63));
    const uint32_t e01 = i01 - c01, e23 = i23 - c23;
    const uint32_t tot0 = t01 & 0xFFFFu, tot1 = t01 >> 16, tot2 = t23 & 0xFFFFu, tot3 = t23 >> 16;
    lr[0] = e01 & 0xFFFFu;
    lr[1] = tot0 + (e01 >> 16);
    lr[2] = tot0 + tot1 + (e23 & 0xFFFFu);
    lr[3] = tot0 + tot1 + tot2 + (e23 >> 16);
    T = tot0 + tot1 + tot2 + tot3;
}

// ChaCha20 message stream for a window: the lanes take 64-byte-aligned groups
// of four 16-byte blocks, lane l block (first & ~3) + base + l, with a uniform
// trip count, so that the four lanes of each quad compute one ChaCha20 block
// together (stream_block_quad); blocks outside [first, last] are computed and
// not used.
// Embedding: message blocks fb..lb, XORed with the stream, byte-swapped into
// win[4 + 4q], q = block - fb.
template <int KS>
__device__ __forceinline__ void stage_window_quad(const Job &J, uint64_t nonce, int lane, int64_t fb, int64_t lb,
                                                  uint32_t *win) {
    const int64_t fa = fb & ~(int64_t)3;
    for (int64_t base = 0; base <= lb - fa; base += 64) {
        const int64_t q = fa + base + lane - fb;
        const bool in = q >= 0 && q <= lb - fb;
        const uint4 mv = in ? gload<uint4>(J.msg + 16 * (uint64_t)(fb + q)) : make_uint4(0, 0, 0, 0);
        const U4 ks = stream_block_quad<KS>(J.key, nonce, kDomainMessage, (uint64_t)(fa + base + lane));
        if (in)
            *reinterpret_cast<uint4 *>(win + 4 + 4 * q) =
                make_uint4(__builtin_bswap32(mv.x ^ ks.x), __builtin_bswap32(mv.y ^ ks.y),
                           __builtin_bswap32(mv.z ^ ks.z), __builtin_bswap32(mv.w ^ ks.w));
    }
}

// Extraction: calls put(block, stream words) for the blocks B0..B1 (and the
// aligned neighbours, whose words put must skip).
template <int KS, typename F>
__device__ __forceinline__ void each_stream_block_quad(const Job &J, uint64_t nonce, int lane, int64_t B0, int64_t B1,
                                                       F &&put) {
    const int64_t Ba = B0 & ~(int64_t)3;
    for (int64_t base = 0; base <= B1 - Ba; base += 64) {
        const int64_t blk = Ba + base + lane;
        put(blk, stream_block_quad<KS>(J.key, nonce, kDomainMessage, (uint64_t)blk));
    }
}

// Whole images are at most kWholeMaxPx pixels, so every bit offset of their
// payload (at most 7 bits per pixel) fits in 32 bits.
static_assert(kWholeMaxPx * 7 < (1ull << 31), "whole-image bit offsets are 32-bit");

// DYN: a b per tile (RDHEI_DEMR): each 16-pixel load takes its tile's b, and
// ranks count payload bits instead of redundant pixels (unit = 1 bit, not rep).
template <bool EMBED, int KS, bool DYN = false>
__device__ __forceinline__ void hide_image_wave(const Job &J, const HideParams &hp, uint32_t *win, const uint32_t *htab) {
    const int lane = threadIdx.x & 63;
    const uint8_t *img = EMBED ? J.out : J.in;
    const uint32_t total = (uint32_t)((uint64_t)J.M * (uint64_t)J.N);
    const uint32_t nseg = (uint32_t)((total + kWSegPx - 1) / kWSegPx);
    const uint32_t rep = DYN ? 4u : hp.rep;          // DYN: only a prefetch estimate
    const uint32_t unit = DYN ? 1u : hp.rep;         // payload bits per rank step
    const uint32_t nbits = (uint32_t)hp.nbits;
    const Hide4 hk0 = hide4_params(hp);
    const double inv_n = 1.0 / (double)J.N;
    uint32_t rank = 0;
    uint32_t carry = 0;          // extraction: bits of the partial word left by the previous step
    uint32_t carry_word = ~0u;   // its word index (none: ~0)
    uint4 nxt[kWLoads];
    wseg_load(img, 0, total < kWSegPx ? total : (uint32_t)kWSegPx, lane, nxt);
    // embedding: message blocks of the next step, loaded a step ahead.  A step
    // needs at most 4096 * 7 bits = 224 blocks from its first one; as many are
    // prefetched as the previous step used, plus two (neighbouring steps of an
    // image hold similar numbers of redundant pixels), and a step loads any
    // further blocks it needs itself.
    uint4 mpre[4];
    uint32_t npre = 0;
    const uint32_t nblk = (nbits + 127) >> 7;
    auto msg_prefetch = [&](uint32_t first_blk, uint32_t n) {
        npre = n;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t blk = first_blk + (uint32_t)(lane + 64 * i);
            mpre[i] = (uint32_t)(lane + 64 * i) < n && blk < nblk ? gload<uint4>(J.msg + 16 * (uint64_t)blk)
                                                                  : make_uint4(0, 0, 0, 0);
        }
    };
    constexpr bool kPrefetch = EMBED && KS != kKsChaCha20;   // ChaCha20 loads its blocks in stage_window_quad
    if (kPrefetch) msg_prefetch(0, (uint32_t)((kWSegPx / 2 * rep + 127) / 128));   // first step: half its pixels
    for (uint32_t seg = 0; seg < nseg; ++seg) {
        const uint32_t s0 = seg * (uint32_t)kWSegPx;
        const uint32_t s1 = s0 + (uint32_t)kWSegPx < total ? s0 + (uint32_t)kWSegPx : total;
        uint4 px[kWLoads];
#pragma unroll
        for (int k = 0; k < kWLoads; ++k) px[k] = nxt[k];
        {   // the next step's pixels (the last step reloads itself)
            const uint32_t ns = seg + 1 < nseg ? seg + 1 : seg;
            const uint32_t n0 = ns * (uint32_t)kWSegPx;
            wseg_load(img, n0, n0 + (uint32_t)kWSegPx < total ? n0 + (uint32_t)kWSegPx : total, lane, nxt);
        }
        uint32_t rm[kWLoads], cnt[kWLoads];
        Hide4 hks[kWLoads];
#pragma unroll
        for (int k = 0; k < kWLoads; ++k) {
            const uint32_t pos = s0 + (uint32_t)k * 1024u + 16u * (uint32_t)lane;
            rm[k] = redundant16(J, px[k], pos, s1);
            hks[k] = hk0;
            if (DYN) hks[k] = hide4_of_b(pos < s1 ? tile_b_at(J, pos, inv_n) : 2u);
            cnt[k] = DYN ? (uint32_t)__popc(rm[k]) * hks[k].rep : (uint32_t)__popc(rm[k]);
        }
        uint32_t lr[kWLoads], T;
        step_ranks(cnt, lr, T);
        const uint32_t wstart = rank * unit;
        if (wstart >= nbits) break;
        uint32_t wend = (rank + T) * unit;
        if (wend > nbits) wend = nbits;
        rank += T;
        if (T > 0 && EMBED) {
            // window bits relative to the first staged 16-byte block (the prefetch base)
            const uint32_t fb = wstart >> 7, lb = (wend - 1) >> 7;
            const uint32_t off0 = wstart - (fb << 7), rend = wend - (fb << 7);
            if constexpr (KS == kKsChaCha20) {
                stage_window_quad<KS>(J, hp.nonce, lane, fb, lb, win);
            } else {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const uint32_t q = (uint32_t)(lane + 64 * i);
                    if (q > lb - fb) continue;
                    const uint4 mv = q < npre ? mpre[i] : gload<uint4>(J.msg + 16 * (uint64_t)(fb + q));
                    const U4 ks = stream_block<KS>(J.key, hp.nonce, kDomainMessage, (uint64_t)(fb + q));
                    *reinterpret_cast<uint4 *>(win + 4 + 4 * q) =
                        make_uint4(__builtin_bswap32(mv.x ^ ks.x), __builtin_bswap32(mv.y ^ ks.y),
                                   __builtin_bswap32(mv.z ^ ks.z), __builtin_bswap32(mv.w ^ ks.w));
                }
            }
            // rank already counts this step
            const uint32_t used = lb - fb + 1u + 2u;
            if (kPrefetch) msg_prefetch((rank * unit) >> 7, used < 256u ? used : 256u);
            wave_sync();
            if (wend == rank * unit) {   // the whole step inside the payload (uniform)
#pragma unroll
                for (int k = 0; k < kWLoads; ++k) {
                    if (!rm[k]) continue;
                    uint32_t w[4] = {px[k].x, px[k].y, px[k].z, px[k].w};
                    embed16<false>(w, rm[k], off0 + lr[k] * unit, rend, win + 3, hks[k], htab);
                    gstore<uint4>(J.out + s0 + (uint64_t)k * 1024u + 16 * (uint64_t)lane, make_uint4(w[0], w[1], w[2], w[3]));
                }
            } else {
#pragma unroll
                for (int k = 0; k < kWLoads; ++k) {
                    const uint32_t rel = off0 + lr[k] * unit;
                    if (!rm[k] || rel >= rend) continue;
                    uint32_t w[4] = {px[k].x, px[k].y, px[k].z, px[k].w};
                    embed16(w, rm[k], rel, rend, win + 3, hks[k], htab);   // word 0 of the window is a guard
                    gstore<uint4>(J.out + s0 + (uint64_t)k * 1024u + 16 * (uint64_t)lane, make_uint4(w[0], w[1], w[2], w[3]));
                }
            }
            wave_sync();
        } else if (T > 0) {
            // The window starts at the first message word of the keystream
            // block holding bit wstart (word 4 B0), so that every block's four
            // words are one aligned 16-byte LDS read.
            const uint32_t W0 = wstart >> 5, W1 = (wend + 31) >> 5, B0 = W0 >> 2;
            const uint32_t base = 4 * B0, off0 = wstart - 32 * base, rend = wend - 32 * base;
            const uint32_t nq = ((W1 - base) >> 2) + 1;    // 16-byte pieces: words 0..W1-base (the last
                                                           // may take a zero OR past the run's end)
            for (uint32_t q = (uint32_t)lane; q < nq; q += 64) {
                uint4 z = make_uint4(0, 0, 0, 0);
                if (carry_word != ~0u && carry_word >= base && (carry_word - base) >> 2 == q) {
                    const uint32_t c = (carry_word - base) & 3u;
                    z.x = c == 0 ? carry : 0u;
                    z.y = c == 1 ? carry : 0u;
                    z.z = c == 2 ? carry : 0u;
                    z.w = c == 3 ? carry : 0u;
                }
                *reinterpret_cast<uint4 *>(win + 4 * q) = z;
            }
            wave_sync();
            if (wend == rank * unit) {   // the whole step inside the payload (uniform)
#pragma unroll
                for (int k = 0; k < kWLoads; ++k) {
                    const uint32_t w[4] = {px[k].x, px[k].y, px[k].z, px[k].w};
                    extract16<false>(w, rm[k], off0 + lr[k] * unit, rend, win, hks[k], htab);
                }
            } else {
#pragma unroll
                for (int k = 0; k < kWLoads; ++k) {
                    const uint32_t rel = off0 + lr[k] * unit;
                    if (!rm[k] || rel >= rend) continue;
                    const uint32_t w[4] = {px[k].x, px[k].y, px[k].z, px[k].w};
                    extract16(w, rm[k], rel, rend, win, hks[k], htab);
                }
            }
            wave_sync();
            // complete words [W0, Wend) go out; a trailing partial word waits for the next step
            const bool partial = (wend & 31) != 0;
            const uint32_t Wend = partial ? W1 - 1 : W1;
            uint32_t *msgw = reinterpret_cast<uint32_t *>(J.msg);
            if (Wend > W0) {   // one keystream block per four message words
                const uint32_t B1 = (Wend - 1) >> 2;
                if constexpr (KS == kKsChaCha20) {
                    each_stream_block_quad<KS>(J, hp.nonce, lane, (int64_t)B0, (int64_t)B1, [&](int64_t blk, const U4 &ks) {
                        const uint32_t kw[4] = {ks.x, ks.y, ks.z, ks.w};
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const uint32_t w = 4 * (uint32_t)blk + (uint32_t)i;
                            if (blk >= (int64_t)B0 && w >= W0 && w < Wend)
                                gstore<uint32_t>(msgw + w, __builtin_bswap32(win[w - base]) ^ kw[i]);
                        }
                    });
                } else {
                    for (uint32_t bq = (uint32_t)lane; bq <= B1 - B0; bq += 64) {
                        const uint32_t blk = B0 + bq;
                        const U4 ks = stream_block<KS>(J.key, hp.nonce, kDomainMessage, (uint64_t)blk);
                        const uint4 v = *reinterpret_cast<const uint4 *>(win + 4 * bq);
                        const uint4 o = make_uint4(__builtin_bswap32(v.x) ^ ks.x, __builtin_bswap32(v.y) ^ ks.y,
                                                   __builtin_bswap32(v.z) ^ ks.z, __builtin_bswap32(v.w) ^ ks.w);
                        const uint32_t w0 = 4 * blk;
                        if (w0 >= W0 && w0 + 4 <= Wend) {
                            gstore<uint4>(msgw + w0, o);            // the whole block
                        } else {
                            const uint32_t ow[4] = {o.x, o.y, o.z, o.w};
#pragma unroll
                            for (int i = 0; i < 4; ++i)
                                if (w0 + i >= W0 && w0 + i < Wend) gstore<uint32_t>(msgw + w0 + i, ow[i]);
                        }
                    }
                }
            }
            carry_word = partial ? W1 - 1 : ~0u;
            carry = partial ? uni(win[W1 - 1 - base]) : 0u;
            wave_sync();
        }
    }
    if (!EMBED && carry_word != ~0u && lane == 0) {
        // the message's last word: bits past nbits are stored as zero
        const uint32_t own = be_mask(carry_word, 0, hp.nbits);
        gstore<uint32_t>(reinterpret_cast<uint32_t *>(J.msg) + carry_word,
                         __builtin_bswap32((carry ^ ks_word<KS>(J.key, hp.nonce, carry_word)) & own));
    }
}

// One wave per workgroup, one image per wave (a grid-stride loop when the grid
// is capped).
template <bool EMBED, int KS, bool DYN = false>
__global__ __launch_bounds__(64) void k_hide_wave(const Job *__restrict__ jobs, int njobs, uint32_t units,
                                                  const uint32_t *__restrict__ ujob) {
    __shared__ __align__(16) uint32_t win[kWWinWords];
    __shared__ uint32_t htab[hide4::kWords];
    const int lane = threadIdx.x;
    if (lane < hide4::kWords) htab[lane] = reinterpret_cast<const uint32_t *>(&kHideTables)[lane];
    wave_sync();
    for (uint32_t u = blockIdx.x; u < units; u += gridDim.x) {
        const int j = (int)uni((uint32_t)find_job<UNIT_IMG>(jobs, njobs, u, ujob));
        const Job &J = jobs[j];
        const HideParams hp = hide_params(J);
        if (!hp.ok) {
            if (lane == 0 && J.meta->status == RDHEI_OK) J.meta->status = RDHEI_ECAPACITY;
        } else {
            hide_image_wave<EMBED, KS, DYN>(J, hp, win, htab);
        }
        wave_sync();
    }
}

// ---- steps of any image: count, scan, hide -------------------------------------
// Every step is one work unit (UNIT_SEG).  Pixels of a step past the image's
// end read as never redundant, so any image size works.
__device__ __forceinline__ void step_load(const uint8_t *img, uint64_t s0, uint64_t s1, int lane, uint4 px[kWLoads]) {
#pragma unroll
    for (int k = 0; k < kWLoads; ++k) {
        const uint64_t pos = s0 + (uint64_t)k * 1024u + 16 * (uint64_t)lane;
        px[k] = pos < s1 ? load16(img, pos, s1) : make_uint4(0x01010101u, 0x01010101u, 0x01010101u, 0x01010101u);
    }
}

// Pass 1: redundant pixels of every step.
__global__ __launch_bounds__(kThreads) void k_seg_count(const Job *__restrict__ jobs, int njobs, uint32_t units,
                                                         const uint32_t *__restrict__ ujob, uint32_t *__restrict__ cnt) {
    const int lane = threadIdx.x & 63, wave = (int)uni(threadIdx.x >> 6);
    const uint32_t stride = gridDim.x * (uint32_t)(kThreads / 64);
    for (uint32_t u = blockIdx.x * (uint32_t)(kThreads / 64) + (uint32_t)wave; u < units; u += stride) {
        const Job &J = jobs[uni((uint32_t)find_job<UNIT_SEG>(jobs, njobs, u, ujob))];
        const uint64_t total = (uint64_t)J.M * (uint64_t)J.N;
        const uint64_t s0 = (uint64_t)(u - J.ubase[UNIT_SEG]) * kWSegPx;
        const uint64_t s1 = s0 + kWSegPx < total ? s0 + kWSegPx : total;
        uint4 px[kWLoads];
        step_load(J.in, s0, s1, lane, px);
        uint32_t c = 0;
        const bool dyn = J.method == RDHEI_DEMR;   // uniform: counts payload bits (a b per tile)
        const double inv_n = 1.0 / (double)J.N;
#pragma unroll
        for (int k = 0; k < kWLoads; ++k) {
            const uint64_t pos = s0 + (uint64_t)k * 1024u + 16 * (uint64_t)lane;
            const uint32_t n = (uint32_t)__popc(redundant16(J, px[k], pos, s1));
            c += dyn && n ? n * tile_b_at(J, pos, inv_n) : n;
        }
        c = wave_scan_incl(c);
        if (lane == 63) cnt[u] = c;
    }
}

// Pass 2: each image's step counts -> exclusive prefix sums, in place.  One
// workgroup of kScanThreads per image, chunks of kScanChunk counts: a chunk
// comes in with coalesced loads (consecutive threads, consecutive counts)
// into LDS, where thread t scans its own run of kScanPer consecutive counts
// (rows padded to an odd stride, so those reads do not collide in banks),
// the runs' totals are scanned across the workgroup, and the prefix sums go
// out with coalesced stores.
constexpr int kScanThreads = 1024, kScanPer = 8;
constexpr uint32_t kScanChunk = kScanThreads * kScanPer;
__device__ __forceinline__ uint32_t scan_slot(uint32_t e) { return e / kScanPer * (kScanPer + 1) + e % kScanPer; }
__global__ __launch_bounds__(kScanThreads) void k_seg_scan(const Job *__restrict__ jobs, uint32_t *__restrict__ cnt) {
    __shared__ uint32_t sh[kScanThreads * (kScanPer + 1)];
    __shared__ uint32_t wsum[kScanThreads / 64];
    const Job &J = jobs[blockIdx.x];
    const uint32_t n = J.ucount[UNIT_SEG];
    if (n == 0) return;   // uniform over the workgroup
    uint32_t *c = cnt + J.ubase[UNIT_SEG];
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    uint32_t carry = 0;   // total of the earlier chunks (uniform)
    for (uint32_t c0 = 0; c0 < n; c0 += kScanChunk) {
        const uint32_t m = n - c0 < kScanChunk ? n - c0 : kScanChunk;
        uint32_t v[kScanPer];
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) {
            const uint32_t e = (uint32_t)k * kScanThreads + tid;
            v[k] = e < m ? c[c0 + e] : 0u;
        }
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) sh[scan_slot((uint32_t)k * kScanThreads + tid)] = v[k];
        __syncthreads();
        uint32_t r[kScanPer], sum = 0;
#pragma unroll
        for (int i = 0; i < kScanPer; ++i) {
            r[i] = sh[tid * (kScanPer + 1) + i];
            sum += r[i];
        }
        const uint32_t incl = wave_scan_incl(sum);
        if (lane == 63) wsum[wave] = incl;
        __syncthreads();
        uint32_t base = carry, tot = 0;
#pragma unroll
        for (uint32_t w = 0; w < kScanThreads / 64; ++w) {
            const uint32_t x = wsum[w];
            base += w < wave ? x : 0u;
            tot += x;
        }
        uint32_t ex = base + incl - sum;
#pragma unroll
        for (int i = 0; i < kScanPer; ++i) {
            sh[tid * (kScanPer + 1) + i] = ex;
            ex += r[i];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) {
            const uint32_t e = (uint32_t)k * kScanThreads + tid;
            if (e < m) c[c0 + e] = sh[scan_slot(e)];
        }
        carry += tot;
        __syncthreads();   // the next chunk reuses sh and wsum
    }
}

// One step's pixels, redundancy masks, field moves and ranks inside the step
// (T: the step's total, in redundant pixels, or payload bits with DYN).
struct StepState {
    uint4 px[kWLoads];
    uint32_t rm[kWLoads], lr[kWLoads], T;
    Hide4 hks[kWLoads];
    uint64_t s0, s1;
};

template <bool DYN>
__device__ __forceinline__ void step_prepare(const Job &J, uint32_t u, const Hide4 &hk0, StepState &S) {
    const int lane = threadIdx.x & 63;
    const uint64_t total = (uint64_t)J.M * (uint64_t)J.N;
    S.s0 = (uint64_t)(u - J.ubase[UNIT_SEG]) * kWSegPx;
    S.s1 = S.s0 + kWSegPx < total ? S.s0 + kWSegPx : total;
    const double inv_n = 1.0 / (double)J.N;
    step_load(J.in, S.s0, S.s1, lane, S.px);
    uint32_t cnt[kWLoads];
#pragma unroll
    for (int k = 0; k < kWLoads; ++k) {
        const uint64_t pos = S.s0 + (uint64_t)k * 1024u + 16 * (uint64_t)lane;
        S.rm[k] = redundant16(J, S.px[k], pos, S.s1);
        S.hks[k] = hk0;
        if (DYN) S.hks[k] = hide4_of_b(pos < S.s1 ? tile_b_at(J, pos, inv_n) : 2u);
        cnt[k] = (uint32_t)__popc(S.rm[k]) * (DYN ? S.hks[k].rep : 1u);
    }
    step_ranks(cnt, S.lr, S.T);
}

// Hide (EMBED) or extract the payload bits of one step whose first redundant
// pixel (or payload bit, DYN) has image-wide rank r0.
template <bool EMBED, int KS, bool DYN>
__device__ __forceinline__ void step_hide(const Job &J, int j, uint32_t u, const HideParams &hp, const StepState &S,
                                          uint64_t r0, uint32_t *win, const uint32_t *htab, PartWord *__restrict__ part) {
    const int lane = threadIdx.x & 63;
    const uint32_t rep = DYN ? 1u : hp.rep;       // payload bits per rank step (DYN: ranks count bits)
    const uint32_t T = S.T;
    const uint64_t s0 = S.s0, s1 = S.s1;
    const int64_t wstart = (int64_t)(r0 * rep);
    int64_t wend = (int64_t)((r0 + T) * rep);
    if (wend > hp.nbits) wend = hp.nbits;
    if (T == 0 || wstart >= wend) return;
    if (EMBED) {
        // window bits relative to the first staged 16-byte block
        const int64_t fb = wstart >> 7, lb = (wend - 1) >> 7;
        const uint32_t off0 = (uint32_t)(wstart - (fb << 7)), rend = (uint32_t)(wend - (fb << 7));
        if constexpr (KS == kKsChaCha20) {
            stage_window_quad<KS>(J, hp.nonce, lane, fb, lb, win);
        } else {
            for (int64_t q = lane; q <= lb - fb; q += 64) {
                const uint64_t blk = (uint64_t)(fb + q);
                const uint4 mv = gload<uint4>(J.msg + 16 * blk);
                const U4 ks = stream_block<KS>(J.key, hp.nonce, kDomainMessage, blk);
                *reinterpret_cast<uint4 *>(win + 4 + 4 * q) =
                    make_uint4(__builtin_bswap32(mv.x ^ ks.x), __builtin_bswap32(mv.y ^ ks.y),
                               __builtin_bswap32(mv.z ^ ks.z), __builtin_bswap32(mv.w ^ ks.w));
            }
        }
        wave_sync();
#pragma unroll
        for (int k = 0; k < kWLoads; ++k) {
            const uint32_t rel = off0 + S.lr[k] * rep;
            if (!S.rm[k] || rel >= rend) continue;
            uint32_t w[4] = {S.px[k].x, S.px[k].y, S.px[k].z, S.px[k].w};
            embed16(w, S.rm[k], rel, rend, win + 3, S.hks[k], htab);   // word 0 of the window is a guard
            store16(J.out, s0 + (uint64_t)k * 1024u + 16 * (uint64_t)lane, s1, make_uint4(w[0], w[1], w[2], w[3]));
        }
    } else {
        const int64_t W0 = wstart >> 5, W1 = (wend + 31) >> 5;
        const uint32_t off0 = (uint32_t)(wstart & 31), rend = (uint32_t)(wend - 32 * W0);
        for (int64_t q = lane; q < W1 - W0 + 1; q += 64) win[q] = 0u;
        wave_sync();
#pragma unroll
        for (int k = 0; k < kWLoads; ++k) {
            const uint32_t rel = off0 + S.lr[k] * rep;
            if (!S.rm[k] || rel >= rend) continue;
            const uint32_t w[4] = {S.px[k].x, S.px[k].y, S.px[k].z, S.px[k].w};
            extract16(w, S.rm[k], rel, rend, win, S.hks[k], htab);
        }
        wave_sync();
        // one keystream block per four message words; words shared with a
        // neighbouring step go to the side records
        uint32_t *msgw = reinterpret_cast<uint32_t *>(J.msg);
        const int64_t B0 = W0 >> 2, B1 = (W1 - 1) >> 2;
        if constexpr (KS == kKsChaCha20) {
            each_stream_block_quad<KS>(J, hp.nonce, lane, B0, B1, [&](int64_t blk, const U4 &ks) {
                const uint32_t kw[4] = {ks.x, ks.y, ks.z, ks.w};
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int64_t w = 4 * blk + i;
                    if (w < W0 || w >= W1) continue;
                    const uint32_t own = be_mask(w, wstart, wend);
                    const uint32_t v = (win[w - W0] ^ __builtin_bswap32(kw[i])) & own;
                    if (own == 0xFFFFFFFFu) {
                        gstore<uint32_t>(msgw + w, __builtin_bswap32(v));
                    } else {
                        PartWord pw;
                        pw.word = w;
                        pw.bits = __builtin_bswap32(v);
                        pw.job = (uint32_t)j;
                        part[2 * u + (w == W0 ? 0 : 1)] = pw;
                    }
                }
            });
        } else {
            for (int64_t bq = lane; bq <= B1 - B0; bq += 64) {
                const U4 ks = stream_block<KS>(J.key, hp.nonce, kDomainMessage, (uint64_t)(B0 + bq));
                const uint32_t kw[4] = {ks.x, ks.y, ks.z, ks.w};
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int64_t w = 4 * (B0 + bq) + i;
                    if (w < W0 || w >= W1) continue;
                    const uint32_t own = be_mask(w, wstart, wend);
                    const uint32_t v = (win[w - W0] ^ __builtin_bswap32(kw[i])) & own;
                    if (own == 0xFFFFFFFFu) {
                        gstore<uint32_t>(msgw + w, __builtin_bswap32(v));
                    } else {
                        PartWord pw;
                        pw.word = w;
                        pw.bits = __builtin_bswap32(v);
                        pw.job = (uint32_t)j;
                        part[2 * u + (w == W0 ? 0 : 1)] = pw;
                    }
                }
            }
        }
    }
}

// Pass 3 of the counted steps: hide or extract every step at the rank the
// scan gave it.
template <bool EMBED, int KS, bool DYN = false>
__global__ __launch_bounds__(kThreads) void k_seg_hide(const Job *__restrict__ jobs, int njobs, uint32_t units,
                                                        const uint32_t *__restrict__ ujob,
                                                        const uint32_t *__restrict__ rank, PartWord *__restrict__ part) {
    __shared__ __align__(16) uint32_t wins[kThreads / 64][kWWinWords];
    __shared__ uint32_t htab[hide4::kWords];
    const int lane = threadIdx.x & 63, wave = (int)uni(threadIdx.x >> 6);
    uint32_t *win = wins[wave];
    stage_hide_tables(htab, (int)threadIdx.x);
    __syncthreads();
    const uint32_t stride = gridDim.x * (uint32_t)(kThreads / 64);
    for (uint32_t u = blockIdx.x * (uint32_t)(kThreads / 64) + (uint32_t)wave; u < units; u += stride) {
        if (!EMBED && lane < 2) part[2 * u + lane].word = -1;
        const int j = (int)uni((uint32_t)find_job<UNIT_SEG>(jobs, njobs, u, ujob));
        const Job &J = jobs[j];
        const HideParams hp = hide_params(J);
        if (!hp.ok) {
            if (lane == 0 && u == J.ubase[UNIT_SEG] && J.meta->status == RDHEI_OK) J.meta->status = RDHEI_ECAPACITY;
            continue;
        }
        StepState S;
        step_prepare<DYN>(J, u, hide4_params(hp), S);
        step_hide<EMBED, KS, DYN>(J, j, u, hp, S, uni(rank[u]), win, htab, part);
        wave_sync();
    }
}

// ---- steps in one pass: decoupled look-back ------------------------------------
// Each wave takes steps in ticket order (an atomic counter), so every step
// before the one it holds has been taken by a running wave.  It publishes its
// step's total (flag AGG), then walks back over the published words of the
// earlier steps of the same image, 64 at a time, until it meets one that
// already holds its inclusive prefix (flag INCL) or the image's first step;
// it publishes its own inclusive prefix and hides at the exclusive one.  A
// step's own total needs nothing from other steps, so every wait ends: the
// image's first step publishes INCL at once.  The image is read once,
// instead of once to count and once to hide.
// Status words: flag in bits 62..63, value below (a prefix is < 7 * 2^31).
constexpr uint64_t kLbAgg = 1ull << 62, kLbIncl = 2ull << 62, kLbValue = (1ull << 62) - 1;
// Polls of one look-back window before the wait is given up (RDHEI_EDEVICE in
// the image's meta); far beyond any real wait.
constexpr uint32_t kLbMaxPolls = 1u << 22;

__device__ __forceinline__ void lb_publish(uint64_t *st, uint64_t v) {
    __hip_atomic_store(st, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t lb_read(const uint64_t *st) {
    return __hip_atomic_load(const_cast<uint64_t *>(st), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Exclusive prefix of step u (first step of its image: ufirst); false when the
// wait was given up.  Every lane runs every iteration (the window's loads are
// clamped into the image's steps, decisions come from ballots), so the loop's
// control flow is the same for all lanes.
__device__ __forceinline__ bool lb_look_back(const uint64_t *status, uint32_t u, uint32_t ufirst, uint64_t &prefix) {
    const int lane = threadIdx.x & 63;
    prefix = 0;
    int64_t p = (int64_t)u - 1;
    uint32_t polls = 0;
    bool done = false, ok = true;
    while (!done) {
        const int64_t q = p - lane;
        const bool inside = q >= (int64_t)ufirst;
        const uint64_t r = lb_read(status + (inside ? q : (int64_t)ufirst));
        const uint64_t s = inside ? r : kLbIncl;                         // before the image: prefix 0
        const uint32_t flag = (uint32_t)(s >> 62);
        const uint64_t incl = __ballot(flag == 2u);
        const uint64_t wait = __ballot(flag == 0u);
        const int li = incl ? (int)__builtin_ctzll(incl) : 64;   // nearest INCL lane
        const uint64_t need = li >= 63 ? ~0ull : ((2ull << li) - 1ull);
        if (wait & need) {
            if (++polls > kLbMaxPolls) {
                ok = false;
                done = true;
            } else {
                __builtin_amdgcn_s_sleep(1);
            }
        } else {
            // the AGG totals (below 2^15 each) of lanes before li, then li's prefix
            const uint32_t a = lane < li ? (uint32_t)(s & kLbValue) : 0u;
            prefix += uni((uint32_t)__builtin_amdgcn_readlane((int)wave_scan_incl(a), 63));
            if (li < 64) {
                const uint64_t v = s & kLbValue;
                prefix += ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), li) << 32) |
                          (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, li);
                done = true;
            } else {
                p -= 64;
                polls = 0;
            }
        }
    }
    return ok;
}

// status: units + 1 words, cleared by k_lb_clear (the last one is the ticket
// counter).  Every lane takes part in the ticket's atomic add (lane 0 adds 1,
// the others 0) and the loop has no early continue, so the control flow
// around the ticket never depends on the lane: a wave's lanes always agree
// on the step they hold.
template <bool EMBED, int KS, bool DYN = false>
__global__ __launch_bounds__(kThreads) void k_seg_hide1(const Job *__restrict__ jobs, int njobs, uint32_t units,
                                                         const uint32_t *__restrict__ ujob, uint64_t *__restrict__ status,
                                                         PartWord *__restrict__ part) {
    __shared__ __align__(16) uint32_t wins[kThreads / 64][kWWinWords];
    __shared__ uint32_t htab[hide4::kWords];
    const int lane = threadIdx.x & 63, wave = (int)uni(threadIdx.x >> 6);
    uint32_t *win = wins[wave];
    stage_hide_tables(htab, (int)threadIdx.x);
    __syncthreads();
    unsigned long long *ticket = reinterpret_cast<unsigned long long *>(status + units);
    auto claim = [&]() -> uint32_t {
        const uint32_t t = (uint32_t)atomicAdd(ticket, lane == 0 ? 1ull : 0ull);
        return uni(t);   // lane 0's: the step this wave takes
    };
    for (uint32_t u = claim(); u < units; u = claim()) {
        if (!EMBED && lane < 2) part[2 * u + lane].word = -1;
        const int j = (int)uni((uint32_t)find_job<UNIT_SEG>(jobs, njobs, u, ujob));
        const Job &J = jobs[j];
        const uint32_t ufirst = J.ubase[UNIT_SEG];
        const HideParams hp = hide_params(J);
        if (hp.ok) {
            StepState S;
            step_prepare<DYN>(J, u, hide4_params(hp), S);
            uint64_t r0 = 0;
            bool have = true;
            if (u == ufirst) {
                if (lane == 0) lb_publish(status + u, kLbIncl | S.T);
            } else {
                if (lane == 0) lb_publish(status + u, kLbAgg | S.T);
                have = lb_look_back(status, u, ufirst, r0);
                if (lane == 0) lb_publish(status + u, have ? (kLbIncl | (r0 + S.T)) : kLbIncl);
                if (!have && lane == 0) J.meta->status = RDHEI_EDEVICE;
            }
            if (have) step_hide<EMBED, KS, DYN>(J, j, u, hp, S, r0, win, htab, part);
        } else if (lane == 0) {
            // every step of the image is skipped; nothing waits on this word
            lb_publish(status + u, kLbIncl);
            if (u == ufirst && J.meta->status == RDHEI_OK) J.meta->status = RDHEI_ECAPACITY;
        }
        wave_sync();
    }
}

__global__ void k_lb_clear(uint64_t *__restrict__ status, uint32_t n) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += gridDim.x * blockDim.x) status[i] = 0;
}

// ---- launchers ---------------------------------------------------------------------
static inline unsigned grid_for(const Launch &L, uint32_t units) {
    uint32_t g = units;
    if (L.max_grid > 0 && g > (uint32_t)L.max_grid) g = (uint32_t)L.max_grid;
    return g ? g : 1;
}

// Waves of k_hide_wave resident on the device.
static uint32_t hide_wave_resident() {
    static uint32_t v = 0;
    if (!v) {
        int dev = 0, cus = 0, per_cu = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_hide_wave<true, kKsPhilox>, 64, 0) != hipSuccess || per_cu < 1)
            per_cu = 1;
        v = (uint32_t)(cus > 0 ? cus : 1) * (uint32_t)per_cu;
    }
    return v;
}

// One wave per image walks the whole image; by default as many waves as are
// resident, each taking images in turn.
void launch_hide_images(const Launch &L, uint32_t units, bool embed) {
    if (!units) return;
    unsigned g;
    if (L.max_grid > 0) {
        g = grid_for(L, units);
    } else {
        const uint32_t res = hide_wave_resident();
        g = units < res ? units : res;
    }
    with_keystream(L.keystream, [&](auto K) {
        constexpr int KS = decltype(K)::value;
        if (embed && L.dyn)
            hipLaunchKernelGGL((k_hide_wave<true, KS, true>), dim3(g), dim3(64), 0, L.stream, L.jobs, L.njobs, units,
                               L.ujob[UNIT_IMG]);
        else if (embed)
            hipLaunchKernelGGL((k_hide_wave<true, KS>), dim3(g), dim3(64), 0, L.stream, L.jobs, L.njobs, units,
                               L.ujob[UNIT_IMG]);
        else if (L.dyn)
            hipLaunchKernelGGL((k_hide_wave<false, KS, true>), dim3(g), dim3(64), 0, L.stream, L.jobs, L.njobs, units,
                               L.ujob[UNIT_IMG]);
        else
            hipLaunchKernelGGL((k_hide_wave<false, KS>), dim3(g), dim3(64), 0, L.stream, L.jobs, L.njobs, units,
                               L.ujob[UNIT_IMG]);
    });
}


// Batches of at least this many small images hide one image per wave: a
// quarter of the waves of k_hide_wave resident on the device, so that the
// walks of the images overlap.  Smaller batches (and single images) take the
// counted steps, which spread every image over many waves.
uint32_t whole_image_min() {
    const uint32_t v = hide_wave_resident() / 4u;
    return v < 1 ? 1 : v;
}

static inline unsigned step_grid(const Launch &L, uint32_t units) {
    return grid_for(L, (units + kThreads / 64 - 1) / (kThreads / 64));
}

// The step path of a hiding op: one pass with look-back, or count, scan and
// hide.  The look-back status words and ticket share the rank region.
template <bool EMBED>
static void launch_steps(const Launch &L, uint32_t units, bool one_pass) {
    uint32_t *cnt = reinterpret_cast<uint32_t *>(L.ws + L.g_status);
    uint64_t *status = reinterpret_cast<uint64_t *>(L.ws + L.g_status);
    PartWord *part = reinterpret_cast<PartWord *>(L.ws + L.g_part);
    const unsigned g = step_grid(L, units);
    if (one_pass) {
        const unsigned gc = (unsigned)std::min<uint32_t>((units + 1 + 255) / 256, 1024u);
        hipLaunchKernelGGL(k_lb_clear, dim3(gc), dim3(256), 0, L.stream, status, units);
        with_keystream(L.keystream, [&](auto K) {
            if (L.dyn)
                hipLaunchKernelGGL((k_seg_hide1<EMBED, decltype(K)::value, true>), dim3(g), dim3(kThreads), 0, L.stream,
                                   L.jobs, L.njobs, units, L.ujob[UNIT_SEG], status, part);
            else
                hipLaunchKernelGGL((k_seg_hide1<EMBED, decltype(K)::value>), dim3(g), dim3(kThreads), 0, L.stream,
                                   L.jobs, L.njobs, units, L.ujob[UNIT_SEG], status, part);
        });
    } else {
        hipLaunchKernelGGL(k_seg_count, dim3(g), dim3(kThreads), 0, L.stream, L.jobs, L.njobs, units, L.ujob[UNIT_SEG],
                           cnt);
        hipLaunchKernelGGL(k_seg_scan, dim3((unsigned)L.njobs), dim3(kScanThreads), 0, L.stream, L.jobs, cnt);
        with_keystream(L.keystream, [&](auto K) {
            if (L.dyn)
                hipLaunchKernelGGL((k_seg_hide<EMBED, decltype(K)::value, true>), dim3(g), dim3(kThreads), 0, L.stream,
                                   L.jobs, L.njobs, units, L.ujob[UNIT_SEG], cnt, part);
            else
                hipLaunchKernelGGL((k_seg_hide<EMBED, decltype(K)::value>), dim3(g), dim3(kThreads), 0, L.stream, L.jobs,
                                   L.njobs, units, L.ujob[UNIT_SEG], cnt, part);
        });
    }
}

void launch_embed(const Launch &L, uint32_t units, bool one_pass) {
    if (!units) return;
    launch_steps<true>(L, units, one_pass);
}

void launch_extract(const Launch &L, uint32_t units, bool one_pass) {
    if (!units) return;
    launch_steps<false>(L, units, one_pass);
    PartWord *part = reinterpret_cast<PartWord *>(L.ws + L.g_part);
    const uint32_t n = 2 * units;
    hipLaunchKernelGGL(k_extract_fix, dim3((n + 255) / 256), dim3(256), 0, L.stream, L.jobs, part, n, 0);
    hipLaunchKernelGGL(k_extract_fix, dim3((n + 255) / 256), dim3(256), 0, L.stream, L.jobs, part, n, 1);
}

uint64_t seg_pixels() { return kWSegPx; }
uint64_t whole_max_pixels() { return kWholeMaxPx; }

// Hiding workspace of a launch: the count / rank of every step (one pass: its
// look-back status word, then the ticket counter), then two partial-word
// records per step.
void hide_ws_layout(uint32_t units, uint64_t base, uint64_t &ranks, uint64_t &part, uint64_t &end) {
    ranks = base;
    part = (ranks + ((uint64_t)units + 1) * 8 + 255) / 256 * 256;
    end = (part + (uint64_t)units * 2 * sizeof(PartWord) + 255) / 256 * 256;
}

}  // namespace rdhei

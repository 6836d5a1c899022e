// Data hiding and extraction (Sec. III-A/B data hiding phase, decoding with
// K2).  The rotated location map decides which pixels are redundant; payload
// bit t lands in redundant pixel floor(t / rep) of the raster order, bits
// top..top-rep+1 (rep = b for EMR, b-1 for LMR), so a pixel's bit offset is
// rep times the number of redundant pixels before it: a prefix sum.
//
// Single pass over the image: each workgroup takes the next 16384-pixel
// raster segment by ticket, counts its redundant pixels, and learns the count
// before it from its predecessors by decoupled look-back (Merrill & Garland,
// "Single-pass parallel prefix scan with decoupled look-back", 2016).  Tickets
// hand segments out in order, so a workgroup only ever waits on segments
// already owned by running workgroups.  The wait is bounded: past a spin limit
// the image is flagged RDHEI_EDEVICE instead of waiting forever.
#include "device.hpp"
#include "hide4.hpp"

namespace rdhei {

constexpr int kSegLoads = 4;                                       // 16-byte loads per thread
constexpr uint64_t kSegPx = (uint64_t)kThreads * 16 * kSegLoads;   // 16384 pixels
constexpr int kWinWords = (int)((kSegPx * 7 + 127) / 128) * 4 + 8; // payload window (words)
constexpr uint32_t kSpinLimit = 1u << 24;

// status word of a segment: bit 63 = inclusive prefix ready, bit 62 =
// aggregate ready, low 62 bits = the value.
constexpr uint64_t kAgg = 1ull << 62, kInc = 1ull << 63, kValMask = kAgg - 1;

struct HideParams {
    uint32_t rep, shift;      // replaceable bits per redundant pixel, position of the lowest
    int64_t nbits;            // bits requested (resolved against the capacity)
    bool ok;
};

__device__ __forceinline__ HideParams hide_params(const Job &J) {
    const rdhei_meta *m = J.meta;
    HideParams h;
    const int b = m->b;
    h.rep = (uint32_t)(J.method == RDHEI_EMR ? b : b - 1);
    h.shift = (uint32_t)(8 - b);
    const int64_t cap = m->capacity_bits;
    h.nbits = J.nbits < 0 ? cap : J.nbits;
    h.ok = (m->status == RDHEI_OK) && h.nbits <= cap && h.rep >= 1 && h.rep <= 7;
    h.rep = uni(h.rep);
    h.shift = uni(h.shift);
    h.nbits = (int64_t)uni64((uint64_t)h.nbits);
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
    if (J.method == RDHEI_EMR) {
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
__device__ __forceinline__ void extract16(const uint32_t w[4], uint32_t rm, uint32_t rel, uint32_t rend, uint32_t *win,
                                          const Hide4 &hk, const uint32_t *T) {
    const uint32_t rep = hk.rep;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint32_t m = (rm >> (4 * q)) & 0xFu;
        const uint32_t pos = rel;
        rel += (uint32_t)__popc(m) * rep;
        if (m == 0 || pos >= rend) continue;
        if (rel <= rend) {
            const uint32_t f = (w[q] >> hk.shift) & hk.low_bytes;
            const uint32_t c = vperm(0u, f, T[m]);
            const uint32_t s = (((c >> 24) << (3u * rep)) | (((c >> 16) & 0xFFu) << (2u * rep)) |
                                (((c >> 8) & 0xFFu) << rep) | (c & 0xFFu)) << (32u - 4u * rep);
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

// Exclusive scan over the workgroup of four 16-bit counters packed in a u64
// (field k = count of load k); returns the thread's exclusive prefix per field
// and the workgroup totals per field.
__device__ __forceinline__ uint64_t block_scan4(uint64_t v, uint64_t &total, uint64_t *sh) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint64_t x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint64_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) sh[wave] = x;
    __syncthreads();
    uint64_t base = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) {
        const uint64_t t = sh[w];
        base += (w < wave) ? t : 0ull;
        tot += t;
    }
    __syncthreads();
    total = tot;
    return base + x - v;
}

// Publish a segment's aggregate, look back over its predecessors in the same
// image, publish its inclusive prefix; returns the exclusive prefix.  Run by
// all 64 lanes of one wave: each pass reads 64 predecessors at once and stops
// at the nearest one that already holds an inclusive prefix.  A status word
// carries its own value, so relaxed device-scope atomics suffice.
__device__ uint64_t look_back(uint64_t *status, uint32_t u, uint32_t first_u, uint64_t agg, bool &timed_out) {
    const int lane = threadIdx.x & 63;
    timed_out = false;
    if (u == first_u) {
        if (lane == 0) __hip_atomic_store(&status[u], kInc | agg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return 0;
    }
    if (lane == 0) __hip_atomic_store(&status[u], kAgg | agg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint64_t prefix = 0;
    int64_t base = (int64_t)u - 1;          // this pass covers base, base-1, ..., base-63
    uint32_t spins = 0;
    while (true) {
        const int64_t idx = base - lane;
        uint64_t s = kInc;                   // before the image's first segment: nothing to add
        if (idx >= (int64_t)first_u)
            s = __hip_atomic_load(&status[idx], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint64_t incl = __ballot((s & kInc) != 0);
        const uint64_t ready = __ballot((s & (kInc | kAgg)) != 0);
        const int d = incl ? __ffsll((unsigned long long)incl) - 1 : 64;   // nearest inclusive
        const uint64_t need = d >= 63 ? ~0ull : ((2ull << d) - 1);
        if ((ready & need) != need) {
            if (++spins > kSpinLimit) { timed_out = true; break; }
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        uint64_t v = (lane <= d) ? (s & kValMask) : 0ull;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        prefix += v;
        if (d < 64) break;
        base -= 64;
    }
    if (lane == 0)
        __hip_atomic_store(&status[u], kInc | (prefix + agg), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return prefix;
}

// Resets the ticket counter and the segment status words of a launch.
__global__ void k_hide_reset(uint64_t *status, uint32_t units, uint32_t *ticket) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < units) status[i] = 0;
    if (i == 0) *ticket = 0;
}

// One segment's pixels, masks and ranks.
struct SegState {
    uint4 px[kSegLoads];
    uint32_t rm[kSegLoads];
    uint64_t rank[kSegLoads];   // rank (in the image) of the thread's first redundant pixel of load k
    uint64_t seg_rank;          // redundant pixels before this segment
    uint64_t seg_count;         // redundant pixels in this segment
    uint64_t s0, s1, total;
    bool timed_out;
};

// Load, count and look back for segment `seg` (work unit u) of job J.
__device__ __forceinline__ void seg_count(const Job &J, const uint8_t *img, uint32_t u, uint32_t seg, uint64_t *status,
                                          uint64_t *sh, uint64_t *shv, SegState &S) {
    const int tid = threadIdx.x;
    S.total = (uint64_t)J.M * (uint64_t)J.N;
    S.s0 = (uint64_t)seg * kSegPx;
    S.s1 = S.s0 + kSegPx < S.total ? S.s0 + kSegPx : S.total;
#pragma unroll
    for (int k = 0; k < kSegLoads; ++k) {
        const uint64_t pos = S.s0 + (uint64_t)k * (kThreads * 16) + 16 * (uint64_t)tid;
        S.px[k] = pos < S.s1 ? load16(img, pos, S.s1) : make_uint4(0x01010101u, 0x01010101u, 0x01010101u, 0x01010101u);
    }
    uint64_t packed = 0;
#pragma unroll
    for (int k = 0; k < kSegLoads; ++k) {
        const uint64_t pos = S.s0 + (uint64_t)k * (kThreads * 16) + 16 * (uint64_t)tid;
        S.rm[k] = redundant16(J, S.px[k], pos, S.s1);
        packed |= (uint64_t)__popc(S.rm[k]) << (16 * k);
    }
    uint64_t tot;
    const uint64_t ex = block_scan4(packed, tot, sh);
    uint64_t chunk_base = 0;
#pragma unroll
    for (int k = 0; k < kSegLoads; ++k) {
        S.rank[k] = chunk_base + ((ex >> (16 * k)) & 0xFFFFu);
        chunk_base += (tot >> (16 * k)) & 0xFFFFu;
    }
    S.seg_count = uni64(chunk_base);
    if (tid < 64) {
        bool to;
        const uint64_t pre = look_back(status, u, u - seg, chunk_base, to);
        if (tid == 0) {
            shv[0] = pre;
            shv[1] = to ? 1u : 0u;
        }
    }
    __syncthreads();
    S.seg_rank = uni64(shv[0]);
    S.timed_out = uni((uint32_t)shv[1]) != 0;
#pragma unroll
    for (int k = 0; k < kSegLoads; ++k) S.rank[k] += S.seg_rank;
    __syncthreads();
}

__device__ __forceinline__ uint32_t grab_ticket(uint32_t *ticket, uint32_t *sh_t) {
    if (threadIdx.x == 0) *sh_t = atomicAdd(ticket, 1u);
    __syncthreads();
    const uint32_t u = uni(*sh_t);
    __syncthreads();
    return u;
}

// Hide the payload bits that fall in one segment.  All branches that guard a
// barrier test wave-uniform values.
__device__ __forceinline__ void embed_unit(const Job &J, const HideParams &hp, uint32_t u, uint32_t seg,
                                           uint64_t *status, uint64_t *sh, uint64_t *shv, uint32_t *win,
                                           const uint32_t *htab) {
    const int tid = threadIdx.x;
    SegState S;
    seg_count(J, J.out, u, seg, status, sh, shv, S);
    if (S.timed_out) {
        if (tid == 0) J.meta->status = RDHEI_EDEVICE;
        return;
    }
    const int64_t wstart = (int64_t)(S.seg_rank * hp.rep);
    int64_t wend = (int64_t)((S.seg_rank + S.seg_count) * hp.rep);
    if (wend > hp.nbits) wend = hp.nbits;
    if (wstart >= wend) return;
    // stage (payload XOR message keystream) for the window, 16-byte blocks, big-endian words
    const int64_t fb = wstart >> 7, lb = (wend - 1) >> 7;
    for (int64_t q = tid; q <= lb - fb; q += kThreads) {
        const uint64_t blk = (uint64_t)(fb + q);
        const uint4 mv = gload<uint4>(J.msg + 16 * blk);
        const U4 ks = stream_block(J.key, kDomainMessage, blk);
        uint32_t *wp = win + 1 + 4 * q;   // word 0 is a guard
        wp[0] = __builtin_bswap32(mv.x ^ ks.x);
        wp[1] = __builtin_bswap32(mv.y ^ ks.y);
        wp[2] = __builtin_bswap32(mv.z ^ ks.z);
        wp[3] = __builtin_bswap32(mv.w ^ ks.w);
    }
    __syncthreads();
    const Hide4 hk = hide4_params(hp);
    const int64_t wbase = fb << 7;
    const uint32_t rend = (uint32_t)(wend - wbase);
#pragma unroll
    for (int k = 0; k < kSegLoads; ++k) {
        const uint32_t rm = S.rm[k];
        const int64_t bit = (int64_t)(S.rank[k] * hp.rep);
        if (!rm || bit >= wend) continue;
        uint32_t w[4] = {S.px[k].x, S.px[k].y, S.px[k].z, S.px[k].w};
        embed16(w, rm, (uint32_t)(bit - wbase), rend, win, hk, htab);
        const uint64_t pos = S.s0 + (uint64_t)k * (kThreads * 16) + 16 * (uint64_t)tid;
        store16(J.out, pos, S.s1, make_uint4(w[0], w[1], w[2], w[3]));
    }
}

// ---- embedding -------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_embed(const Job *__restrict__ jobs, int njobs, uint32_t units,
                                                     const uint32_t *__restrict__ ujob, uint64_t *__restrict__ status,
                                                     uint32_t *__restrict__ ticket) {
    __shared__ uint64_t sh[kThreads / 64];
    __shared__ uint64_t shv[2];
    __shared__ uint32_t sh_t;
    __shared__ uint32_t win[kWinWords];
    __shared__ uint32_t htab[hide4::kWords];
    const int tid = threadIdx.x;
    stage_hide_tables(htab, tid);   // read after the ticket barrier
    while (true) {
        const uint32_t u = grab_ticket(ticket, &sh_t);
        if (u >= units) break;
        const int j = (int)uni((uint32_t)find_job<UNIT_SEG>(jobs, njobs, u, ujob));
        const Job &J = jobs[j];
        const HideParams hp = hide_params(J);
        if (!hp.ok) {
            if (tid == 0 && u == J.ubase[UNIT_SEG] && J.meta->status == RDHEI_OK) J.meta->status = RDHEI_ECAPACITY;
        } else {
            embed_unit(J, hp, u, u - J.ubase[UNIT_SEG], status, sh, shv, win, htab);
        }
        __syncthreads();
    }
}

// ---- extraction -------------------------------------------------------------------
// Message words a segment only partly owns (shared with a neighbouring
// segment, or the message's last word) go to a side record; two small passes
// clear, then OR them into place.
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
__device__ __forceinline__ uint32_t ks_word(uint64_t key, int64_t w) {
    const U4 ks = stream_block(key, kDomainMessage, (uint64_t)w >> 2);
    const uint32_t kw = (w & 3) == 0 ? ks.x : (w & 3) == 1 ? ks.y : (w & 3) == 2 ? ks.z : ks.w;
    return __builtin_bswap32(kw);
}

// Extract the payload bits of one segment.
__device__ __forceinline__ void extract_unit(const Job &J, const HideParams &hp, int j, uint32_t u, uint32_t seg,
                                             uint64_t *status, uint64_t *sh, uint64_t *shv, uint32_t *win,
                                             PartWord *part, const uint32_t *htab) {
    const int tid = threadIdx.x;
    SegState S;
    seg_count(J, J.in, u, seg, status, sh, shv, S);
    if (S.timed_out) {
        if (tid == 0) J.meta->status = RDHEI_EDEVICE;
        return;
    }
    const int64_t wstart = (int64_t)(S.seg_rank * hp.rep);
    int64_t wend = (int64_t)((S.seg_rank + S.seg_count) * hp.rep);
    if (wend > hp.nbits) wend = hp.nbits;
    if (wstart >= wend) return;
    const int64_t W0 = wstart >> 5, W1 = (wend + 31) >> 5;
    for (int64_t q = tid; q < W1 - W0 + 1; q += kThreads) win[q] = 0u;
    __syncthreads();
    const Hide4 hk = hide4_params(hp);
    const uint32_t rend = (uint32_t)(wend - 32 * W0);
#pragma unroll
    for (int k = 0; k < kSegLoads; ++k) {
        const uint32_t rm = S.rm[k];
        const int64_t bit = (int64_t)(S.rank[k] * hp.rep);
        if (!rm || bit >= wend) continue;
        const uint32_t w[4] = {S.px[k].x, S.px[k].y, S.px[k].z, S.px[k].w};
        extract16(w, rm, (uint32_t)(bit - 32 * W0), rend, win, hk, htab);
    }
    __syncthreads();
    uint32_t *msgw = reinterpret_cast<uint32_t *>(J.msg);
    // one keystream block per four message words
    const int64_t B0 = W0 >> 2, B1 = (W1 - 1) >> 2;
    for (int64_t bq = tid; bq <= B1 - B0; bq += kThreads) {
        const U4 ks = stream_block(J.key, kDomainMessage, (uint64_t)(B0 + bq));
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

__global__ __launch_bounds__(kThreads) void k_extract(const Job *__restrict__ jobs, int njobs, uint32_t units,
                                                       const uint32_t *__restrict__ ujob, uint64_t *__restrict__ status,
                                                       uint32_t *__restrict__ ticket, PartWord *__restrict__ part) {
    __shared__ uint64_t sh[kThreads / 64];
    __shared__ uint64_t shv[2];
    __shared__ uint32_t sh_t;
    __shared__ uint32_t win[kWinWords];
    __shared__ uint32_t htab[hide4::kWords];
    const int tid = threadIdx.x;
    stage_hide_tables(htab, tid);   // read after the ticket barrier
    while (true) {
        const uint32_t u = grab_ticket(ticket, &sh_t);
        if (u >= units) break;
        if (tid < 2) part[2 * u + tid].word = -1;
        const int j = (int)uni((uint32_t)find_job<UNIT_SEG>(jobs, njobs, u, ujob));
        const Job &J = jobs[j];
        const HideParams hp = hide_params(J);
        if (!hp.ok) {
            if (tid == 0 && u == J.ubase[UNIT_SEG] && J.meta->status == RDHEI_OK) J.meta->status = RDHEI_ECAPACITY;
        } else {
            extract_unit(J, hp, j, u, u - J.ubase[UNIT_SEG], status, sh, shv, win, part, htab);
        }
        __syncthreads();
    }
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
// Images of at most kSeqMaxSeg look-back segments, in batches large enough to
// fill the device, are walked by one wave each, 4096 pixels per step: the
// rank carries over in registers, the next step's pixels are loaded while the
// current one is processed, ranks inside a step come from a wave scan (DPP),
// and nothing waits on another wave.  Larger images and small batches use the
// look-back kernels above.
constexpr int kSeqMaxSeg = 64;
constexpr int kWLoads = 4;                                           // 16-byte loads per lane
constexpr uint64_t kWSegPx = 64ull * 16 * kWLoads;                   // 4096 pixels
constexpr int kWWinWords = (int)((kWSegPx * 7 + 127) / 128 + 1) * 4 + 8;

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

template <bool EMBED>
__device__ __forceinline__ void hide_image_wave(const Job &J, const HideParams &hp, uint32_t *win, const uint32_t *htab) {
    const int lane = threadIdx.x & 63;
    const uint8_t *img = EMBED ? J.out : J.in;
    const uint64_t total = (uint64_t)J.M * (uint64_t)J.N;
    const uint32_t nseg = (uint32_t)((total + kWSegPx - 1) / kWSegPx);
    const uint32_t rep = hp.rep;
    const Hide4 hk = hide4_params(hp);
    uint64_t rank = 0;
    uint32_t carry = 0;          // extraction: bits of the partial word left by the previous step
    int64_t carry_word = -1;
    uint4 nxt[kWLoads];
    wseg_load(img, 0, total < kWSegPx ? total : kWSegPx, lane, nxt);
    // embedding: the message blocks of the next step, loaded a step ahead
    // (a step needs at most 4096 * 7 bits = 224 blocks from its first one)
    uint4 mpre[4];
    auto msg_prefetch = [&](uint64_t first_blk) {
        const uint64_t nblk = (uint64_t)(hp.nbits + 127) >> 7;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint64_t blk = first_blk + (uint64_t)(lane + 64 * i);
            mpre[i] = blk < nblk ? gload<uint4>(J.msg + 16 * blk) : make_uint4(0, 0, 0, 0);
        }
    };
    if (EMBED) msg_prefetch(0);
    for (uint32_t seg = 0; seg < nseg; ++seg) {
        const uint64_t s0 = (uint64_t)seg * kWSegPx;
        const uint64_t s1 = s0 + kWSegPx < total ? s0 + kWSegPx : total;
        uint4 px[kWLoads];
#pragma unroll
        for (int k = 0; k < kWLoads; ++k) px[k] = nxt[k];
        {   // the next step's pixels (the last step reloads itself)
            const uint32_t ns = seg + 1 < nseg ? seg + 1 : seg;
            const uint64_t n0 = (uint64_t)ns * kWSegPx;
            wseg_load(img, n0, n0 + kWSegPx < total ? n0 + kWSegPx : total, lane, nxt);
        }
        uint32_t rm[kWLoads];
#pragma unroll
        for (int k = 0; k < kWLoads; ++k)
            rm[k] = redundant16(J, px[k], s0 + (uint64_t)k * 1024u + 16 * (uint64_t)lane, s1);
        // ranks: counts of loads 0, 1 and 2, 3 in 16-bit halves (at most 1024 each)
        const uint32_t c01 = (uint32_t)__popc(rm[0]) | ((uint32_t)__popc(rm[1]) << 16);
        const uint32_t c23 = (uint32_t)__popc(rm[2]) | ((uint32_t)__popc(rm[3]) << 16);
        const uint32_t i01 = wave_scan_incl(c01), i23 = wave_scan_incl(c23);
        const uint32_t t01 = uni((uint32_t)__builtin_amdgcn_readlane((int)i01, 63));
        const uint32_t t23 = uni((uint32_t)__builtin_amdgcn_readlane((int)i23, 63));
        const uint32_t e01 = i01 - c01, e23 = i23 - c23;
        const uint32_t tot0 = t01 & 0xFFFFu, tot1 = t01 >> 16, tot2 = t23 & 0xFFFFu, tot3 = t23 >> 16;
        const uint32_t lr[kWLoads] = {e01 & 0xFFFFu, tot0 + (e01 >> 16), tot0 + tot1 + (e23 & 0xFFFFu),
                                      tot0 + tot1 + tot2 + (e23 >> 16)};
        const uint32_t T = tot0 + tot1 + tot2 + tot3;
        const int64_t wstart = (int64_t)(rank * rep);
        if (wstart >= hp.nbits) break;
        int64_t wend = (int64_t)((rank + T) * rep);
        if (wend > hp.nbits) wend = hp.nbits;
        rank += T;
        if (T > 0 && EMBED) {
            // window bits relative to the first staged 16-byte block (the prefetch base)
            const int64_t fb = wstart >> 7, lb = (wend - 1) >> 7;
            const uint32_t off0 = (uint32_t)(wstart - (fb << 7)), rend = (uint32_t)(wend - (fb << 7));
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int64_t q = lane + 64 * i;
                if (q > lb - fb) continue;
                const uint4 mv = mpre[i];
                const U4 ks = stream_block(J.key, kDomainMessage, (uint64_t)(fb + q));
                *reinterpret_cast<uint4 *>(win + 4 + 4 * q) =
                    make_uint4(__builtin_bswap32(mv.x ^ ks.x), __builtin_bswap32(mv.y ^ ks.y),
                               __builtin_bswap32(mv.z ^ ks.z), __builtin_bswap32(mv.w ^ ks.w));
            }
            msg_prefetch((rank * rep) >> 7);   // rank already counts this step
            wave_sync();
#pragma unroll
            for (int k = 0; k < kWLoads; ++k) {
                const uint32_t rel = off0 + lr[k] * rep;
                if (!rm[k] || rel >= rend) continue;
                uint32_t w[4] = {px[k].x, px[k].y, px[k].z, px[k].w};
                embed16(w, rm[k], rel, rend, win + 3, hk, htab);   // word 0 of the window is a guard
                gstore<uint4>(J.out + s0 + (uint64_t)k * 1024u + 16 * (uint64_t)lane, make_uint4(w[0], w[1], w[2], w[3]));
            }
            wave_sync();
        } else if (T > 0) {
            const int64_t W0 = wstart >> 5, W1 = (wend + 31) >> 5;
            const uint32_t off0 = (uint32_t)(wstart & 31), rend = (uint32_t)(wend - 32 * W0);
            for (int64_t q = lane; q < W1 - W0 + 1; q += 64) win[q] = (q == 0 && carry_word == W0) ? carry : 0u;
            wave_sync();
#pragma unroll
            for (int k = 0; k < kWLoads; ++k) {
                const uint32_t rel = off0 + lr[k] * rep;
                if (!rm[k] || rel >= rend) continue;
                const uint32_t w[4] = {px[k].x, px[k].y, px[k].z, px[k].w};
                extract16(w, rm[k], rel, rend, win, hk, htab);
            }
            wave_sync();
            // complete words go out; a trailing partial word waits for the next step
            const bool partial = (wend & 31) != 0;
            const int64_t nstore = partial ? (W1 - 1 - W0) : (W1 - W0);
            uint32_t *msgw = reinterpret_cast<uint32_t *>(J.msg);
            if (nstore > 0) {   // one keystream block per four message words
                const int64_t B0 = W0 >> 2, B1 = (W0 + nstore - 1) >> 2;
                for (int64_t bq = lane; bq <= B1 - B0; bq += 64) {
                    const U4 ks = stream_block(J.key, kDomainMessage, (uint64_t)(B0 + bq));
                    const uint32_t kw[4] = {ks.x, ks.y, ks.z, ks.w};
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int64_t w = 4 * (B0 + bq) + i;
                        if (w >= W0 && w < W0 + nstore) gstore<uint32_t>(msgw + w, __builtin_bswap32(win[w - W0]) ^ kw[i]);
                    }
                }
            }
            carry_word = partial ? W1 - 1 : -1;
            carry = partial ? uni(win[W1 - 1 - W0]) : 0u;
            wave_sync();
        }
    }
    if (!EMBED && carry_word >= 0 && lane == 0) {
        // the message's last word: bits past nbits are stored as zero
        const uint32_t own = be_mask(carry_word, 0, hp.nbits);
        gstore<uint32_t>(reinterpret_cast<uint32_t *>(J.msg) + carry_word,
                         __builtin_bswap32((carry ^ ks_word(J.key, carry_word)) & own));
    }
}

// One wave per workgroup, one image per wave (a grid-stride loop when the grid
// is capped).
template <bool EMBED>
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
            hide_image_wave<EMBED>(J, hp, win, htab);
        }
        wave_sync();
    }
}

// ---- launchers ---------------------------------------------------------------------
static inline unsigned grid_for(const Launch &L, uint32_t units) {
    uint32_t g = units;
    if (L.max_grid > 0 && g > (uint32_t)L.max_grid) g = (uint32_t)L.max_grid;
    return g ? g : 1;
}

void launch_hide_images(const Launch &L, uint32_t units, bool embed) {
    if (!units) return;
    const unsigned g = grid_for(L, units);
    if (embed)
        hipLaunchKernelGGL(k_hide_wave<true>, dim3(g), dim3(64), 0, L.stream, L.jobs, L.njobs, units, L.ujob[UNIT_IMG]);
    else
        hipLaunchKernelGGL(k_hide_wave<false>, dim3(g), dim3(64), 0, L.stream, L.jobs, L.njobs, units, L.ujob[UNIT_IMG]);
}

int seq_max_segments() { return kSeqMaxSeg; }

// Batches of at least this many small images hide one image per wave: a
// quarter of the waves of k_hide_wave resident on the device, so that the
// walks of the images overlap.  Smaller batches (and single images) take the
// segment path, whose latency per image is a few segments deep.
uint32_t whole_image_min() {
    static uint32_t v = 0;
    if (!v) {
        int dev = 0, cus = 0, per_cu = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_hide_wave<true>, 64, 0) != hipSuccess || per_cu < 1)
            per_cu = 1;
        v = (uint32_t)(cus > 0 ? cus : 1) * (uint32_t)per_cu / 4u;
        if (v < 1) v = 1;
    }
    return v;
}

void launch_embed(const Launch &L, uint32_t units) {
    if (!units) return;
    uint64_t *status = reinterpret_cast<uint64_t *>(L.ws + L.g_status);
    uint32_t *ticket = reinterpret_cast<uint32_t *>(L.ws + L.g_ticket);
    hipLaunchKernelGGL(k_hide_reset, dim3((units + 255) / 256), dim3(256), 0, L.stream, status, units, ticket);
    hipLaunchKernelGGL(k_embed, dim3(grid_for(L, units)), dim3(kThreads), 0, L.stream, L.jobs, L.njobs, units,
                       L.ujob[UNIT_SEG], status, ticket);
}

void launch_extract(const Launch &L, uint32_t units) {
    if (!units) return;
    uint64_t *status = reinterpret_cast<uint64_t *>(L.ws + L.g_status);
    uint32_t *ticket = reinterpret_cast<uint32_t *>(L.ws + L.g_ticket);
    PartWord *part = reinterpret_cast<PartWord *>(L.ws + L.g_part);
    hipLaunchKernelGGL(k_hide_reset, dim3((units + 255) / 256), dim3(256), 0, L.stream, status, units, ticket);
    hipLaunchKernelGGL(k_extract, dim3(grid_for(L, units)), dim3(kThreads), 0, L.stream, L.jobs, L.njobs, units,
                       L.ujob[UNIT_SEG], status, ticket, part);
    const uint32_t n = 2 * units;
    hipLaunchKernelGGL(k_extract_fix, dim3((n + 255) / 256), dim3(256), 0, L.stream, L.jobs, part, n, 0);
    hipLaunchKernelGGL(k_extract_fix, dim3((n + 255) / 256), dim3(256), 0, L.stream, L.jobs, part, n, 1);
}

uint64_t seg_pixels() { return kSegPx; }

// Launch-wide hiding workspace: status words, ticket, partial-word records.
void hide_ws_layout(uint32_t units, uint64_t base, uint64_t &status, uint64_t &ticket, uint64_t &part, uint64_t &end) {
    status = base;
    ticket = (status + (uint64_t)units * 8 + 255) / 256 * 256;
    part = ticket + 256;
    end = (part + (uint64_t)units * 2 * sizeof(PartWord) + 255) / 256 * 256;
}

}  // namespace rdhei

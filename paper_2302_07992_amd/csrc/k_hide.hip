// Data hiding and extraction (Sec. III-A/B data hiding phase, decoding with
// K2).  The rotated location map decides which pixels are redundant; payload
// bit t lands in redundant pixel floor(t / rep) of the raster order, bits
// top..top-rep+1 (rep = b for EMR, b-1 for LMR), so a pixel's bit offset is
// rep times the number of redundant pixels before it: a prefix sum.
//
// Each workgroup walks one raster segment chunk by chunk (4096 pixels, 16 per
// thread) with a workgroup scan; segments of one image get their starting
// ranks from a count pass and a per-image scan.
#include "device.hpp"

namespace rdhei {

constexpr int kSegChunks = 64;                       // 64 chunks = 262144 pixels
constexpr uint64_t kSegPx = (uint64_t)kSegChunks * kChunk;
constexpr int kWinWords = (kChunk * 7 + 127) / 128 * 4 + 8;   // payload window of one chunk

struct HideParams {
    uint32_t rep, shift;      // replaceable bits per redundant pixel, position of the lowest
    int64_t nbits;            // bits requested (already resolved against the capacity)
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
    h.ok = (m->status == RDHEI_OK) && h.nbits <= cap;
    return h;
}

// 16 pixels starting at raster index pos (multiple of 16) of an image of
// `total` pixels; pixels past the end read as 0x01 (never redundant).
__device__ __forceinline__ uint4 load16(const uint8_t *img, uint64_t pos, uint64_t total) {
    if (pos + 16 <= total) return *reinterpret_cast<const uint4 *>(img + pos);
    uint32_t w[4] = {0x01010101u, 0x01010101u, 0x01010101u, 0x01010101u};
    for (int k = 0; k < 16; ++k)
        if (pos + k < total) w[k >> 2] = (w[k >> 2] & ~(0xFFu << (8 * (k & 3)))) | ((uint32_t)img[pos + k] << (8 * (k & 3)));
    return make_uint4(w[0], w[1], w[2], w[3]);
}

__device__ __forceinline__ void store16(uint8_t *img, uint64_t pos, uint64_t total, uint4 v) {
    if (pos + 16 <= total) { *reinterpret_cast<uint4 *>(img + pos) = v; return; }
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
    for (int k = 0; k < 16; ++k)
        if (pos + k < total) img[pos + k] = (uint8_t)(w[k >> 2] >> (8 * (k & 3)));
}

// Redundancy mask of 16 pixels: bit k set when pixel pos+k is labelled 0.
__device__ __forceinline__ uint32_t redundant16(const Job &J, uint4 px, uint64_t pos, uint64_t total) {
    uint32_t m = 0;
    if (J.method == RDHEI_EMR) {
        const uint32_t w[4] = {px.x, px.y, px.z, px.w};
#pragma unroll
        for (int k = 0; k < 16; ++k) m |= ((~(w[k >> 2] >> (8 * (k & 3)))) & 1u) << k;
    } else {
        const uint32_t be = ((uint32_t)J.lbits[pos >> 3] << 8) | (pos + 8 < total ? J.lbits[(pos >> 3) + 1] : 0xFFu);
#pragma unroll
        for (int k = 0; k < 16; ++k) m |= ((~(be >> (15 - k))) & 1u) << k;
    }
    if (pos + 16 > total) m &= (total > pos) ? ((1u << (uint32_t)(total - pos)) - 1u) : 0u;
    return m;
}

__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t &total, uint32_t *sh) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) sh[wave] = x;
    __syncthreads();
    uint32_t base = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) {
        const uint32_t t = sh[w];
        base += (w < wave) ? t : 0u;
        tot += t;
    }
    __syncthreads();
    total = tot;
    return base + x - v;
}

// ---- count pass: redundant pixels per segment (images with > 1 segment) ----
__global__ __launch_bounds__(kThreads) void k_seg_count(const Job *__restrict__ jobs, int njobs,
                                                         uint8_t *__restrict__ ws, uint32_t units,
    const uint32_t *__restrict__ ujob) {
    __shared__ uint32_t sh[kThreads / 64];
    for (uint32_t u = blockIdx.x; u < units; u += gridDim.x) {
        const int j = find_job<UNIT_SEG>(jobs, njobs, u, ujob);
        const Job &J = jobs[j];
        if (J.nseg <= 1) continue;
        const uint32_t seg = u - J.ubase[UNIT_SEG];
        const uint64_t total = (uint64_t)J.M * (uint64_t)J.N;
        const uint64_t s0 = (uint64_t)seg * kSegPx;
        const uint64_t s1 = s0 + kSegPx < total ? s0 + kSegPx : total;
        uint32_t cnt = 0;
        for (uint64_t pos = s0 + 16 * threadIdx.x; pos < s1; pos += kChunk) {
            const uint4 px = load16(J.in ? J.in : J.out, pos, total);
            cnt += __popc(redundant16(J, px, pos, total));
        }
        uint32_t tot;
        block_excl_scan(cnt, tot, sh);
        if (threadIdx.x == 0) reinterpret_cast<uint32_t *>(ws + J.ws_seg)[seg] = tot;
    }
}

// ---- per-image exclusive scan of the segment counts ---------------------------
// Also clears the message words that two segments share (both OR into them).
__global__ __launch_bounds__(kThreads) void k_seg_scan(const Job *__restrict__ jobs, int njobs,
                                                        uint8_t *__restrict__ ws, int clear_shared) {
    __shared__ uint32_t sh[kThreads / 64];
    for (int j = blockIdx.x; j < njobs; j += gridDim.x) {
        const Job &J = jobs[j];
        if (J.nseg <= 1) continue;
        const HideParams hp = hide_params(J);
        uint32_t *cnt = reinterpret_cast<uint32_t *>(ws + J.ws_seg);
        uint32_t *off = cnt + J.nseg;
        uint32_t carry = 0;
        for (int base = 0; base < J.nseg; base += kThreads) {
            const int s = base + threadIdx.x;
            const uint32_t c = s < J.nseg ? cnt[s] : 0u;
            uint32_t tot;
            const uint32_t ex = block_excl_scan(c, tot, sh);
            if (s < J.nseg) {
                off[s] = carry + ex;
                const int64_t B = (int64_t)hp.rep * (int64_t)(carry + ex);
                if (clear_shared && hp.ok && s > 0 && (B & 31) && B < hp.nbits)
                    reinterpret_cast<uint32_t *>(J.msg)[B >> 5] = 0u;
            }
            carry += tot;
        }
    }
}

// ---- embedding -------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_embed(const Job *__restrict__ jobs, int njobs,
                                                     uint8_t *__restrict__ ws, uint32_t units,
    const uint32_t *__restrict__ ujob) {
    __shared__ uint32_t sh[kThreads / 64];
    __shared__ uint32_t win[kWinWords];
    const int tid = threadIdx.x;
    for (uint32_t u = blockIdx.x; u < units; u += gridDim.x) {
        const int j = find_job<UNIT_SEG>(jobs, njobs, u, ujob);
        const Job &J = jobs[j];
        const HideParams hp = hide_params(J);
        if (!hp.ok) {
            if (tid == 0 && u == J.ubase[UNIT_SEG] && J.meta->status == RDHEI_OK) J.meta->status = RDHEI_ECAPACITY;
            continue;
        }
        const uint32_t seg = u - J.ubase[UNIT_SEG];
        const uint64_t total = (uint64_t)J.M * (uint64_t)J.N;
        const uint64_t s0 = (uint64_t)seg * kSegPx;
        const uint64_t s1 = s0 + kSegPx < total ? s0 + kSegPx : total;
        uint64_t rank = J.nseg > 1 ? reinterpret_cast<const uint32_t *>(ws + J.ws_seg)[J.nseg + seg] : 0u;
        if ((int64_t)(rank * hp.rep) >= hp.nbits) continue;
        uint8_t *img = J.out;
        for (uint64_t c0 = s0; c0 < s1; c0 += kChunk) {
            const uint64_t pos = c0 + 16 * (uint64_t)tid;
            const bool mine = pos < s1;
            const uint4 px = mine ? load16(img, pos, s1) : make_uint4(0x01010101u, 0x01010101u, 0x01010101u, 0x01010101u);
            const uint32_t rm = mine ? redundant16(J, px, pos, s1) : 0u;
            uint32_t tot;
            const uint32_t ex = block_excl_scan(__popc(rm), tot, sh);
            const int64_t wstart = (int64_t)(rank * hp.rep);
            int64_t wend = (int64_t)((rank + tot) * hp.rep);
            if (wend > hp.nbits) wend = hp.nbits;
            if (wstart >= hp.nbits) break;
            if (tot == 0) continue;
            // stage payload XOR message keystream, 16-byte blocks, big-endian words
            const int64_t fb = wstart >> 7, lb = (wend - 1) >> 7;
            if (tid <= lb - fb) {
                const uint64_t blk = (uint64_t)(fb + tid);
                const uint4 mv = *reinterpret_cast<const uint4 *>(J.msg + 16 * blk);
                const U4 ks = stream_block(J.key, kDomainMessage, blk);
                uint32_t *wp = win + 4 * tid;
                wp[0] = __builtin_bswap32(mv.x ^ ks.x);
                wp[1] = __builtin_bswap32(mv.y ^ ks.y);
                wp[2] = __builtin_bswap32(mv.z ^ ks.z);
                wp[3] = __builtin_bswap32(mv.w ^ ks.w);
            }
            __syncthreads();
            if (mine && rm) {
                int64_t bit = (int64_t)((rank + ex) * hp.rep);
                uint32_t w[4] = {px.x, px.y, px.z, px.w};
                const uint32_t top = hp.shift + hp.rep - 1;
#pragma unroll
                for (int k = 0; k < 16; ++k) {
                    if (((rm >> k) & 1u) && bit < wend) {
                        const int64_t rel = bit - (fb << 7);
                        const uint32_t wi = (uint32_t)(rel >> 5), sb = (uint32_t)(rel & 31);
                        const uint64_t v64 = ((uint64_t)win[wi] << 32) | win[wi + 1];
                        const uint32_t val = (uint32_t)((v64 << sb) >> (64 - hp.rep));
                        const int64_t left = wend - bit;
                        const uint32_t take = left < (int64_t)hp.rep ? (uint32_t)left : hp.rep;
                        const uint32_t wmask = ((1u << take) - 1u) << (top + 1 - take);
                        const uint32_t pv = (w[k >> 2] >> (8 * (k & 3))) & 0xFFu;
                        const uint32_t nv = (pv & ~wmask) | ((val << hp.shift) & wmask);
                        w[k >> 2] = (w[k >> 2] & ~(0xFFu << (8 * (k & 3)))) | (nv << (8 * (k & 3)));
                        bit += hp.rep;
                    }
                }
                store16(img, pos, s1, make_uint4(w[0], w[1], w[2], w[3]));
            }
            rank += tot;
            __syncthreads();
        }
    }
}

// ---- extraction -----------------------------------------------------------------
// Store one finished message word (big-endian bit order in `be`), XORed with the
// message keystream; `own` selects the bits this workgroup produced (the rest
// is stored as zero).  Words two segments share are ORed into memory the scan
// pass cleared.
__device__ __forceinline__ void put_word(const Job &J, int64_t w, uint32_t be, uint32_t own, bool shared) {
    const U4 ks = stream_block(J.key, kDomainMessage, (uint64_t)w >> 2);
    const uint32_t kw = (w & 3) == 0 ? ks.x : (w & 3) == 1 ? ks.y : (w & 3) == 2 ? ks.z : ks.w;
    const uint32_t v = (be ^ __builtin_bswap32(kw)) & own;
    uint32_t *dst = reinterpret_cast<uint32_t *>(J.msg) + w;
    if (shared) atomicOr(dst, __builtin_bswap32(v));
    else *dst = __builtin_bswap32(v);
}

// mask of BE bits [lo, hi) of word w (bit 0 of the stream = bit 31 of the word)
__device__ __forceinline__ uint32_t be_mask(int64_t w, int64_t lo, int64_t hi) {
    int64_t a = lo - 32 * w, b = hi - 32 * w;
    if (a < 0) a = 0;
    if (b > 32) b = 32;
    if (b <= a) return 0u;
    const uint32_t upto_b = b >= 32 ? 0xFFFFFFFFu : ~(0xFFFFFFFFu >> b);
    const uint32_t upto_a = a == 0 ? 0u : ~(0xFFFFFFFFu >> a);
    return upto_b & ~upto_a;
}

__global__ __launch_bounds__(kThreads) void k_extract(const Job *__restrict__ jobs, int njobs,
                                                       uint8_t *__restrict__ ws, uint32_t units,
    const uint32_t *__restrict__ ujob) {
    __shared__ uint32_t sh[kThreads / 64];
    __shared__ uint32_t win[kWinWords];
    const int tid = threadIdx.x;
    for (uint32_t u = blockIdx.x; u < units; u += gridDim.x) {
        const int j = find_job<UNIT_SEG>(jobs, njobs, u, ujob);
        const Job &J = jobs[j];
        const HideParams hp = hide_params(J);
        if (!hp.ok) {
            if (tid == 0 && u == J.ubase[UNIT_SEG] && J.meta->status == RDHEI_OK) J.meta->status = RDHEI_ECAPACITY;
            continue;
        }
        const uint32_t seg = u - J.ubase[UNIT_SEG];
        const uint64_t total = (uint64_t)J.M * (uint64_t)J.N;
        const uint64_t s0 = (uint64_t)seg * kSegPx;
        const uint64_t s1 = s0 + kSegPx < total ? s0 + kSegPx : total;
        uint64_t rank = J.nseg > 1 ? reinterpret_cast<const uint32_t *>(ws + J.ws_seg)[J.nseg + seg] : 0u;
        const int64_t seg_start = (int64_t)(rank * hp.rep);
        if (seg_start >= hp.nbits) continue;
        // the segment's bit range ends where the next segment's begins (or at nbits)
        int64_t seg_end = hp.nbits;
        if (J.nseg > 1 && (int)seg + 1 < J.nseg) {
            const int64_t nx = (int64_t)hp.rep * reinterpret_cast<const uint32_t *>(ws + J.ws_seg)[J.nseg + seg + 1];
            if (nx < seg_end) seg_end = nx;
        }
        const bool shared_start = seg > 0 && (seg_start & 31);
        const bool shared_end = (seg_end & 31) && seg_end < hp.nbits;
        uint32_t carry = 0;           // bits of the partial word left by the previous chunk
        int64_t carry_word = -1;
        for (uint64_t c0 = s0; c0 < s1; c0 += kChunk) {
            const uint64_t pos = c0 + 16 * (uint64_t)tid;
            const bool mine = pos < s1;
            const uint4 px = mine ? load16(J.in, pos, s1) : make_uint4(0x01010101u, 0x01010101u, 0x01010101u, 0x01010101u);
            const uint32_t rm = mine ? redundant16(J, px, pos, s1) : 0u;
            uint32_t tot;
            const uint32_t ex = block_excl_scan(__popc(rm), tot, sh);
            const int64_t wstart = (int64_t)(rank * hp.rep);
            int64_t wend = (int64_t)((rank + tot) * hp.rep);
            if (wend > hp.nbits) wend = hp.nbits;
            if (wstart >= hp.nbits) break;
            if (tot == 0) continue;
            const int64_t W0 = wstart >> 5, W1 = (wend + 31) >> 5;
            for (int k = tid; k < W1 - W0 + 2; k += kThreads) win[k] = (k == 0 && carry_word == W0) ? carry : 0u;
            __syncthreads();
            if (mine && rm) {
                int64_t bit = (int64_t)((rank + ex) * hp.rep);
                const uint32_t w[4] = {px.x, px.y, px.z, px.w};
                int64_t cw = (bit >> 5) - W0;            // current LDS word
                uint32_t nacc = (uint32_t)(bit & 31);    // bits already in acc (alignment)
                uint64_t acc = 0;
#pragma unroll
                for (int k = 0; k < 16; ++k) {
                    if (((rm >> k) & 1u) && bit < wend) {
                        const uint32_t pv = (w[k >> 2] >> (8 * (k & 3))) & 0xFFu;
                        const int64_t left = wend - bit;
                        const uint32_t take = left < (int64_t)hp.rep ? (uint32_t)left : hp.rep;
                        const uint32_t val = (pv >> (hp.shift + hp.rep - take)) & ((1u << take) - 1u);
                        acc |= (uint64_t)val << (64 - nacc - take);
                        nacc += take;
                        bit += take;
                        if (nacc >= 32) {
                            atomicOr(&win[cw], (uint32_t)(acc >> 32));
                            ++cw;
                            acc <<= 32;
                            nacc -= 32;
                        }
                    }
                }
                if (nacc) atomicOr(&win[cw], (uint32_t)(acc >> 32));
            }
            __syncthreads();
            // words W0 .. W1-1; the last stays in LDS when the next chunk continues it
            const bool last_partial = (wend & 31) != 0;
            const int64_t nstore = last_partial ? (W1 - 1 - W0) : (W1 - W0);
            for (int64_t k = tid; k < nstore; k += kThreads) {
                const int64_t w = W0 + k;
                const bool sh_w = (w == (seg_start >> 5)) && shared_start;
                put_word(J, w, win[k], sh_w ? be_mask(w, seg_start, seg_end) : 0xFFFFFFFFu, sh_w);
            }
            if (last_partial) {
                carry = win[W1 - 1 - W0];
                carry_word = W1 - 1;
            } else {
                carry_word = -1;
            }
            rank += tot;
            __syncthreads();
        }
        // flush the final partial word of the segment
        if (carry_word >= 0 && tid == 0) {
            const int64_t w = carry_word;
            const bool sh_w = (w == (seg_start >> 5) && shared_start) || shared_end;
            put_word(J, w, carry, be_mask(w, seg_start, seg_end), sh_w);
        }
        __syncthreads();
    }
}

// ---- launchers ---------------------------------------------------------------------
static inline unsigned grid_for(const Launch &L, uint32_t units) {
    uint32_t g = units;
    if (L.max_grid > 0 && g > (uint32_t)L.max_grid) g = (uint32_t)L.max_grid;
    return g ? g : 1;
}

void launch_seg_count(const Launch &L, uint32_t units) {
    const uint32_t *UJ = L.ujob[UNIT_SEG];
    if (units) hipLaunchKernelGGL(k_seg_count, dim3(grid_for(L, units)), dim3(kThreads), 0, L.stream, L.jobs, L.njobs, L.ws, units, UJ);
}
void launch_seg_scan(const Launch &L, int clear_shared) {
    if (L.njobs) hipLaunchKernelGGL(k_seg_scan, dim3(grid_for(L, (uint32_t)L.njobs)), dim3(kThreads), 0, L.stream, L.jobs, L.njobs, L.ws, clear_shared);
}
void launch_embed(const Launch &L, uint32_t units) {
    const uint32_t *UJ = L.ujob[UNIT_SEG];
    if (units) hipLaunchKernelGGL(k_embed, dim3(grid_for(L, units)), dim3(kThreads), 0, L.stream, L.jobs, L.njobs, L.ws, units, UJ);
}
void launch_extract(const Launch &L, uint32_t units) {
    const uint32_t *UJ = L.ujob[UNIT_SEG];
    if (units) hipLaunchKernelGGL(k_extract, dim3(grid_for(L, units)), dim3(kThreads), 0, L.stream, L.jobs, L.njobs, L.ws, units, UJ);
}

uint64_t seg_pixels() { return kSegPx; }

}  // namespace rdhei

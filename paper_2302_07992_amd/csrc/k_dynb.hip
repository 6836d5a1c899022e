// Per-tile b: for each 64x64 tile, the counts Z_b(t) (b = 2..7) of pixels
// (other than those of image column 0) whose b MSBs equal their left
// neighbour's -- for a tile's first column the neighbour lies in the tile to
// the left --, the tile's b_t (first b reaching the largest b * Z_b(t)) and
// the image's capacity, sum of b_t * Z_{b_t}(t): the choice and capacity of
// the dynamic-b variant (one b per tile, the conclusion's suggestion).  Reads
// 1 B/px (plus the byte left of each tile row) and writes one byte per tile.
#include "device.hpp"

namespace rdhei {

__global__ void k_tile_b_zero(int64_t *__restrict__ cap, int njobs) {
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < njobs) cap[i] = 0;
}

// One workgroup per tile (grid-stride): thread (r, g) reads row r, columns
// 16g..16g+15.  Per pixel, c = min(max(lambda, 1), 7) - 1 for lambda = the
// number of leading bits shared with the left neighbour, so that
// Z_b = #(c >= b - 1); each lane counts c in 8-bit fields of a 64-bit word (at
// most 16 per field), the wave adds the seven counts with DPP scans.
__global__ __launch_bounds__(kThreads) void k_tile_b(const TileBJob *__restrict__ jobs, int njobs, uint32_t tiles,
                                                      uint8_t *__restrict__ tile_b, int64_t *__restrict__ cap) {
    constexpr int kW = kThreads / 64;
    __shared__ uint32_t part[kW][8];
    const int tid = (int)threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r = tid >> 2, g = tid & 3;
    for (uint32_t t = blockIdx.x; t < tiles; t += gridDim.x) {
        int lo = 0, hi = njobs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (jobs[mid].tile_first <= t) lo = mid; else hi = mid - 1;
        }
        const TileBJob &J = jobs[lo];
        const uint32_t lt = t - J.tile_first, tpr = (uint32_t)J.N / kTile;
        const uint32_t ty = lt / tpr, tx = lt % tpr;
        const uint8_t *row = J.img + (uint64_t)(ty * kTile + r) * (uint64_t)J.N + tx * kTile + 16 * g;
        const uint4 v = gload<uint4>(row);
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
        // byte 15 of the segment to the left in the same tile row (lane - 1 of
        // the quad); for the tile's first column, the byte left of the tile
        uint32_t from_left = qperm<0x90>(v.w >> 24);
        if (g == 0) from_left = tx > 0 ? (uint32_t)gload<uint8_t>(row - 1) : 0u;
        uint64_t acc = 0;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const uint32_t x = (w[k >> 2] >> (8 * (k & 3))) & 0xFFu;
            const uint32_t left = k == 0 ? from_left : (w[(k - 1) >> 2] >> (8 * ((k - 1) & 3))) & 0xFFu;
            const uint32_t lam = __clz(((x ^ left) << 24) | 0x00800000u);   // 0..8
            const uint32_t c = (lam < 7u ? (lam > 1u ? lam : 1u) : 7u) - 1u;
            if (k > 0 || g > 0 || tx > 0) acc += 1ull << (8 * c);           // image column 0 has no left pixel
        }
#pragma unroll
        for (int c = 0; c < 7; ++c) {
            const uint32_t n = wave_scan_incl((uint32_t)(acc >> (8 * c)) & 0xFFu);
            if (lane == 63) part[wave][c] = n;
        }
        __syncthreads();
        if (tid == 0) {
            uint32_t h[7];
#pragma unroll
            for (int c = 0; c < 7; ++c) h[c] = part[0][c] + part[1][c] + part[2][c] + part[3][c];
            // Z_b = #(c >= b - 1), b = 2..7; first b with the largest b * Z_b
            uint32_t zb[8] = {0, 0, 0, 0, 0, 0, 0, h[6]};
            for (int b = 6; b >= 2; --b) zb[b] = zb[b + 1] + h[b - 1];
            uint32_t best_b = 2, best = 2u * zb[2];
            for (uint32_t b = 3; b <= 7; ++b)
                if (b * zb[b] > best) {
                    best = b * zb[b];
                    best_b = b;
                }
            tile_b[t] = (uint8_t)best_b;
            atomicAdd(reinterpret_cast<unsigned long long *>(cap + lo), (unsigned long long)best);
        }
        __syncthreads();
    }
}

void launch_tile_b(const TileBJob *jobs, int njobs, uint32_t tiles, uint8_t *tile_b, int64_t *cap, hipStream_t st) {
    hipLaunchKernelGGL(k_tile_b_zero, dim3((unsigned)((njobs + 255) / 256)), dim3(256), 0, st, cap, njobs);
    if (!tiles) return;
    const uint32_t g = tiles < 16384u ? tiles : 16384u;
    hipLaunchKernelGGL(k_tile_b, dim3(g), dim3(kThreads), 0, st, jobs, njobs, tiles, tile_b, cap);
}

}  // namespace rdhei

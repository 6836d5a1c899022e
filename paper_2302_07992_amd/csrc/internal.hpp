// Internal declarations shared by the HIP translation units of librdhei.
// Device code for gfx950 (wave64).  Nothing here is part of the C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>
#include <vector>

#include "../../include/rdhei.h"

namespace rdhei {

// Fast-path tile: 64 x 64 pixels, one 256-thread workgroup per tile.
constexpr int kTileLog = 6;
constexpr int kTile = 1 << kTileLog;
constexpr int kThreads = 256;

// Per-tile record of in-tile rotation codes, levels 1..kTileLog, 2 bits per
// block, row-major per level.  Level m starts at kCodeOff[m].
__host__ __device__ constexpr int code_bytes_level(int m) { return ((kTile >> m) * (kTile >> m) + 3) / 4; }
__host__ __device__ constexpr int code_off(int m) {
    int off = 0;
    for (int k = 1; k < m; ++k) off += code_bytes_level(k);
    return off;
}
constexpr int kCodeRecord = (code_off(kTileLog + 1) + 15) / 16 * 16;   // 352 bytes for 64 x 64

// Statistics of an image: Z_b for b = 2..8 (pixels whose leading-shared-bit
// count lambda is at least b) + 1 pad word, in stat_slots() copies that
// workgroups add into by turns (spreads the atomics of a large image), then
// the image's Z as 64-bit values for the host.
constexpr int kStatWords = 8;

// Work-unit kinds (how a batch is cut into workgroup-sized pieces).
// Tiles, tile rows (LMR recovery), hiding steps, whole images, and band
// pairs (tile rows 2p, 2p + 1: encryption and EMR recovery go by 2x2 quads).
enum UnitKind { UNIT_TILE = 0, UNIT_BAND = 1, UNIT_SEG = 2, UNIT_IMG = 3, UNIT_QROW = 4, UNIT_KINDS = 5 };

// Keystream families (the values of RDHEI_OPT_KEYSTREAM).  Kernels that draw
// from the keystream are instantiated once per family.
constexpr int kKsPhilox = RDHEI_KEYSTREAM_PHILOX;
constexpr int kKsChaCha20 = RDHEI_KEYSTREAM_CHACHA20;

// Calls f(std::integral_constant<int, KS>{}) for keystream family ks.
template <typename F>
inline void with_keystream(int ks, F &&f) {
    if (ks == kKsChaCha20) f(std::integral_constant<int, kKsChaCha20>{});
    else f(std::integral_constant<int, kKsPhilox>{});
}

// Tile-map entries hold destination tile coordinates in 14 bits each, so the
// tiled path takes images of at most this many tiles along each side.
constexpr int kTmapMaxTiles = 1 << 14;

// Encryption and EMR recovery cut band pairs into segments of at most
// Job::qseg 2x2 tile quads (one work unit each); kQuadSeg is the default, the
// autotuner may choose another length per plan (1..kQuadSegMax).
constexpr int kQuadSeg = 4;
constexpr int kQuadSegMax = 64;

// Device-side descriptor of one image of a launch.
struct Job {
    const uint8_t *in;
    uint8_t *out;
    uint8_t *msg;
    rdhei_meta *meta;
    const uint8_t *lbits;     // LMR: rotated location-map bit plane (encrypted domain)
    const uint8_t *etabits;   // LMR: rotated first-MSB bit plane (encrypted domain)
    const uint8_t *stream;    // LMR encrypt: map stream for the MSB plane
    uint8_t *btab;            // DEMR: b of every tile, encrypted-tile order (caller's)
    uint64_t key;
    uint64_t nonce;           // keystream nonce (encryption: the caller's; other ops read meta->nonce)
    int64_t nbits;            // embed/extract request (< 0: capacity)
    int64_t stream_bits;      // LMR encrypt: stream length in bits
    int32_t M, N;
    int32_t method;           // RDHEI_EMR / RDHEI_LMR
    int32_t min_level;        // 1 (EMR) or 4 (LMR)
    int32_t max_level;        // n = floor(log2 min(M, N))
    int32_t fixed_b;          // > 0: b chosen on the host (LMR); 0: read meta->b
    int32_t fast;             // 1: tiled path; 0: per-pixel path
    int32_t tiles_x, tiles_y;
    int32_t nseg;             // hiding / extraction steps of seg_pixels() raster pixels
    int32_t nonce_meta;       // 1: the keystream nonce comes from meta->nonce (device)
    int32_t qseg;             // 2x2 tile quads per work unit of encryption / EMR recovery
    uint32_t ubase[UNIT_KINDS];
    uint32_t ucount[UNIT_KINDS];
    uint64_t ws_codes;        // tile code records (fast) / all-level codes (per-pixel path)
    uint64_t ws_pyr;          // tile sums + upper levels (fast path)
    uint64_t ws_tmap;         // per tile: destination tile and quarter turns (fast path)
    uint64_t ws_stats;        // statistics records
    uint64_t ws_bytes;        // per-pixel path: byte-per-pixel scratch
    uint64_t ws_fix;          // EMR recovery of images cut into quad segments: per segment and row,
                              // leading pixels without a carry, then the last labelled value (u16 each)
    uint64_t ws_btab;         // DEMR encryption: b of every tile in original order
};

// Counter slots of an image's statistics: one per 64 tiles, at most 64.
__host__ __device__ inline uint32_t stat_slots(const Job &J) {
    if (!J.fast) return 1u;
    const uint32_t t = (uint32_t)(J.tiles_x * J.tiles_y) / 64u;
    return t < 1u ? 1u : (t > 64u ? 64u : t);
}
__host__ __device__ inline uint64_t stat_z_offset(const Job &J) {
    return J.ws_stats + (uint64_t)stat_slots(J) * kStatWords * 4;
}
// DEMR: the image's redundant pixels and capacity summed over its tiles (two
// u64 after the 64-bit Z values).
__host__ __device__ inline uint64_t stat_dyn_acc(const Job &J) { return stat_z_offset(J) + 64; }

// Per-tile b of one image (k_dynb.hip): 64x64 tiles numbered from tile_first.
struct TileBJob {
    const uint8_t *img;
    int32_t M, N;
    uint32_t tile_first;
    uint32_t pad;
};
void launch_tile_b(const TileBJob *jobs, int njobs, uint32_t tiles, uint8_t *tile_b, int64_t *cap, hipStream_t st);

// ---- launchers (defined in the .hip files) ---------------------------------
struct Launch {
    const Job *jobs;          // device job table
    const uint32_t *ujob[UNIT_KINDS] = {};   // unit -> job tables
    int32_t njobs;
    uint8_t *ws;              // device workspace base
    hipStream_t stream;
    int max_grid;             // cap on workgroups of a grid-stride launch
    uint64_t g_status = 0, g_part = 0;   // hiding workspace: step counts / ranks, partial-word records
    int keystream = kKsPhilox;           // keystream family of every job of the launch
    bool dyn = false;                    // the launch's images use one b per tile (RDHEI_DEMR)
};

void launch_tile_prep(const Launch &L, uint32_t units, bool stats);
// LMR batch helpers (k_lmr.hip)
void launch_gather_z(const Launch &L, int64_t *out);
void launch_gather_meta(const Launch &L, rdhei_meta *out);
void launch_scatter_meta(const Launch &L, const rdhei_meta *in);
void launch_msb_plane(const Launch &L, const uint64_t *off, uint8_t *out, uint64_t max_bytes);

// Images with at least kBigTiles tiles are finalised across many workgroups,
// in blocks of kFinBlock x kFinBlock tiles.
constexpr uint32_t kBigTiles = 4096;
constexpr int kFinBlock = 16;
// big: indices of such jobs; hj: the host copy of the job table
void launch_finalize(const Launch &L, bool stats, const std::vector<int> &big, const std::vector<Job> &hj);
void launch_encrypt_tiles(const Launch &L, uint32_t units, int mode);
// EMR / DEMR encryption and recovery of whole images, one workgroup per image
// (of kEncImageWaves waves for encryption): statistics or keystream codes,
// finalisation and the permuting pass in one kernel.  Every image of the
// launch must be tiled, with at most kImageWgMaxTiles tiles; for recovery
// every band pair must be one quad segment.
constexpr uint32_t kImageWgMaxTiles = 1024;
constexpr int kEncImageWaves = 8;
void launch_encrypt_images(const Launch &L);
void launch_recover_images(const Launch &L);
// fix_rows, fix_segs: most rows and most quad segments per band pair of the EMR
// images cut into segments (fix_rows 0: none)
void launch_recover_bands(const Launch &L, uint32_t units, int method, uint32_t fix_rows, uint32_t fix_segs);
uint64_t seg_pixels();          // pixels per hiding step (work unit)
uint64_t whole_max_pixels();    // largest image walked whole by one wave
uint32_t whole_image_min();
void launch_hide_images(const Launch &L, uint32_t units, bool embed);
void hide_ws_layout(uint32_t units, uint64_t base, uint64_t &ranks, uint64_t &part, uint64_t &end);
// one_pass: steps hidden in one pass with a decoupled look-back; otherwise
// counted, scanned and hidden in three passes
void launch_embed(const Launch &L, uint32_t units, bool one_pass);
void launch_extract(const Launch &L, uint32_t units, bool one_pass);
// per-pixel path, one image (job index j of the table; host copy h)
void launch_generic_levels(const Launch &L, int j, const Job &h);
void launch_generic_stats(const Launch &L, int j, const Job &h);
void launch_generic_encrypt(const Launch &L, int j, const Job &h, int mode);
void launch_generic_recover(const Launch &L, int j, const Job &h);
uint64_t generic_code_bytes(int M, int N, int n);

// Encrypt-kernel modes.
enum EncMode { ENC_EMR = 0, ENC_LMR = 1, ENC_LMR_MAPS = 2, ENC_DEMR = 3 };

// ---- image metrics (rdhei_metrics) ----
// One image pair of a metrics launch.  Work units: kMetricChunk-pixel runs of
// the image for the histogram-and-difference pass, tiles of kSsimRows x
// kSsimCols window anchors for SSIM; *_first are each job's first unit.
constexpr uint32_t kMetricChunk = 1u << 18;
constexpr int kSsimWin = 7, kSsimRows = 64, kSsimCols = 256;
struct MetricJob {
    const uint8_t *a;
    const uint8_t *b;          // nullptr: single-image metrics only
    int32_t M, N;
    int32_t vec;               // 1: both images 16-byte aligned (vector loads)
    int32_t pad;
    uint32_t sum_first, ssim_first;
};
// Per-job accumulators, cleared by the launch: level counts of a and b, the
// number of differing pixels, the sums of |a - b| and of a^2 + b^2 - 2ab (=
// sum of squared differences), and the sum of the windows' SSIM.
struct MetricAcc {
    uint32_t ha[256], hb[256];
    unsigned long long ndiff, sabs, ssq;
    double ssim;
};
void launch_metrics(const MetricJob *jobs, int njobs, MetricAcc *acc, uint32_t sum_units, uint32_t ssim_tiles,
                    int with_ssim, double *out, hipStream_t st);

}  // namespace rdhei

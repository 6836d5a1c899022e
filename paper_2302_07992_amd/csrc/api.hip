// Host side of librdhei: argument checks, job tables, workspace layout, the
// launch sequence of every stage, plans (hipGraph capture/replay), and the
// LMR host stages.
#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <functional>
#include <map>
#include <mutex>
#include <thread>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "internal.hpp"

namespace rdhei {
int lmr_compress_impl(const uint8_t *eta_bits, const uint8_t *l_bits, int32_t M, int32_t N, uint8_t *stream,
                      int64_t capacity_bytes, int64_t *stream_bits);
int lmr_decompress_impl(const uint8_t *stream, int64_t stream_bytes, int32_t M, int32_t N, uint8_t *eta_bits,
                        uint8_t *l_bits);
}  // namespace rdhei

using namespace rdhei;

namespace {

thread_local std::string g_err;

void set_err(const char *what, hipError_t e) {
    char buf[512];
    snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
    g_err = buf;
}

#define HIPCHK(call)                                      \
    do {                                                  \
        hipError_t e_ = (call);                           \
        if (e_ != hipSuccess) {                           \
            set_err(#call, e_);                           \
            return RDHEI_EDEVICE;                         \
        }                                                 \
    } while (0)

// Growable device buffer.
struct DevBuf {
    uint8_t *p = nullptr;
    size_t n = 0;
    int need(size_t bytes) {
        if (bytes <= n) return RDHEI_OK;
        if (p) {
            (void)hipDeviceSynchronize();
            (void)hipFree(p);
            p = nullptr;
            n = 0;
        }
        size_t want = std::max<size_t>(bytes, 4096);
        hipError_t e = hipMalloc(&p, want);
        if (e != hipSuccess) {
            set_err("hipMalloc", e);
            p = nullptr;
            return RDHEI_ENOMEM;
        }
        n = want;
        return RDHEI_OK;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
};

// Growable pinned host buffer (staging for bulk copies).
struct HostBuf {
    uint8_t *p = nullptr;
    size_t n = 0;
    int need(size_t bytes) {
        if (bytes <= n) return RDHEI_OK;
        if (p) (void)hipHostFree(p);
        p = nullptr;
        n = 0;
        hipError_t e = hipHostMalloc((void **)&p, std::max<size_t>(bytes, 1 << 16), hipHostMallocDefault);
        if (e != hipSuccess) {
            set_err("hipHostMalloc", e);
            p = nullptr;
            return RDHEI_ENOMEM;
        }
        n = std::max<size_t>(bytes, 1 << 16);
        return RDHEI_OK;
    }
    void release() {
        if (p) (void)hipHostFree(p);
        p = nullptr;
        n = 0;
    }
};

inline uint64_t align_up(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }

int floor_log2_min(int32_t M, int32_t N) {
    int64_t m = std::min(M, N);
    int n = 0;
    while (((int64_t)2 << n) <= m) ++n;
    return n;
}

// Bytes of the fast path's tile-sum pyramid (levels kTileLog..n).
uint64_t pyr_bytes(int32_t M, int32_t N, int n) {
    uint64_t b = 0;
    for (int k = kTileLog; k <= n; ++k) b += (uint64_t)(M >> k) * (uint64_t)(N >> k);
    return b;
}

struct Layout {
    std::vector<Job> jobs;
    std::vector<uint32_t> ujob[UNIT_KINDS];   // job index of every work unit (batches)
    std::vector<int> per_pixel;        // jobs on the per-pixel path
    uint64_t ws_bytes = 0;
    uint32_t units[UNIT_KINDS] = {};
    uint64_t g_status = 0, g_part = 0;   // hiding workspace (embed/extract)
    bool one_pass = false;               // steps hidden in one pass (look-back), else counted first
    bool images = false;                 // encryption / recovery one workgroup per image, else by stages
    int op = 0;
    int method = RDHEI_EMR;
    int keystream = kKsPhilox;
};

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

// Build the device job table and workspace layout of one op over a batch.
struct LayoutOpts {
    bool per_pixel = false;   // every image on the per-pixel path
    int hide_mode = 0;        // RDHEI_OPT_HIDE_MODE
    int lmr_min_level = 4;    // RDHEI_OPT_LMR_MIN_LEVEL
    int keystream = kKsPhilox;   // RDHEI_OPT_KEYSTREAM
    int qseg = kQuadSeg;         // quads per encryption / EMR recovery work unit
    int wg_image = 0;            // RDHEI_OPT_WG_PER_IMAGE
};

// Whether image q of a hiding op may be walked whole by one workgroup.
// Segments of at most J.qseg 2x2 tile quads per band pair (tiled images).
uint32_t quad_segments(const Job &J) {
    const uint32_t nq = (uint32_t)((J.tiles_x + 1) / 2);
    return (nq + (uint32_t)J.qseg - 1) / (uint32_t)J.qseg;
}

bool whole_eligible(int op, const rdhei_job &q) {
    if (op != RDHEI_OP_EMBED && op != RDHEI_OP_EXTRACT) return false;
    const uint64_t MN = (uint64_t)q.height * (uint64_t)q.width;
    const void *pin = op == RDHEI_OP_EMBED ? (const void *)q.out : (const void *)q.in;
    return MN <= whole_max_pixels() && MN % 16 == 0 &&
           aligned16(pin) && aligned16(q.out);
}

// Whether image q of a rotation role (encrypt / recover) takes the tiled path:
// sides multiples of 64, 16-byte aligned buffers, at most kTmapMaxTiles tiles
// along each side (the tile map's coordinate width).
bool tiled_ok(int op, const rdhei_job &q, bool force_per_pixel) {
    const bool rot = op == RDHEI_OP_ENCRYPT || op == RDHEI_OP_RECOVER;
    return rot && !force_per_pixel && q.height % kTile == 0 && q.width % kTile == 0 && aligned16(q.in) &&
           aligned16(q.out) && q.height / kTile <= kTmapMaxTiles && q.width / kTile <= kTmapMaxTiles;
}

// Whether a batch of a rotation role may go one workgroup per image: EMR or
// DEMR, every image tiled with at most kImageWgMaxTiles tiles.
bool wg_image_ok(int op, const rdhei_job *in, int n, bool force_per_pixel) {
    if (op != RDHEI_OP_ENCRYPT && op != RDHEI_OP_RECOVER) return false;
    for (int i = 0; i < n; ++i) {
        const rdhei_job &q = in[i];
        if (q.method != RDHEI_EMR && q.method != RDHEI_DEMR) return false;
        if (!tiled_ok(op, q, force_per_pixel)) return false;
        if ((uint64_t)(q.height / kTile) * (uint64_t)(q.width / kTile) > kImageWgMaxTiles) return false;
    }
    return n > 0;
}

// Images from which RDHEI_OPT_WG_PER_IMAGE 0 goes one workgroup per image:
// four per compute unit (fewer leave too little to interleave on each CU and
// the last round of images too large a part of the launch: with two per CU
// recovery is slower than by stages).
size_t wg_image_min() {
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        (void)hipGetDevice(&dev);
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 256;
    }
    return 4 * (size_t)cus;
}

int make_layout(int op, const rdhei_job *in, int n, const LayoutOpts &opt, Layout &L) {
    L = Layout();
    L.op = op;
    L.keystream = opt.keystream;
    if (n < 1) return RDHEI_EINVAL;
    L.method = in[0].method;
    L.one_pass = opt.hide_mode == 3;
    const bool force_per_pixel = opt.per_pixel;
    L.images = opt.wg_image != 1 && wg_image_ok(op, in, n, force_per_pixel) &&
               (opt.wg_image == 2 || (size_t)n >= wg_image_min());
    bool whole_ok = opt.hide_mode == 1;
    if (opt.hide_mode == 0) {
        uint32_t eligible = 0;
        for (int i = 0; i < n; ++i) eligible += whole_eligible(op, in[i]) ? 1u : 0u;
        whole_ok = eligible >= whole_image_min();
    }
    uint64_t ws = 0;
    for (int i = 0; i < n; ++i) {
        const rdhei_job &q = in[i];
        if (q.height < 1 || q.width < 1) return RDHEI_EINVAL;
        if ((int64_t)q.height * q.width > ((int64_t)1 << 31)) return RDHEI_EINVAL;
        if (q.method != RDHEI_EMR && q.method != RDHEI_LMR && q.method != RDHEI_DEMR) return RDHEI_EINVAL;
        if (q.method != L.method) return RDHEI_EINVAL;
        if (!q.meta) return RDHEI_EINVAL;
        switch (op) {
            case RDHEI_OP_ENCRYPT: if (!q.in || !q.out || q.in == q.out) return RDHEI_EINVAL; break;
            case RDHEI_OP_EMBED: if (!q.out || !q.msg || !aligned16(q.msg)) return RDHEI_EINVAL; break;
            case RDHEI_OP_EXTRACT: if (!q.in || !q.msg || !aligned16(q.msg)) return RDHEI_EINVAL; break;
            case RDHEI_OP_RECOVER: if (!q.in || !q.out || q.in == q.out) return RDHEI_EINVAL; break;
            default: return RDHEI_EINVAL;
        }
        Job J;
        memset(&J, 0, sizeof J);
        J.in = op == RDHEI_OP_EMBED ? q.out : q.in;
        J.out = q.out;
        J.msg = q.msg;
        J.meta = q.meta;
        J.key = q.key;
        J.nonce = op == RDHEI_OP_ENCRYPT ? q.nonce : 0;
        J.nonce_meta = op == RDHEI_OP_ENCRYPT ? 0 : 1;
        J.nbits = q.nbits;
        J.M = q.height;
        J.N = q.width;
        J.method = q.method;
        J.min_level = q.method == RDHEI_LMR ? opt.lmr_min_level : 1;
        J.max_level = floor_log2_min(q.height, q.width);
        const uint64_t MN = (uint64_t)q.height * (uint64_t)q.width;
        const bool rot = op == RDHEI_OP_ENCRYPT || op == RDHEI_OP_RECOVER;
        // the tile map holds 14-bit tile coordinates: images with more tiles
        // along a side take the per-pixel path
        J.fast = tiled_ok(op, q, force_per_pixel) ? 1 : 0;
        if (q.method == RDHEI_DEMR) {
            // one b per tile: the tiled path for every op, and the tile table;
            // payload bit offsets stay below 2^32 (images of at most 2^29 pixels)
            if ((int64_t)q.height * q.width > ((int64_t)1 << 29)) return RDHEI_EINVAL;
            if (!q.btab || !(rot ? J.fast : (q.height % kTile == 0 && q.width % kTile == 0 &&
                                             q.height / kTile <= kTmapMaxTiles && q.width / kTile <= kTmapMaxTiles)))
                return RDHEI_EINVAL;
            J.btab = q.btab;
            J.tiles_x = q.width / kTile;
            J.tiles_y = q.height / kTile;
        }
        if (J.fast) {
            J.tiles_x = q.width / kTile;
            J.tiles_y = q.height / kTile;
        }
        J.nseg = (int32_t)((MN + seg_pixels() - 1) / seg_pixels());
        J.qseg = opt.qseg;
        if (L.images) J.qseg = std::max(opt.qseg, (J.tiles_x + 1) / 2);   // a band pair is one segment
        if (rot) {
            const uint64_t tiles = (uint64_t)J.tiles_x * J.tiles_y;
            J.ws_codes = ws;
            ws = align_up(ws + (J.fast ? tiles * kCodeRecord : generic_code_bytes(J.M, J.N, J.max_level)), 256);
            J.ws_pyr = ws;
            ws = align_up(ws + (J.fast ? pyr_bytes(J.M, J.N, J.max_level) : 0), 256);
            J.ws_tmap = ws;
            ws = align_up(ws + (J.fast ? tiles * 4 : 0), 256);
            J.ws_stats = ws;
            // counter slots, then Z as 64-bit values, then the DEMR accumulators
            ws = align_up(stat_dyn_acc(J) + 16, 256);
            if (q.method == RDHEI_DEMR && op == RDHEI_OP_ENCRYPT) {
                J.ws_btab = ws;                          // b of every tile, original order
                ws = align_up(ws + tiles, 256);
            }
            if (op == RDHEI_OP_RECOVER && q.method != RDHEI_LMR && J.fast && quad_segments(J) > 1) {
                J.ws_fix = ws;   // two u16 per image row and quad segment
                ws = align_up(ws + (uint64_t)J.M * quad_segments(J) * 4u, 256);
            }
            if (q.method == RDHEI_LMR && !J.fast) {
                J.ws_bytes = ws;
                ws = align_up(ws + MN, 256);
            }
        }
        // hiding: whole small images go to one wave each (UNIT_IMG), others
        // are cut into 4096-pixel steps (UNIT_SEG)
        const bool hide = op == RDHEI_OP_EMBED || op == RDHEI_OP_EXTRACT;
        const bool whole = whole_ok && whole_eligible(op, q);
        const bool quads = J.fast && (op == RDHEI_OP_ENCRYPT || (op == RDHEI_OP_RECOVER && q.method != RDHEI_LMR));
        const bool bands = J.fast && op == RDHEI_OP_RECOVER && q.method == RDHEI_LMR;
        const uint32_t cnt[UNIT_KINDS] = {J.fast ? (uint32_t)(J.tiles_x * J.tiles_y) : 0u,
                                          bands ? (uint32_t)J.tiles_y : 0u,
                                          hide && !whole ? (uint32_t)J.nseg : 0u, whole ? 1u : 0u,
                                          quads ? (uint32_t)((J.tiles_y + 1) / 2) * quad_segments(J) : 0u};
        for (int k = 0; k < UNIT_KINDS; ++k) {
            J.ubase[k] = L.units[k];
            J.ucount[k] = cnt[k];
            L.units[k] += cnt[k];
        }
        if (rot && !J.fast) L.per_pixel.push_back(i);
        if (n > 1)
            for (int k = 0; k < UNIT_KINDS; ++k) L.ujob[k].insert(L.ujob[k].end(), cnt[k], (uint32_t)i);
        L.jobs.push_back(J);
    }
    if (op == RDHEI_OP_EMBED || op == RDHEI_OP_EXTRACT) {
        uint64_t end;
        hide_ws_layout(L.units[UNIT_SEG], ws, L.g_status, L.g_part, end);
        ws = end;
    }
    L.ws_bytes = std::max<uint64_t>(ws, 256);
    return RDHEI_OK;
}

// The launch sequence of an op, as named stages (the paper's phase order).
struct Stage {
    const char *name;
    std::function<void(const Launch &)> fn;
};

std::vector<Stage> stages_of(const Layout &Ly, const uint32_t *units_in, std::vector<int> pp) {
    std::vector<Stage> S;
    const int op = Ly.op;
    const std::vector<Job> hj = Ly.jobs;
    uint32_t units[UNIT_KINDS];
    for (int k = 0; k < UNIT_KINDS; ++k) units[k] = units_in[k];
    const uint32_t ut = units[UNIT_TILE], ub = units[UNIT_BAND], us = units[UNIT_SEG], uq = units[UNIT_QROW];
    const int method = Ly.method;
    std::vector<int> big;   // images finalised across many workgroups
    for (size_t i = 0; i < hj.size(); ++i)
        if (hj[i].fast && (uint32_t)(hj[i].tiles_x * hj[i].tiles_y) >= kBigTiles) big.push_back((int)i);
    if (op == RDHEI_OP_ENCRYPT && Ly.images) {
        S.push_back({"encrypt_images", [=](const Launch &L) { launch_encrypt_images(L); }});
    } else if (op == RDHEI_OP_RECOVER && Ly.images) {
        S.push_back({"recover_images", [=](const Launch &L) { launch_recover_images(L); }});
    } else if (op == RDHEI_OP_ENCRYPT) {
        if (ut) S.push_back({"tile_prep_stats", [=](const Launch &L) { launch_tile_prep(L, ut, true); }});
        if (!pp.empty())
            S.push_back({"per_pixel_levels_stats", [=](const Launch &L) {
                             for (int j : pp) { launch_generic_levels(L, j, hj[j]); launch_generic_stats(L, j, hj[j]); }
                         }});
        S.push_back({"finalize_stats", [=](const Launch &L) { launch_finalize(L, true, big, hj); }});
        const int emode = method == RDHEI_DEMR ? ENC_DEMR : ENC_EMR;
        if (uq) S.push_back({"encrypt_tiles", [=](const Launch &L) { launch_encrypt_tiles(L, uq, emode); }});
        if (!pp.empty())
            S.push_back({"per_pixel_encrypt", [=](const Launch &L) {
                             for (int j : pp) launch_generic_encrypt(L, j, hj[j], ENC_EMR);
                         }});
    } else if (op == RDHEI_OP_RECOVER) {
        if (ut) S.push_back({"tile_prep", [=](const Launch &L) { launch_tile_prep(L, ut, false); }});
        if (!pp.empty())
            S.push_back({"per_pixel_levels", [=](const Launch &L) {
                             for (int j : pp) launch_generic_levels(L, j, hj[j]);
                         }});
        if (ut) S.push_back({"finalize_pyramid", [=](const Launch &L) { launch_finalize(L, false, big, hj); }});
        const uint32_t urec = method != RDHEI_LMR ? uq : ub;
        uint32_t fix_rows = 0, fix_segs = 0;   // images cut into quad segments get their rows completed afterwards
        for (const Job &J : hj)
            if (J.fast && method != RDHEI_LMR && quad_segments(J) > 1) {
                fix_rows = std::max(fix_rows, (uint32_t)J.M);
                fix_segs = std::max(fix_segs, quad_segments(J));
            }
        if (urec)
            S.push_back({"recover_bands", [=](const Launch &L) {
                             launch_recover_bands(L, urec, method, fix_rows, fix_segs);
                         }});
        if (!pp.empty())
            S.push_back({"per_pixel_recover", [=](const Launch &L) {
                             for (int j : pp) launch_generic_recover(L, j, hj[j]);
                         }});
    } else if (op == RDHEI_OP_EMBED || op == RDHEI_OP_EXTRACT) {
        const uint32_t ui = units[UNIT_IMG];
        const bool emb = op == RDHEI_OP_EMBED;
        if (ui) S.push_back({emb ? "embed_images" : "extract_images", [=](const Launch &L) { launch_hide_images(L, ui, emb); }});
        const bool one = Ly.one_pass;
        if (us && op == RDHEI_OP_EMBED) S.push_back({"embed", [=](const Launch &L) { launch_embed(L, us, one); }});
        else if (us) S.push_back({"extract", [=](const Launch &L) { launch_extract(L, us, one); }});
    }
    return S;
}

void issue(const Layout &Ly, const Launch &L, const uint32_t *units, const int *pp, int npp, int) {
    for (const Stage &s : stages_of(Ly, units, std::vector<int>(pp, pp + npp))) s.fn(L);
}

}  // namespace

// ------------------------------------------------------------------------------
// One autotuner choice: the layout variant and each stage's workgroup count.
struct TuneRecord {
    int hide_mode = 0;
    int qseg = kQuadSeg;
    int wg_image = 0;
    std::vector<int> grids;
};

// Ring of pinned host buffers for asynchronous job-table uploads: a slot is
// reused only after the copy issued from it has completed.
struct PinnedRing {
    static constexpr int kSlots = 16;
    uint8_t *buf[kSlots] = {};
    size_t cap[kSlots] = {};
    hipEvent_t done[kSlots] = {};
    bool used[kSlots] = {};
    int next = 0;
    int acquire(size_t bytes, uint8_t **out, int *slot) {
        const int k = next;
        next = (next + 1) % kSlots;
        if (used[k]) {
            HIPCHK(hipEventSynchronize(done[k]));
            used[k] = false;
        }
        if (!done[k]) HIPCHK(hipEventCreateWithFlags(&done[k], hipEventDisableTiming));
        if (cap[k] < bytes) {
            if (buf[k]) (void)hipHostFree(buf[k]);
            buf[k] = nullptr;
            cap[k] = 0;
            const size_t want = std::max<size_t>(bytes, 1 << 16);
            HIPCHK(hipHostMalloc((void **)&buf[k], want, hipHostMallocDefault));
            cap[k] = want;
        }
        *out = buf[k];
        *slot = k;
        return RDHEI_OK;
    }
    void release_all() {
        for (int k = 0; k < kSlots; ++k) {
            if (used[k]) (void)hipEventSynchronize(done[k]);
            if (buf[k]) (void)hipHostFree(buf[k]);
            if (done[k]) (void)hipEventDestroy(done[k]);
            buf[k] = nullptr;
            done[k] = nullptr;
            used[k] = false;
        }
    }
};

struct rdhei_ctx {
    int device = 0;
    uint8_t *static_ws = nullptr;      // this device's address of the static scratch array
    int per_pixel = 0;
    int hide_mode = 0;
    int lmr_min_level = 4;
    int keystream = kKsPhilox;
    int qseg = kQuadSeg;
    int wg_image = 0;
    std::map<std::string, TuneRecord> tuned;   // autotuner choices by device/op/size class
    std::string tune_file;              // where the choices persist (empty: memory only)
    int max_grid = 0;
    DevBuf ws, jobs, scratch, batch_tables, lmr_dev, metrics, tileb;
    HostBuf lmr_host;
    PinnedRing ring;
    std::vector<uint8_t> h_a, h_b, h_c;
};

struct rdhei_plan {
    rdhei_ctx *ctx = nullptr;
    int op = 0;
    std::vector<rdhei_job> src;    // the caller's jobs (host copy), for re-layout by the autotuner
    LayoutOpts opts;               // layout options the plan is laid out with
    Layout layout;
    DevBuf ws, jobs, single;       // single: per-image one-job tables
    int flags = 0;
    int max_grid = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<Stage> stages;     // batched sequence (for per-stage runs)
    std::vector<int> stage_grid;   // per-stage workgroup count (0: the launcher's default)
    Launch base;                   // device tables of the batched sequence
    // PER_IMAGE plans: each image laid out and launched on its own, exactly
    // as the single-image entry points would
    struct One {
        Layout layout;
        size_t table_off = 0;
        std::vector<Stage> stages;
    };
    std::vector<One> per_image;
};

namespace {

LayoutOpts opts_of(const rdhei_ctx *ctx) {
    LayoutOpts o;
    o.per_pixel = ctx->per_pixel != 0;
    o.hide_mode = ctx->hide_mode;
    o.lmr_min_level = ctx->lmr_min_level;
    o.keystream = ctx->keystream;
    o.qseg = ctx->qseg;
    o.wg_image = ctx->wg_image;
    return o;
}

int set_device(int dev) {
    HIPCHK(hipSetDevice(dev));
    return RDHEI_OK;
}

// Bytes of a layout's device table: jobs, then the unit -> job arrays.
size_t table_bytes(const Layout &Ly, size_t off[UNIT_KINDS]) {
    size_t b = align_up(Ly.jobs.size() * sizeof(Job), 256);
    for (int k = 0; k < UNIT_KINDS; ++k) {
        off[k] = b;
        b = align_up(b + Ly.ujob[k].size() * sizeof(uint32_t), 256);
    }
    return b;
}

// Copy the job table and unit tables to `dst` (device) and fill L's pointers.
int upload_tables(const Layout &Ly, uint8_t *dst, hipStream_t st, bool sync, Launch &L) {
    size_t off[UNIT_KINDS];
    table_bytes(Ly, off);
    if (sync) {
        HIPCHK(hipMemcpy(dst, Ly.jobs.data(), Ly.jobs.size() * sizeof(Job), hipMemcpyHostToDevice));
    } else {
        HIPCHK(hipMemcpyAsync(dst, Ly.jobs.data(), Ly.jobs.size() * sizeof(Job), hipMemcpyHostToDevice, st));
    }
    L.jobs = reinterpret_cast<const Job *>(dst);
    for (int k = 0; k < UNIT_KINDS; ++k) {
        L.ujob[k] = nullptr;
        if (Ly.ujob[k].empty()) continue;
        if (sync) {
            HIPCHK(hipMemcpy(dst + off[k], Ly.ujob[k].data(), Ly.ujob[k].size() * 4, hipMemcpyHostToDevice));
        } else {
            HIPCHK(hipMemcpyAsync(dst + off[k], Ly.ujob[k].data(), Ly.ujob[k].size() * 4, hipMemcpyHostToDevice, st));
        }
        L.ujob[k] = reinterpret_cast<const uint32_t *>(dst + off[k]);
    }
    return RDHEI_OK;
}

// Upload a layout's job table into `jobs` and size `ws`; returns the Launch.
int stage(rdhei_ctx *ctx, const Layout &Ly, DevBuf &jobs, DevBuf &ws, hipStream_t st, Launch &L) {
    size_t off[UNIT_KINDS];
    int rc = jobs.need(table_bytes(Ly, off));
    if (rc) return rc;
    rc = ws.need(Ly.ws_bytes);
    if (rc) return rc;
    rc = upload_tables(Ly, jobs.p, st, false, L);
    if (rc) return rc;
    L.njobs = (int32_t)Ly.jobs.size();
    L.ws = ws.p;
    L.stream = st;
    L.max_grid = ctx->max_grid;
    L.g_status = Ly.g_status;
    L.g_part = Ly.g_part;
    L.keystream = Ly.keystream;
    L.dyn = Ly.method == RDHEI_DEMR;
    return RDHEI_OK;
}

int run_single(rdhei_ctx *ctx, int op, const rdhei_job &job, hipStream_t st) {
    int rc = set_device(ctx->device);
    if (rc) return rc;
    Layout Ly;
    rc = make_layout(op, &job, 1, opts_of(ctx), Ly);
    if (rc) return rc;
    Launch L;
    rc = stage(ctx, Ly, ctx->jobs, ctx->ws, st, L);
    if (rc) return rc;
    issue(Ly, L, Ly.units, Ly.per_pixel.data(), (int)Ly.per_pixel.size(), 0);
    HIPCHK(hipGetLastError());
    return RDHEI_OK;
}

// ---- LMR (Sec. III-B): host stages around the GPU kernels ----------------------

// Bit 7 of the first `bits` pixels (raster order), packed MSB-first.
void msb_plane(const uint8_t *img, int64_t bits, std::vector<uint8_t> &out) {
    out.assign((size_t)((bits + 7) / 8) + 16, 0);
    for (int64_t p = 0; p < bits; ++p) out[(size_t)(p >> 3)] |= (uint8_t)(((img[p] >> 7) & 1u) << (7 - (p & 7)));
}

int lmr_encrypt(rdhei_ctx *ctx, const uint8_t *d_img, uint8_t *d_enc, int32_t M, int32_t N, uint64_t k1,
                uint64_t nonce, rdhei_meta *d_meta, hipStream_t st) {
    int rc = set_device(ctx->device);
    if (rc) return rc;
    rdhei_job q{};
    q.in = d_img; q.out = d_enc; q.meta = d_meta; q.key = k1; q.nonce = nonce; q.nbits = 0;
    q.height = M; q.width = N; q.method = RDHEI_LMR;
    Layout Ly;
    rc = make_layout(RDHEI_OP_ENCRYPT, &q, 1, opts_of(ctx), Ly);
    if (rc) return rc;
    const uint64_t MN = (uint64_t)M * N;
    const uint64_t plane = align_up((MN + 7) / 8 + 16, 256);
    // scratch: l plane, eta plane, stream
    rc = ctx->scratch.need(3 * plane);
    if (rc) return rc;
    uint8_t *d_l = ctx->scratch.p, *d_eta = d_l + plane, *d_stream = d_eta + plane;
    Launch L;
    rc = stage(ctx, Ly, ctx->jobs, ctx->ws, st, L);
    if (rc) return rc;
    const Job J0 = Ly.jobs[0];   // a copy: the candidate loop rewrites Ly.jobs[0]
    launch_tile_prep(L, Ly.units[UNIT_TILE], true);
    if (!J0.fast) {
        launch_generic_levels(L, 0, J0);
        launch_generic_stats(L, 0, J0);
    }
    {
        std::vector<int> big;
        if (J0.fast && (uint32_t)(J0.tiles_x * J0.tiles_y) >= kBigTiles) big.push_back(0);
        launch_finalize(L, true, big, Ly.jobs);
    }
    int64_t Z[7];
    const uint64_t zoff = stat_z_offset(J0);
    HIPCHK(hipMemcpyAsync(Z, ctx->ws.p + zoff, sizeof Z, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    // candidates in order of LMR capacity (b-1)*Z_b, smaller b first on ties
    std::vector<int> cand;
    for (int b = 2; b <= 8; ++b) cand.push_back(b);
    std::stable_sort(cand.begin(), cand.end(), [&](int a, int b) {
        return (int64_t)(a - 1) * Z[a - 2] > (int64_t)(b - 1) * Z[b - 2];
    });
    std::vector<uint8_t> &hl = ctx->h_a, &he = ctx->h_b, &hs = ctx->h_c;
    hl.assign(plane, 0);
    he.assign(plane, 0);
    hs.assign(plane, 0);
    int chosen = 0;
    int64_t sbits = 0;
    for (int b : cand) {
        Job J = J0;
        J.fixed_b = b;
        J.out = d_l;
        J.msg = d_eta;
        Ly.jobs[0] = J;
        HIPCHK(hipMemcpyAsync(ctx->jobs.p, &Ly.jobs[0], sizeof(Job), hipMemcpyHostToDevice, st));
        if (J.fast) launch_encrypt_tiles(L, Ly.units[UNIT_QROW], ENC_LMR_MAPS);
        else launch_generic_encrypt(L, 0, J, ENC_LMR_MAPS);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(hl.data(), d_l, (MN + 7) / 8, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(he.data(), d_eta, (MN + 7) / 8, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        int64_t bits = 0;
        const int r = lmr_compress_impl(he.data(), hl.data(), M, N, hs.data(), (int64_t)(MN / 8), &bits);
        if (r == RDHEI_OK) {
            chosen = b;
            sbits = bits;
            break;
        }
        if (r != RDHEI_ENOFIT) return r;
    }
    rdhei_meta m{};
    m.height = M; m.width = N; m.method = RDHEI_LMR; m.min_level = J0.min_level; m.max_level = J0.max_level;
    m.nonce = nonce;
    if (!chosen) {
        m.status = RDHEI_ENOFIT;
        HIPCHK(hipMemcpyAsync(d_meta, &m, sizeof m, hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
        return RDHEI_ENOFIT;
    }
    m.b = chosen;
    m.redundant = Z[chosen - 2];
    m.capacity_bits = (int64_t)(chosen - 1) * Z[chosen - 2];
    m.map_bits = sbits;
    m.status = RDHEI_OK;
    HIPCHK(hipMemcpyAsync(d_meta, &m, sizeof m, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(d_stream, hs.data(), (size_t)((sbits + 7) / 8), hipMemcpyHostToDevice, st));
    Job J = J0;
    J.fixed_b = chosen;
    J.stream = d_stream;
    J.stream_bits = sbits;
    Ly.jobs[0] = J;
    HIPCHK(hipMemcpyAsync(ctx->jobs.p, &Ly.jobs[0], sizeof(Job), hipMemcpyHostToDevice, st));
    if (J.fast) launch_encrypt_tiles(L, Ly.units[UNIT_QROW], ENC_LMR);
    else launch_generic_encrypt(L, 0, J, ENC_LMR);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    return RDHEI_OK;
}

// Decompress the maps of an LMR image into device bit planes (ctx scratch).
int lmr_maps_to_device(rdhei_ctx *ctx, const uint8_t *d_marked, int32_t M, int32_t N, rdhei_meta *d_meta,
                       hipStream_t st, rdhei_meta &m, uint8_t *&d_l, uint8_t *&d_eta) {
    HIPCHK(hipMemcpyAsync(&m, d_meta, sizeof m, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (m.status != RDHEI_OK) return m.status;
    if (m.method != RDHEI_LMR || m.height != M || m.width != N) return RDHEI_EINVAL;
    const uint64_t MN = (uint64_t)M * N;
    if (m.map_bits < 64 || (uint64_t)m.map_bits > MN) return RDHEI_ECORRUPT;
    const uint64_t plane = align_up((MN + 7) / 8 + 16, 256);
    int rc = ctx->scratch.need(3 * plane);
    if (rc) return rc;
    d_l = ctx->scratch.p;
    d_eta = d_l + plane;
    std::vector<uint8_t> head((size_t)m.map_bits);
    HIPCHK(hipMemcpyAsync(head.data(), d_marked, (size_t)m.map_bits, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    std::vector<uint8_t> stream;
    msb_plane(head.data(), m.map_bits, stream);
    std::vector<uint8_t> &hl = ctx->h_a, &he = ctx->h_b;
    hl.assign(plane, 0);
    he.assign(plane, 0);
    rc = lmr_decompress_impl(stream.data(), (m.map_bits + 7) / 8, M, N, he.data(), hl.data());
    if (rc) return rc;
    HIPCHK(hipMemcpyAsync(d_l, hl.data(), plane, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(d_eta, he.data(), plane, hipMemcpyHostToDevice, st));
    return RDHEI_OK;
}

int lmr_stage(rdhei_ctx *ctx, int op, const uint8_t *d_marked, uint8_t *d_out, int32_t M, int32_t N,
              rdhei_meta *d_meta, uint8_t *d_msg, int64_t nbits, uint64_t key, hipStream_t st) {
    int rc = set_device(ctx->device);
    if (rc) return rc;
    rdhei_meta m;
    uint8_t *d_l = nullptr, *d_eta = nullptr;
    rc = lmr_maps_to_device(ctx, d_marked, M, N, d_meta, st, m, d_l, d_eta);
    if (rc) return rc;
    rdhei_job q{};
    q.in = d_marked; q.out = d_out; q.msg = d_msg; q.meta = d_meta; q.key = key; q.nbits = nbits;
    q.height = M; q.width = N; q.method = RDHEI_LMR;
    Layout Ly;
    rc = make_layout(op, &q, 1, opts_of(ctx), Ly);
    if (rc) return rc;
    Ly.jobs[0].lbits = d_l;
    Ly.jobs[0].etabits = d_eta;
    Launch L;
    rc = stage(ctx, Ly, ctx->jobs, ctx->ws, st, L);
    if (rc) return rc;
    issue(Ly, L, Ly.units, Ly.per_pixel.data(), (int)Ly.per_pixel.size(), 1);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    return RDHEI_OK;
}

// ---- LMR batches (Sec. III-B) ------------------------------------------------------
// Device stages run batched; the map coder runs on host threads.

using Clock = std::chrono::steady_clock;
inline double secs(Clock::time_point a, Clock::time_point b) { return std::chrono::duration<double>(b - a).count(); }

template <typename F>
void parallel_for(int n, int threads, F f) {
    if (n <= 0) return;
    if (threads < 1) threads = (int)std::max(1u, std::thread::hardware_concurrency());
    threads = std::min(threads, n);
    std::atomic<int> next(0);
    auto work = [&]() {
        for (int i; (i = next.fetch_add(1)) < n;) f(i);
    };
    std::vector<std::thread> pool;
    for (int t = 1; t < threads; ++t) pool.emplace_back(work);
    work();
    for (std::thread &t : pool) t.join();
}

// The jobs idx of a layout as a layout of their own: each job keeps its
// workspace offsets; unit bases and unit tables are rebuilt.
Layout subset_layout(const Layout &full, const std::vector<int> &idx) {
    Layout S;
    S.op = full.op;
    S.method = full.method;
    S.keystream = full.keystream;
    S.ws_bytes = full.ws_bytes;
    S.g_status = full.g_status;
    S.g_part = full.g_part;
    const bool rot = full.op == RDHEI_OP_ENCRYPT || full.op == RDHEI_OP_RECOVER;
    for (size_t q = 0; q < idx.size(); ++q) {
        Job J = full.jobs[(size_t)idx[q]];
        for (int k = 0; k < UNIT_KINDS; ++k) {
            J.ubase[k] = S.units[k];
            S.units[k] += J.ucount[k];
        }
        if (rot && !J.fast) S.per_pixel.push_back((int)q);
        S.jobs.push_back(J);
    }
    if (idx.size() > 1)
        for (size_t q = 0; q < S.jobs.size(); ++q)
            for (int k = 0; k < UNIT_KINDS; ++k) S.ujob[k].insert(S.ujob[k].end(), S.jobs[q].ucount[k], (uint32_t)q);
    return S;
}

std::vector<int> big_jobs(const Layout &Ly) {
    std::vector<int> big;
    for (size_t i = 0; i < Ly.jobs.size(); ++i)
        if (Ly.jobs[i].fast && (uint32_t)(Ly.jobs[i].tiles_x * Ly.jobs[i].tiles_y) >= kBigTiles) big.push_back((int)i);
    return big;
}

struct LmrTimes {
    double device = 0, coder = 0;
};

int lmr_encrypt_batch(rdhei_ctx *ctx, const rdhei_job *jobs, int n, int threads, LmrTimes &T, hipStream_t st) {
    Layout Ly;
    int rc = make_layout(RDHEI_OP_ENCRYPT, jobs, n, opts_of(ctx), Ly);
    if (rc) return rc;
    if (Ly.method != RDHEI_LMR) return RDHEI_EINVAL;
    // per image: l plane, eta plane, coder output (MN/8 bytes at most)
    std::vector<uint64_t> plane((size_t)n), poff((size_t)n);
    uint64_t tot = 0;
    for (int i = 0; i < n; ++i) {
        const uint64_t MN = (uint64_t)Ly.jobs[(size_t)i].M * (uint64_t)Ly.jobs[(size_t)i].N;
        plane[(size_t)i] = align_up((MN + 7) / 8 + 16, 256);
        poff[(size_t)i] = tot;
        tot += 3 * plane[(size_t)i];
    }
    const uint64_t zoff = tot, moff = zoff + align_up((uint64_t)n * 56, 256);
    const uint64_t soff = moff + align_up((uint64_t)n * sizeof(rdhei_meta), 256);   // packed streams
    const uint64_t all = soff + tot / 3 + 256;
    if ((rc = ctx->lmr_dev.need(all)) || (rc = ctx->lmr_host.need(all))) return rc;
    uint8_t *D = ctx->lmr_dev.p, *H = ctx->lmr_host.p;
    auto t0 = Clock::now();
    Launch L;
    if ((rc = stage(ctx, Ly, ctx->jobs, ctx->ws, st, L))) return rc;
    launch_tile_prep(L, Ly.units[UNIT_TILE], true);
    for (int j : Ly.per_pixel) {
        launch_generic_levels(L, j, Ly.jobs[(size_t)j]);
        launch_generic_stats(L, j, Ly.jobs[(size_t)j]);
    }
    launch_finalize(L, true, big_jobs(Ly), Ly.jobs);
    launch_gather_z(L, reinterpret_cast<int64_t *>(D + zoff));
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(H + zoff, D + zoff, (size_t)n * 56, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    T.device += secs(t0, Clock::now());
    const int64_t *Z = reinterpret_cast<const int64_t *>(H + zoff);
    // candidates in order of LMR capacity (b-1)*Z_b, smaller b first on ties
    std::vector<std::vector<int>> cand((size_t)n);
    for (int i = 0; i < n; ++i) {
        std::vector<int> &c = cand[(size_t)i];
        for (int b = 2; b <= 8; ++b) c.push_back(b);
        const int64_t *z = Z + 7 * i;
        std::stable_sort(c.begin(), c.end(),
                         [&](int a, int b) { return (int64_t)(a - 1) * z[a - 2] > (int64_t)(b - 1) * z[b - 2]; });
    }
    std::vector<int> cur((size_t)n, 0), chosen((size_t)n, 0), res;
    std::vector<int64_t> sbits((size_t)n, 0);
    std::vector<int> pending;
    for (int i = 0; i < n; ++i) pending.push_back(i);
    while (!pending.empty()) {
        auto t1 = Clock::now();
        Layout S = subset_layout(Ly, pending);
        for (size_t q = 0; q < pending.size(); ++q) {
            const int i = pending[q];
            Job &J = S.jobs[q];
            J.fixed_b = cand[(size_t)i][(size_t)cur[(size_t)i]];
            J.out = D + poff[(size_t)i];
            J.msg = D + poff[(size_t)i] + plane[(size_t)i];
        }
        Launch LS;
        if ((rc = stage(ctx, S, ctx->jobs, ctx->ws, st, LS))) return rc;
        if (S.units[UNIT_QROW]) launch_encrypt_tiles(LS, S.units[UNIT_QROW], ENC_LMR_MAPS);
        for (int q : S.per_pixel) launch_generic_encrypt(LS, q, S.jobs[(size_t)q], ENC_LMR_MAPS);
        HIPCHK(hipGetLastError());
        if (pending.size() == (size_t)n) {
            HIPCHK(hipMemcpyAsync(H, D, (size_t)tot, hipMemcpyDeviceToHost, st));
        } else {
            for (int i : pending)
                HIPCHK(hipMemcpyAsync(H + poff[(size_t)i], D + poff[(size_t)i], (size_t)(2 * plane[(size_t)i]),
                                      hipMemcpyDeviceToHost, st));
        }
        HIPCHK(hipStreamSynchronize(st));
        auto t2 = Clock::now();
        T.device += secs(t1, t2);
        res.assign(pending.size(), 0);
        parallel_for((int)pending.size(), threads, [&](int q) {
            const int i = pending[(size_t)q];
            const Job &J = Ly.jobs[(size_t)i];
            const uint64_t MN = (uint64_t)J.M * (uint64_t)J.N;
            uint8_t *hl = H + poff[(size_t)i], *he = hl + plane[(size_t)i], *hs = he + plane[(size_t)i];
            res[(size_t)q] = lmr_compress_impl(he, hl, J.M, J.N, hs, (int64_t)(MN / 8), &sbits[(size_t)i]);
        });
        T.coder += secs(t2, Clock::now());
        std::vector<int> next;
        for (size_t q = 0; q < pending.size(); ++q) {
            const int i = pending[q];
            if (res[q] == RDHEI_OK) chosen[(size_t)i] = cand[(size_t)i][(size_t)cur[(size_t)i]];
            else if (res[q] == RDHEI_ENOFIT) {
                if (++cur[(size_t)i] < 7) next.push_back(i);
            } else return res[q];
        }
        pending.swap(next);
    }
    auto t3 = Clock::now();
    // meta records, packed streams, then the encryption of every image that fits
    rdhei_meta *hm = reinterpret_cast<rdhei_meta *>(H + moff);
    std::vector<uint64_t> so((size_t)n, 0);
    std::vector<int> ok;
    uint64_t sp = 0;
    for (int i = 0; i < n; ++i) {
        const Job &J = Ly.jobs[(size_t)i];
        rdhei_meta m{};
        m.height = J.M; m.width = J.N; m.method = RDHEI_LMR; m.min_level = J.min_level; m.max_level = J.max_level;
        m.nonce = J.nonce;
        const int b = chosen[(size_t)i];
        if (b) {
            const int64_t *z = Z + 7 * i;
            m.b = b;
            m.redundant = z[b - 2];
            m.capacity_bits = (int64_t)(b - 1) * z[b - 2];
            m.map_bits = sbits[(size_t)i];
            m.status = RDHEI_OK;
            so[(size_t)i] = sp;
            memcpy(H + soff + sp, H + poff[(size_t)i] + 2 * plane[(size_t)i], (size_t)((sbits[(size_t)i] + 7) / 8));
            sp = align_up(sp + (uint64_t)((sbits[(size_t)i] + 7) / 8), 16);
            ok.push_back(i);
        } else {
            m.status = RDHEI_ENOFIT;
        }
        hm[i] = m;
    }
    HIPCHK(hipMemcpyAsync(D + moff, H + moff, (size_t)n * sizeof(rdhei_meta), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(D + soff, H + soff, (size_t)std::max<uint64_t>(sp, 16), hipMemcpyHostToDevice, st));
    if ((rc = stage(ctx, Ly, ctx->jobs, ctx->ws, st, L))) return rc;
    launch_scatter_meta(L, reinterpret_cast<const rdhei_meta *>(D + moff));
    if (!ok.empty()) {
        Layout S = subset_layout(Ly, ok);
        for (size_t q = 0; q < ok.size(); ++q) {
            const int i = ok[q];
            Job &J = S.jobs[q];
            J.fixed_b = chosen[(size_t)i];
            J.stream = D + soff + so[(size_t)i];
            J.stream_bits = sbits[(size_t)i];
        }
        Launch LS;
        if ((rc = stage(ctx, S, ctx->jobs, ctx->ws, st, LS))) return rc;
        if (S.units[UNIT_QROW]) launch_encrypt_tiles(LS, S.units[UNIT_QROW], ENC_LMR);
        for (int q : S.per_pixel) launch_generic_encrypt(LS, q, S.jobs[(size_t)q], ENC_LMR);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    T.device += secs(t3, Clock::now());
    return RDHEI_OK;
}

// Decode the maps of every usable LMR image of a layout (status OK, shape as
// recorded, stream length in range) and point its job at device bit planes;
// returns the usable jobs in ok.  A stream that fails to decode marks its
// image RDHEI_ECORRUPT.
int lmr_decode_batch(rdhei_ctx *ctx, Layout &Ly, int threads, LmrTimes &T, hipStream_t st, std::vector<int> &ok) {
    const int n = (int)Ly.jobs.size();
    std::vector<uint64_t> plane((size_t)n), poff((size_t)n), soffs((size_t)n, 0);
    uint64_t tot = 0, smax = 0;
    for (int i = 0; i < n; ++i) {
        const uint64_t MN = (uint64_t)Ly.jobs[(size_t)i].M * (uint64_t)Ly.jobs[(size_t)i].N;
        plane[(size_t)i] = align_up((MN + 7) / 8 + 16, 256);
        poff[(size_t)i] = tot;
        tot += 2 * plane[(size_t)i];
        soffs[(size_t)i] = smax;
        smax += plane[(size_t)i];
    }
    const uint64_t moff = tot, ooff = moff + align_up((uint64_t)n * sizeof(rdhei_meta), 256);
    const uint64_t soff = ooff + align_up((uint64_t)n * 8, 256), all = soff + smax;
    int rc;
    if ((rc = ctx->lmr_dev.need(all)) || (rc = ctx->lmr_host.need(all))) return rc;
    uint8_t *D = ctx->lmr_dev.p, *H = ctx->lmr_host.p;
    auto t0 = Clock::now();
    Launch L;
    if ((rc = stage(ctx, Ly, ctx->jobs, ctx->ws, st, L))) return rc;
    launch_gather_meta(L, reinterpret_cast<rdhei_meta *>(D + moff));
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(H + moff, D + moff, (size_t)n * sizeof(rdhei_meta), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    rdhei_meta *hm = reinterpret_cast<rdhei_meta *>(H + moff);
    uint64_t *ho = reinterpret_cast<uint64_t *>(H + ooff);
    uint64_t maxb = 0;
    ok.clear();
    for (int i = 0; i < n; ++i) {
        const Job &J = Ly.jobs[(size_t)i];
        const rdhei_meta &m = hm[i];
        const int64_t MN = (int64_t)J.M * J.N;
        ho[i] = soffs[(size_t)i];
        if (m.status == RDHEI_OK && m.method == RDHEI_LMR && m.height == J.M && m.width == J.N && m.map_bits >= 64 &&
            m.map_bits <= MN) {
            ok.push_back(i);
            maxb = std::max<uint64_t>(maxb, (uint64_t)(m.map_bits + 7) / 8);
        }
    }
    HIPCHK(hipMemcpyAsync(D + ooff, H + ooff, (size_t)n * 8, hipMemcpyHostToDevice, st));
    launch_msb_plane(L, reinterpret_cast<const uint64_t *>(D + ooff), D + soff, maxb);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(H + soff, D + soff, (size_t)smax, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    auto t1 = Clock::now();
    T.device += secs(t0, t1);
    std::vector<int> res(ok.size(), 0);
    parallel_for((int)ok.size(), threads, [&](int q) {
        const int i = ok[(size_t)q];
        const Job &J = Ly.jobs[(size_t)i];
        uint8_t *hl = H + poff[(size_t)i], *he = hl + plane[(size_t)i];
        res[(size_t)q] = lmr_decompress_impl(H + soff + soffs[(size_t)i], (hm[i].map_bits + 7) / 8, J.M, J.N, he, hl);
    });
    auto t2 = Clock::now();
    T.coder += secs(t1, t2);
    std::vector<int> good;
    bool corrupt = false;
    for (size_t q = 0; q < ok.size(); ++q) {
        const int i = ok[q];
        if (res[q] == RDHEI_OK) {
            good.push_back(i);
            Ly.jobs[(size_t)i].lbits = D + poff[(size_t)i];
            Ly.jobs[(size_t)i].etabits = D + poff[(size_t)i] + plane[(size_t)i];
        } else {
            hm[i].status = RDHEI_ECORRUPT;
            corrupt = true;
        }
    }
    ok.swap(good);
    HIPCHK(hipMemcpyAsync(D, H, (size_t)tot, hipMemcpyHostToDevice, st));
    if (corrupt) {
        HIPCHK(hipMemcpyAsync(D + moff, H + moff, (size_t)n * sizeof(rdhei_meta), hipMemcpyHostToDevice, st));
        launch_scatter_meta(L, reinterpret_cast<const rdhei_meta *>(D + moff));
    }
    T.device += secs(t2, Clock::now());
    return RDHEI_OK;
}

int lmr_batch(rdhei_ctx *ctx, int op, const rdhei_job *jobs, int n, int threads, LmrTimes &T, hipStream_t st) {
    if (op == RDHEI_OP_ENCRYPT) return lmr_encrypt_batch(ctx, jobs, n, threads, T, st);
    Layout Ly;
    int rc = make_layout(op, jobs, n, opts_of(ctx), Ly);
    if (rc) return rc;
    if (Ly.method != RDHEI_LMR) return RDHEI_EINVAL;
    std::vector<int> ok;
    if ((rc = lmr_decode_batch(ctx, Ly, threads, T, st, ok))) return rc;
    auto t0 = Clock::now();
    if (!ok.empty()) {
        Layout S = subset_layout(Ly, ok);
        Launch L;
        if ((rc = stage(ctx, S, ctx->jobs, ctx->ws, st, L))) return rc;
        for (const Stage &sg : stages_of(S, S.units, S.per_pixel)) sg.fn(L);
        HIPCHK(hipGetLastError());
    }
    HIPCHK(hipStreamSynchronize(st));
    T.device += secs(t0, Clock::now());
    return RDHEI_OK;
}

// Launch a plan's sequence (batched) or image by image.
int plan_issue(rdhei_plan *P, hipStream_t st) {
    Launch L;
    L.ws = P->ws.p;
    L.stream = st;
    L.max_grid = P->max_grid;
    const Layout &Ly = P->layout;
    L.keystream = Ly.keystream;
    L.dyn = Ly.method == RDHEI_DEMR;
    L.g_status = Ly.g_status;
    L.g_part = Ly.g_part;
    if (P->flags == RDHEI_PLAN_PER_IMAGE) {
        for (const rdhei_plan::One &o : P->per_image) {
            L.jobs = reinterpret_cast<const Job *>(P->single.p + o.table_off);
            for (int k = 0; k < UNIT_KINDS; ++k) L.ujob[k] = nullptr;
            L.njobs = 1;
            L.g_status = o.layout.g_status;
            L.g_part = o.layout.g_part;
            for (const Stage &s : o.stages) s.fn(L);
        }
    } else {
        L.jobs = P->base.jobs;
        for (int k = 0; k < UNIT_KINDS; ++k) L.ujob[k] = P->base.ujob[k];
        L.njobs = (int32_t)Ly.jobs.size();
        for (size_t i = 0; i < P->stages.size(); ++i) {
            L.max_grid = P->stage_grid[i] ? P->stage_grid[i] : P->max_grid;
            P->stages[i].fn(L);
        }
    }
    HIPCHK(hipGetLastError());
    return RDHEI_OK;
}

// ---- Autotuner helpers ------------------------------------------------------------

// Cache key of a plan: the device (architecture and compute units), the op,
// the keystream family, the per-pixel switch and the size class (log2 of the
// plan's pixels and images).
std::string tune_key(const rdhei_plan *P, int cus) {
    hipDeviceProp_t prop;
    std::string arch = "gpu";
    if (hipGetDeviceProperties(&prop, P->ctx->device) == hipSuccess) arch = prop.gcnArchName;
    for (char &c : arch)
        if (c == '"' || c == '\\' || c == ' ') c = '_';
    uint64_t px = 0;
    for (const rdhei_job &q : P->src) px += (uint64_t)q.height * (uint64_t)q.width;
    int px_cls = 0, job_cls = 0;
    while ((px >> px_cls) > 1) ++px_cls;
    while (((uint64_t)P->src.size() >> job_cls) > 1) ++job_cls;
    return arch + ":" + std::to_string(cus) + "cu/op" + std::to_string(P->op) + "/ks" + std::to_string(P->opts.keystream) +
           "/pp" + std::to_string(P->opts.per_pixel ? 1 : 0) + "/px" + std::to_string(px_cls) + "/jobs" +
           std::to_string(job_cls);
}

// Lay the plan out with a tuner record's variant (if it differs) and take its
// workgroup counts; drops a captured graph.
int plan_apply(rdhei_plan *P, const TuneRecord &v) {
    LayoutOpts o = P->opts;
    o.hide_mode = v.hide_mode;
    o.qseg = v.qseg;
    o.wg_image = v.wg_image;
    if (o.hide_mode != P->opts.hide_mode || o.qseg != P->opts.qseg || o.wg_image != P->opts.wg_image) {
        Layout Ly;
        int rc = make_layout(P->op, P->src.data(), (int)P->src.size(), o, Ly);
        if (rc) return rc;
        size_t off[UNIT_KINDS];
        if ((rc = P->jobs.need(table_bytes(Ly, off))) || (rc = P->ws.need(Ly.ws_bytes))) return rc;
        Launch L;
        if ((rc = upload_tables(Ly, P->jobs.p, nullptr, true, L))) return rc;
        L.keystream = Ly.keystream;
        L.dyn = Ly.method == RDHEI_DEMR;
        P->base = L;
        P->layout = Ly;
        P->opts = o;
        P->stages = stages_of(P->layout, P->layout.units, P->layout.per_pixel);
    }
    P->stage_grid.assign(P->stages.size(), 0);
    if (v.grids.size() == P->stages.size()) P->stage_grid = v.grids;
    if (P->exec) { (void)hipGraphExecDestroy(P->exec); P->exec = nullptr; }
    if (P->graph) { (void)hipGraphDestroy(P->graph); P->graph = nullptr; }
    return RDHEI_OK;
}

// The context's choices as JSON in its tune file (written to a temporary file,
// then renamed over the old one).
void tune_save(const rdhei_ctx *ctx) {
    if (ctx->tune_file.empty()) return;
    const std::string tmp = ctx->tune_file + ".tmp";
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) return;
    fprintf(f, "{\n  \"rdhei_tune\": 1,\n  \"entries\": {");
    bool first = true;
    for (const auto &kv : ctx->tuned) {
        fprintf(f, "%s\n    \"%s\": {\"hide_mode\": %d, \"qseg\": %d, \"wg_image\": %d, \"grids\": [", first ? "" : ",",
                kv.first.c_str(), kv.second.hide_mode, kv.second.qseg, kv.second.wg_image);
        for (size_t i = 0; i < kv.second.grids.size(); ++i) fprintf(f, "%s%d", i ? ", " : "", kv.second.grids[i]);
        fprintf(f, "]}");
        first = false;
    }
    fprintf(f, "\n  }\n}\n");
    const bool ok = fclose(f) == 0;
    if (ok) (void)std::rename(tmp.c_str(), ctx->tune_file.c_str());
}

// Reads the entries a tune file holds (the format tune_save writes); a missing
// file is an empty cache, a malformed one RDHEI_EINVAL.
int tune_load(rdhei_ctx *ctx) {
    FILE *f = fopen(ctx->tune_file.c_str(), "r");
    if (!f) return RDHEI_OK;
    std::string t;
    char buf[4096];
    size_t n;
    while ((n = fread(buf, 1, sizeof buf, f)) > 0) t.append(buf, n);
    fclose(f);
    size_t p = t.find("\"entries\"");
    if (p == std::string::npos) return RDHEI_EINVAL;
    p = t.find('{', p);
    if (p == std::string::npos) return RDHEI_EINVAL;
    auto int_after = [&](const std::string &name, size_t from, size_t to, int &out) {
        const size_t k = t.find("\"" + name + "\"", from);
        if (k == std::string::npos || k > to) return false;
        const size_t c = t.find(':', k);
        if (c == std::string::npos || c > to) return false;
        out = (int)strtol(t.c_str() + c + 1, nullptr, 10);
        return true;
    };
    std::map<std::string, TuneRecord> got;
    for (;;) {
        const size_t k0 = t.find('"', p + 1);
        if (k0 == std::string::npos) break;
        const size_t k1 = t.find('"', k0 + 1);
        const size_t o0 = k1 == std::string::npos ? std::string::npos : t.find('{', k1);
        const size_t o1 = o0 == std::string::npos ? std::string::npos : t.find('}', o0);
        if (o1 == std::string::npos) return RDHEI_EINVAL;
        TuneRecord r;
        if (!int_after("hide_mode", o0, o1, r.hide_mode) || !int_after("qseg", o0, o1, r.qseg)) return RDHEI_EINVAL;
        if (!int_after("wg_image", o0, o1, r.wg_image)) r.wg_image = 0;   // files written before the field existed
        if (r.hide_mode < 0 || r.hide_mode > 3 || r.qseg < 1 || r.qseg > kQuadSegMax || r.wg_image < 0 ||
            r.wg_image > 2)
            return RDHEI_EINVAL;
        const size_t g0 = t.find('[', o0), g1 = t.find(']', o0);
        if (g0 == std::string::npos || g1 == std::string::npos || g1 > o1) return RDHEI_EINVAL;
        for (const char *c = t.c_str() + g0 + 1; c < t.c_str() + g1;) {
            char *e = nullptr;
            const long v = strtol(c, &e, 10);
            if (e == c) { ++c; continue; }
            if (v < 0 || v > (1 << 30)) return RDHEI_EINVAL;
            r.grids.push_back((int)v);
            c = e;
        }
        got[t.substr(k0 + 1, k1 - k0 - 1)] = r;
        p = o1;
        const size_t nx = t.find_first_not_of(" \t\r\n", o1 + 1);
        if (nx == std::string::npos || t[nx] != ',') break;
        p = nx;
    }
    for (auto &kv : got) ctx->tuned[kv.first] = kv.second;
    return RDHEI_OK;
}

}  // namespace

// ---- Static scratch for callers that cannot allocate ------------------------------
// rdhei_run_batch_static keeps its job tables and workspace in this file-scope
// device array instead of allocating.  Every GPU the library runs on holds
// its own copy, at its own address, until the process ends.  In host code the
// name `scratch` is only a stand-in: kernels and copies get the address that
// hipGetSymbolAddress returns for the current device.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
static __device__ __align__(256) uint8_t scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint8_t *g_scratch_addr[kMaxDevices] = {};

// Device address of `scratch` on `device`, which must be the current device;
// looked up once per device.
int scratch_address(int device, uint8_t **out) {
    if (device < 0 || device >= kMaxDevices) return RDHEI_EINVAL;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_addr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_err("hipGetSymbolAddress(scratch)", e);
            return RDHEI_EDEVICE;
        }
        g_scratch_addr[device] = static_cast<uint8_t *>(p);
    }
    *out = g_scratch_addr[device];
    return RDHEI_OK;
}
}  // namespace

// ---- C ABI ---------------------------------------------------------------------------
extern "C" {

int rdhei_ctx_create(rdhei_ctx **out, int device) {
    if (!out) return RDHEI_EINVAL;
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess) {
        set_err("hipGetDeviceCount", e);
        return RDHEI_EDEVICE;
    }
    if (device < 0 || device >= n) return RDHEI_EINVAL;
    e = hipSetDevice(device);
    if (e != hipSuccess) {
        set_err("hipSetDevice", e);
        return RDHEI_EDEVICE;
    }
    uint8_t *sw = nullptr;
    const int rc = scratch_address(device, &sw);
    if (rc) return rc;
    rdhei_ctx *c = new (std::nothrow) rdhei_ctx();
    if (!c) return RDHEI_ENOMEM;
    c->device = device;
    c->static_ws = sw;
    *out = c;
    return RDHEI_OK;
}

void rdhei_ctx_destroy(rdhei_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    ctx->ws.release();
    ctx->jobs.release();
    ctx->scratch.release();
    ctx->batch_tables.release();
    ctx->lmr_dev.release();
    ctx->metrics.release();
    ctx->tileb.release();
    ctx->lmr_host.release();
    ctx->ring.release_all();
    delete ctx;
}

int rdhei_ctx_set_option(rdhei_ctx *ctx, int32_t option, int64_t value) {
    if (!ctx) return RDHEI_EINVAL;
    if (option == RDHEI_OPT_PER_PIXEL) ctx->per_pixel = value ? 1 : 0;
    else if (option == RDHEI_OPT_MAX_GRID) {
        if (value < 0 || value > (1 << 30)) return RDHEI_EINVAL;
        ctx->max_grid = (int)value;
    } else if (option == RDHEI_OPT_HIDE_MODE) {
        if (value < 0 || value > 3) return RDHEI_EINVAL;
        ctx->hide_mode = (int)value;
    } else if (option == RDHEI_OPT_LMR_MIN_LEVEL) {
        if (value < 1 || value > 4) return RDHEI_EINVAL;
        ctx->lmr_min_level = (int)value;
    } else if (option == RDHEI_OPT_KEYSTREAM) {
        if (value != RDHEI_KEYSTREAM_PHILOX && value != RDHEI_KEYSTREAM_CHACHA20) return RDHEI_EINVAL;
        ctx->keystream = (int)value;
    } else if (option == RDHEI_OPT_QUAD_SEG) {
        if (value < 1 || value > kQuadSegMax) return RDHEI_EINVAL;
        ctx->qseg = (int)value;
    } else if (option == RDHEI_OPT_WG_PER_IMAGE) {
        if (value < 0 || value > 2) return RDHEI_EINVAL;
        ctx->wg_image = (int)value;
    } else if (option == RDHEI_OPT_RESERVE_WS) {
        if (value < 0) return RDHEI_EINVAL;
        int rc = set_device(ctx->device);
        if (rc) return rc;
        return ctx->ws.need((size_t)value);
    } else return RDHEI_EINVAL;
    return RDHEI_OK;
}

int rdhei_encrypt(rdhei_ctx *ctx, const uint8_t *d_img, uint8_t *d_enc, int32_t M, int32_t N, uint64_t k1,
                  uint64_t nonce, int32_t method, rdhei_meta *d_meta, void *stream) {
    if (!ctx) return RDHEI_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (method == RDHEI_LMR) {
        if (!d_img || !d_enc || !d_meta || d_img == d_enc || M < 1 || N < 1) return RDHEI_EINVAL;
        return lmr_encrypt(ctx, d_img, d_enc, M, N, k1, nonce, d_meta, st);
    }
    if (method != RDHEI_EMR) return RDHEI_EINVAL;
    rdhei_job q{};
    q.in = d_img; q.out = d_enc; q.meta = d_meta; q.key = k1; q.nonce = nonce;
    q.height = M; q.width = N; q.method = RDHEI_EMR;
    return run_single(ctx, RDHEI_OP_ENCRYPT, q, st);
}

int rdhei_embed(rdhei_ctx *ctx, uint8_t *d_marked, int32_t M, int32_t N, int32_t method, rdhei_meta *d_meta,
                const uint8_t *d_msg, int64_t nbits, uint64_t k2, void *stream) {
    if (!ctx || !d_marked || !d_meta || !d_msg || !aligned16(d_msg) || M < 1 || N < 1) return RDHEI_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (method == RDHEI_LMR)
        return lmr_stage(ctx, RDHEI_OP_EMBED, d_marked, d_marked, M, N, d_meta, const_cast<uint8_t *>(d_msg), nbits, k2, st);
    if (method != RDHEI_EMR) return RDHEI_EINVAL;
    rdhei_job q{};
    q.out = d_marked; q.msg = const_cast<uint8_t *>(d_msg); q.meta = d_meta; q.key = k2; q.nbits = nbits;
    q.height = M; q.width = N; q.method = RDHEI_EMR;
    return run_single(ctx, RDHEI_OP_EMBED, q, st);
}

int rdhei_extract(rdhei_ctx *ctx, const uint8_t *d_marked, int32_t M, int32_t N, int32_t method,
                  rdhei_meta *d_meta, uint8_t *d_msg, int64_t nbits, uint64_t k2, void *stream) {
    if (!ctx || !d_marked || !d_meta || !d_msg || !aligned16(d_msg) || M < 1 || N < 1) return RDHEI_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (method == RDHEI_LMR)
        return lmr_stage(ctx, RDHEI_OP_EXTRACT, d_marked, nullptr, M, N, d_meta, d_msg, nbits, k2, st);
    if (method != RDHEI_EMR) return RDHEI_EINVAL;
    rdhei_job q{};
    q.in = d_marked; q.msg = d_msg; q.meta = d_meta; q.key = k2; q.nbits = nbits;
    q.height = M; q.width = N; q.method = RDHEI_EMR;
    return run_single(ctx, RDHEI_OP_EXTRACT, q, st);
}

int rdhei_recover(rdhei_ctx *ctx, const uint8_t *d_marked, int32_t M, int32_t N, int32_t method,
                  rdhei_meta *d_meta, uint8_t *d_img, uint64_t k1, void *stream) {
    if (!ctx || !d_marked || !d_meta || !d_img || d_marked == d_img || M < 1 || N < 1) return RDHEI_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (method == RDHEI_LMR)
        return lmr_stage(ctx, RDHEI_OP_RECOVER, d_marked, d_img, M, N, d_meta, nullptr, 0, k1, st);
    if (method != RDHEI_EMR) return RDHEI_EINVAL;
    rdhei_job q{};
    q.in = d_marked; q.out = d_img; q.meta = d_meta; q.key = k1;
    q.height = M; q.width = N; q.method = RDHEI_EMR;
    return run_single(ctx, RDHEI_OP_RECOVER, q, st);
}

int rdhei_lmr_batch(rdhei_ctx *ctx, int32_t op, const rdhei_job *jobs, int32_t njobs, int32_t threads,
                    double *times, void *stream) {
    if (!ctx || !jobs || njobs < 1 || threads < 0) return RDHEI_EINVAL;
    if (op < RDHEI_OP_ENCRYPT || op > RDHEI_OP_RECOVER) return RDHEI_EINVAL;
    int rc = set_device(ctx->device);
    if (rc) return rc;
    LmrTimes T;
    const auto t0 = Clock::now();
    rc = lmr_batch(ctx, op, jobs, njobs, threads, T, reinterpret_cast<hipStream_t>(stream));
    if (times) {
        times[0] = T.device;
        times[1] = T.coder;
        times[2] = secs(t0, Clock::now());
    }
    return rc;
}

int rdhei_workspace_size(rdhei_ctx *ctx, int32_t op, const rdhei_job *jobs, int32_t njobs, int64_t *bytes) {
    if (!ctx || !jobs || njobs < 1 || !bytes) return RDHEI_EINVAL;
    int rc = set_device(ctx->device);
    if (rc) return rc;
    Layout Ly;
    rc = make_layout(op, jobs, njobs, opts_of(ctx), Ly);
    if (rc) return rc;
    *bytes = (int64_t)Ly.ws_bytes;
    return RDHEI_OK;
}

int rdhei_metrics(rdhei_ctx *ctx, const rdhei_metric_job *jobs, int32_t njobs, int32_t flags, double *d_out,
                  void *stream) {
    if (!ctx || !jobs || njobs < 1 || !d_out || (flags & ~RDHEI_METRIC_SSIM)) return RDHEI_EINVAL;
    int rc = set_device(ctx->device);
    if (rc) return rc;
    const bool with_ssim = (flags & RDHEI_METRIC_SSIM) != 0;
    std::vector<MetricJob> hj((size_t)njobs);
    uint64_t units = 0, tiles = 0;
    for (int i = 0; i < njobs; ++i) {
        const rdhei_metric_job &q = jobs[i];
        if (!q.a || q.height < 1 || q.width < 1) return RDHEI_EINVAL;
        MetricJob &m = hj[(size_t)i];
        m.a = q.a;
        m.b = q.b;
        m.M = q.height;
        m.N = q.width;
        m.vec = aligned16(q.a) && (!q.b || aligned16(q.b)) ? 1 : 0;
        m.pad = 0;
        const uint64_t MN = (uint64_t)q.height * (uint64_t)q.width;
        m.sum_first = (uint32_t)units;
        m.ssim_first = (uint32_t)tiles;
        units += (MN + kMetricChunk - 1) / kMetricChunk;
        if (with_ssim && q.b && q.height >= kSsimWin && q.width >= kSsimWin)
            tiles += (uint64_t)((q.height - kSsimWin + 1 + kSsimRows - 1) / kSsimRows) *
                     (uint64_t)((q.width - kSsimWin + 1 + kSsimCols - 1) / kSsimCols);
        if (units > 0xFFFFFFFFull || tiles > 0xFFFFFFFFull) return RDHEI_EINVAL;
    }
    // device: job table, then the accumulators
    const size_t tb = align_up((uint64_t)njobs * sizeof(MetricJob), 256);
    const size_t total = tb + (size_t)njobs * sizeof(MetricAcc);
    rc = ctx->metrics.need(total);
    if (rc) return rc;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    uint8_t *host = nullptr;
    int slot = 0;
    rc = ctx->ring.acquire(tb, &host, &slot);
    if (rc) return rc;
    memcpy(host, hj.data(), (size_t)njobs * sizeof(MetricJob));
    HIPCHK(hipMemcpyAsync(ctx->metrics.p, host, (size_t)njobs * sizeof(MetricJob), hipMemcpyHostToDevice, st));
    HIPCHK(hipEventRecord(ctx->ring.done[slot], st));
    ctx->ring.used[slot] = true;
    launch_metrics(reinterpret_cast<const MetricJob *>(ctx->metrics.p), njobs,
                   reinterpret_cast<MetricAcc *>(ctx->metrics.p + tb), (uint32_t)units, (uint32_t)tiles,
                   with_ssim ? 1 : 0, d_out, st);
    HIPCHK(hipGetLastError());
    return RDHEI_OK;
}

int rdhei_tile_b(rdhei_ctx *ctx, const rdhei_metric_job *jobs, int32_t njobs, uint8_t *d_tile_b, int64_t *d_capacity,
                 void *stream) {
    if (!ctx || !jobs || njobs < 1 || !d_tile_b || !d_capacity) return RDHEI_EINVAL;
    std::vector<TileBJob> hj((size_t)njobs);
    uint64_t tiles = 0;
    for (int i = 0; i < njobs; ++i) {
        const rdhei_metric_job &q = jobs[i];
        if (!q.a || !aligned16(q.a) || q.height < kTile || q.width < kTile || q.height % kTile || q.width % kTile)
            return RDHEI_EINVAL;
        TileBJob &t = hj[(size_t)i];
        t.img = q.a;
        t.M = q.height;
        t.N = q.width;
        t.tile_first = (uint32_t)tiles;
        t.pad = 0;
        tiles += (uint64_t)(q.height / kTile) * (uint64_t)(q.width / kTile);
        if (tiles > (1ull << 31)) return RDHEI_EINVAL;   // tile indices and the grid stride stay below 2^32
    }
    int rc = set_device(ctx->device);
    if (rc) return rc;
    const size_t tb = (size_t)njobs * sizeof(TileBJob);
    rc = ctx->tileb.need(tb);
    if (rc) return rc;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    uint8_t *host = nullptr;
    int slot = 0;
    rc = ctx->ring.acquire(tb, &host, &slot);
    if (rc) return rc;
    memcpy(host, hj.data(), tb);
    HIPCHK(hipMemcpyAsync(ctx->tileb.p, host, tb, hipMemcpyHostToDevice, st));
    HIPCHK(hipEventRecord(ctx->ring.done[slot], st));
    ctx->ring.used[slot] = true;
    launch_tile_b(reinterpret_cast<const TileBJob *>(ctx->tileb.p), njobs, (uint32_t)tiles, d_tile_b, d_capacity, st);
    HIPCHK(hipGetLastError());
    return RDHEI_OK;
}

int rdhei_run_batch(rdhei_ctx *ctx, int32_t op, const rdhei_job *jobs, int32_t njobs, void *d_workspace,
                    int64_t workspace_bytes, void *stream) {
    if (!ctx || !jobs || njobs < 1) return RDHEI_EINVAL;
    if (d_workspace && ((uintptr_t)d_workspace & 255)) return RDHEI_EINVAL;
    int rc = set_device(ctx->device);
    if (rc) return rc;
    Layout Ly;
    rc = make_layout(op, jobs, njobs, opts_of(ctx), Ly);
    if (rc) return rc;
    if (Ly.method == RDHEI_LMR) return RDHEI_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    uint8_t *ws = (uint8_t *)d_workspace;
    if (ws) {
        if (workspace_bytes < (int64_t)Ly.ws_bytes) return RDHEI_EINVAL;
    } else {
        rc = ctx->ws.need(Ly.ws_bytes);
        if (rc) return rc;
        ws = ctx->ws.p;
    }
    size_t off[UNIT_KINDS];
    const size_t tb = table_bytes(Ly, off);
    // device tables: one region per staging slot inside one buffer, so a new
    // batch never overwrites tables that an earlier launch may still read
    // (stream order makes a region safe to rewrite kSlots calls later)
    const size_t region = align_up(std::max<size_t>(tb, 1 << 16), 256);
    if (ctx->batch_tables.n < PinnedRing::kSlots * region) {
        rc = ctx->batch_tables.need(PinnedRing::kSlots * region);  // synchronises
        if (rc) return rc;
    }
    uint8_t *host = nullptr;
    int slot = 0;
    rc = ctx->ring.acquire(tb, &host, &slot);
    if (rc) return rc;
    uint8_t *dtab = ctx->batch_tables.p + (size_t)slot * (ctx->batch_tables.n / PinnedRing::kSlots);
    memcpy(host, Ly.jobs.data(), Ly.jobs.size() * sizeof(Job));
    for (int k = 0; k < UNIT_KINDS; ++k)
        if (!Ly.ujob[k].empty()) memcpy(host + off[k], Ly.ujob[k].data(), Ly.ujob[k].size() * 4);
    HIPCHK(hipMemcpyAsync(dtab, host, tb, hipMemcpyHostToDevice, st));
    HIPCHK(hipEventRecord(ctx->ring.done[slot], st));
    ctx->ring.used[slot] = true;
    Launch L;
    L.jobs = reinterpret_cast<const Job *>(dtab);
    for (int k = 0; k < UNIT_KINDS; ++k) L.ujob[k] = Ly.ujob[k].empty() ? nullptr : reinterpret_cast<const uint32_t *>(dtab + off[k]);
    L.njobs = (int32_t)Ly.jobs.size();
    L.ws = ws;
    L.stream = st;
    L.max_grid = ctx->max_grid;
    L.g_status = Ly.g_status;
    L.g_part = Ly.g_part;
    L.keystream = Ly.keystream;
    L.dyn = Ly.method == RDHEI_DEMR;
    for (const Stage &sg : stages_of(Ly, Ly.units, Ly.per_pixel)) sg.fn(L);
    HIPCHK(hipGetLastError());
    return RDHEI_OK;
}

// Several ops of one batch in stream order, sharing one workspace: every
// op's layout, then all their tables in one staging slot and one upload.
static int roles_layouts(rdhei_ctx *ctx, int32_t n_ops, const int32_t *ops, const rdhei_job *const *jobs,
                         const int32_t *njobs, std::vector<Layout> &lys, uint64_t &ws_bytes) {
    if (!ctx || n_ops < 1 || n_ops > 8 || !ops || !jobs || !njobs) return RDHEI_EINVAL;
    lys.assign((size_t)n_ops, Layout());
    ws_bytes = 256;
    for (int i = 0; i < n_ops; ++i) {
        if (!jobs[i] || njobs[i] < 1) return RDHEI_EINVAL;
        const int rc = make_layout(ops[i], jobs[i], njobs[i], opts_of(ctx), lys[(size_t)i]);
        if (rc) return rc;
        if (lys[(size_t)i].method == RDHEI_LMR) return RDHEI_EINVAL;
        ws_bytes = std::max<uint64_t>(ws_bytes, lys[(size_t)i].ws_bytes);
    }
    return RDHEI_OK;
}

int rdhei_roles_workspace_size(rdhei_ctx *ctx, int32_t n_ops, const int32_t *ops, const rdhei_job *const *jobs,
                               const int32_t *njobs, int64_t *bytes) {
    if (!ctx || !bytes) return RDHEI_EINVAL;
    const int rs = set_device(ctx->device);
    if (rs) return rs;
    std::vector<Layout> lys;
    uint64_t ws = 0;
    const int rc = roles_layouts(ctx, n_ops, ops, jobs, njobs, lys, ws);
    if (rc) return rc;
    *bytes = (int64_t)ws;
    return RDHEI_OK;
}

int rdhei_run_roles(rdhei_ctx *ctx, int32_t n_ops, const int32_t *ops, const rdhei_job *const *jobs,
                    const int32_t *njobs, void *d_workspace, int64_t workspace_bytes, void *stream) {
    if (!ctx || ((uintptr_t)d_workspace & 255)) return RDHEI_EINVAL;
    int rc = set_device(ctx->device);
    if (rc) return rc;
    std::vector<Layout> lys;
    uint64_t ws_need = 0;
    rc = roles_layouts(ctx, n_ops, ops, jobs, njobs, lys, ws_need);
    if (rc) return rc;
    uint8_t *ws = (uint8_t *)d_workspace;
    if (ws) {
        if (workspace_bytes < (int64_t)ws_need) return RDHEI_EINVAL;
    } else {
        rc = ctx->ws.need(ws_need);
        if (rc) return rc;
        ws = ctx->ws.p;
    }
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    // the ops' tables back to back in one staging slot
    std::vector<size_t> base((size_t)n_ops);
    std::vector<std::array<size_t, UNIT_KINDS>> offs((size_t)n_ops);
    size_t tb = 0;
    for (int i = 0; i < n_ops; ++i) {
        base[(size_t)i] = tb;
        tb += align_up(table_bytes(lys[(size_t)i], offs[(size_t)i].data()), 256);
    }
    const size_t region = align_up(std::max<size_t>(tb, 1 << 16), 256);
    if (ctx->batch_tables.n / PinnedRing::kSlots < region) {
        rc = ctx->batch_tables.need(PinnedRing::kSlots * region);   // synchronises
        if (rc) return rc;
    }
    uint8_t *host = nullptr;
    int slot = 0;
    rc = ctx->ring.acquire(tb, &host, &slot);
    if (rc) return rc;
    uint8_t *dtab = ctx->batch_tables.p + (size_t)slot * (ctx->batch_tables.n / PinnedRing::kSlots);
    for (int i = 0; i < n_ops; ++i) {
        const Layout &Ly = lys[(size_t)i];
        uint8_t *h = host + base[(size_t)i];
        memcpy(h, Ly.jobs.data(), Ly.jobs.size() * sizeof(Job));
        for (int k = 0; k < UNIT_KINDS; ++k)
            if (!Ly.ujob[k].empty()) memcpy(h + offs[(size_t)i][k], Ly.ujob[k].data(), Ly.ujob[k].size() * 4);
    }
    HIPCHK(hipMemcpyAsync(dtab, host, tb, hipMemcpyHostToDevice, st));
    HIPCHK(hipEventRecord(ctx->ring.done[slot], st));
    ctx->ring.used[slot] = true;
    for (int i = 0; i < n_ops; ++i) {
        const Layout &Ly = lys[(size_t)i];
        uint8_t *d = dtab + base[(size_t)i];
        Launch L;
        L.jobs = reinterpret_cast<const Job *>(d);
        for (int k = 0; k < UNIT_KINDS; ++k)
            L.ujob[k] = Ly.ujob[k].empty() ? nullptr : reinterpret_cast<const uint32_t *>(d + offs[(size_t)i][k]);
        L.njobs = (int32_t)Ly.jobs.size();
        L.ws = ws;
        L.stream = st;
        L.max_grid = ctx->max_grid;
        L.g_status = Ly.g_status;
        L.g_part = Ly.g_part;
        L.keystream = Ly.keystream;
        L.dyn = Ly.method == RDHEI_DEMR;
        for (const Stage &sg : stages_of(Ly, Ly.units, Ly.per_pixel)) sg.fn(L);
    }
    HIPCHK(hipGetLastError());
    return RDHEI_OK;
}

int rdhei_run_batch_static(rdhei_ctx *ctx, int32_t op, const rdhei_job *jobs, int32_t njobs, void *stream) {
    if (!ctx || !jobs || njobs < 1) return RDHEI_EINVAL;
    if (!ctx->static_ws) return RDHEI_EDEVICE;
    int rc = set_device(ctx->device);
    if (rc) return rc;
    Layout Ly;
    rc = make_layout(op, jobs, njobs, opts_of(ctx), Ly);
    if (rc) return rc;
    if (Ly.method == RDHEI_LMR) return RDHEI_EINVAL;
    size_t off[UNIT_KINDS];
    const uint64_t tb = align_up(table_bytes(Ly, off), 256);
    if (tb + Ly.ws_bytes > kStaticScratchBytes) {
        char buf[160];
        snprintf(buf, sizeof buf, "rdhei_run_batch_static: batch needs %llu bytes of scratch, the static array holds %llu",
                 (unsigned long long)(tb + Ly.ws_bytes), (unsigned long long)kStaticScratchBytes);
        g_err = buf;
        return RDHEI_ENOMEM;
    }
    // job and unit tables at the start of the array, the workspace after them;
    // the tables are copied from pageable host memory, which the copy stages
    // before it returns, so nothing outlives the call
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    uint8_t *base = ctx->static_ws;
    Launch L;
    rc = upload_tables(Ly, base, st, false, L);
    if (rc) return rc;
    L.njobs = (int32_t)Ly.jobs.size();
    L.ws = base + tb;
    L.stream = st;
    L.max_grid = ctx->max_grid;
    L.g_status = Ly.g_status;
    L.g_part = Ly.g_part;
    L.keystream = Ly.keystream;
    L.dyn = Ly.method == RDHEI_DEMR;
    for (const Stage &sg : stages_of(Ly, Ly.units, Ly.per_pixel)) sg.fn(L);
    HIPCHK(hipGetLastError());
    return RDHEI_OK;
}

int rdhei_plan_create(rdhei_ctx *ctx, int32_t op, const rdhei_job *jobs, int32_t njobs, int32_t flags,
                      rdhei_plan **out) {
    if (!ctx || !jobs || njobs < 1 || !out) return RDHEI_EINVAL;
    if (flags != RDHEI_PLAN_GRAPH && flags != RDHEI_PLAN_EAGER && flags != RDHEI_PLAN_PER_IMAGE) return RDHEI_EINVAL;
    *out = nullptr;
    int rc = set_device(ctx->device);
    if (rc) return rc;
    rdhei_plan *P = new (std::nothrow) rdhei_plan();
    if (!P) return RDHEI_ENOMEM;
    P->ctx = ctx;
    P->op = op;
    P->flags = flags;
    P->max_grid = ctx->max_grid;
    P->opts = opts_of(ctx);
    P->src.assign(jobs, jobs + njobs);
    rc = make_layout(op, jobs, njobs, P->opts, P->layout);
    if (!rc && P->layout.method == RDHEI_LMR) rc = RDHEI_EINVAL;
    size_t toff[UNIT_KINDS];
    if (!rc) rc = P->jobs.need(table_bytes(P->layout, toff));
    if (!rc) rc = P->ws.need(P->layout.ws_bytes);
    if (!rc) rc = upload_tables(P->layout, P->jobs.p, nullptr, true, P->base);
    P->base.keystream = P->layout.keystream;
    P->base.dyn = P->layout.method == RDHEI_DEMR;
    if (!rc && flags == RDHEI_PLAN_PER_IMAGE) {
        P->per_image.resize((size_t)njobs);
        size_t total = 0;
        uint64_t ws = P->layout.ws_bytes;
        for (int i = 0; i < njobs && !rc; ++i) {
            rdhei_plan::One &o = P->per_image[(size_t)i];
            rc = make_layout(op, jobs + i, 1, opts_of(ctx), o.layout);
            o.table_off = total;
            size_t off1[UNIT_KINDS];
            total += align_up(table_bytes(o.layout, off1), 256);
            ws = std::max<uint64_t>(ws, o.layout.ws_bytes);
        }
        if (!rc) rc = P->single.need(total);
        if (!rc) rc = P->ws.need(ws);
        for (int i = 0; i < njobs && !rc; ++i) {
            rdhei_plan::One &o = P->per_image[(size_t)i];
            hipError_t e = hipMemcpy(P->single.p + o.table_off, o.layout.jobs.data(), sizeof(Job), hipMemcpyHostToDevice);
            if (e != hipSuccess) { set_err("hipMemcpy", e); rc = RDHEI_EDEVICE; }
            o.stages = stages_of(o.layout, o.layout.units, o.layout.per_pixel);
        }
    }
    if (rc) {
        P->jobs.release();
        P->ws.release();
        P->single.release();
        delete P;
        return rc;
    }
    P->stages = stages_of(P->layout, P->layout.units, P->layout.per_pixel);
    P->stage_grid.assign(P->stages.size(), 0);
    *out = P;
    return RDHEI_OK;
}

int rdhei_plan_set_grid(rdhei_plan *plan, int32_t max_workgroups) {
    if (!plan || max_workgroups < 0) return RDHEI_EINVAL;
    if (plan->max_grid != max_workgroups || std::any_of(plan->stage_grid.begin(), plan->stage_grid.end(),
                                                          [](int g) { return g != 0; })) {
        plan->max_grid = max_workgroups;
        std::fill(plan->stage_grid.begin(), plan->stage_grid.end(), 0);
        if (plan->exec) { (void)hipGraphExecDestroy(plan->exec); plan->exec = nullptr; }
        if (plan->graph) { (void)hipGraphDestroy(plan->graph); plan->graph = nullptr; }
    }
    return RDHEI_OK;
}

int rdhei_plan_run(rdhei_plan *P, void *stream) {
    if (!P) return RDHEI_EINVAL;
    int rc = set_device(P->ctx->device);
    if (rc) return rc;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (P->flags != RDHEI_PLAN_GRAPH) return plan_issue(P, st);
    if (!P->exec) {
        hipStream_t cap;
        HIPCHK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
        hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) { (void)hipStreamDestroy(cap); set_err("hipStreamBeginCapture", e); return RDHEI_EDEVICE; }
        rc = plan_issue(P, cap);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(cap, &g);
        (void)hipStreamDestroy(cap);
        if (rc) { if (g) (void)hipGraphDestroy(g); return rc; }
        if (e != hipSuccess) { set_err("hipStreamEndCapture", e); return RDHEI_EDEVICE; }
        e = hipGraphInstantiate(&P->exec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) { (void)hipGraphDestroy(g); set_err("hipGraphInstantiate", e); return RDHEI_EDEVICE; }
        P->graph = g;
    }
    HIPCHK(hipGraphLaunch(P->exec, st));
    return RDHEI_OK;
}

int rdhei_plan_stage_count(rdhei_plan *P) { return P ? (int)P->stages.size() : RDHEI_EINVAL; }

const char *rdhei_plan_stage_name(rdhei_plan *P, int32_t k) {
    if (!P || k < 0 || k >= (int)P->stages.size()) return "";
    return P->stages[(size_t)k].name;
}

int rdhei_plan_run_stage(rdhei_plan *P, int32_t k, void *stream) {
    if (!P || k < 0 || k >= (int)P->stages.size()) return RDHEI_EINVAL;
    int rc = set_device(P->ctx->device);
    if (rc) return rc;
    Launch L = P->base;
    L.njobs = (int32_t)P->layout.jobs.size();
    L.g_status = P->layout.g_status;
    L.g_part = P->layout.g_part;
    L.ws = P->ws.p;
    L.stream = reinterpret_cast<hipStream_t>(stream);
    L.max_grid = P->stage_grid[(size_t)k] ? P->stage_grid[(size_t)k] : P->max_grid;
    P->stages[(size_t)k].fn(L);
    HIPCHK(hipGetLastError());
    return RDHEI_OK;
}

int rdhei_plan_stage_grid(rdhei_plan *P, int32_t k) {
    if (!P || k < 0 || k >= (int)P->stages.size()) return RDHEI_EINVAL;
    return P->stage_grid[(size_t)k];
}

int rdhei_plan_autotune(rdhei_plan *P, int32_t reps, int32_t flags, void *stream) {
    if (!P || reps < 1 || reps > 1000 || (flags & ~RDHEI_TUNE_FORCE)) return RDHEI_EINVAL;
    if (P->flags == RDHEI_PLAN_PER_IMAGE) return RDHEI_OK;      // per-image launches keep their defaults
    int rc = set_device(P->ctx->device);
    if (rc) return rc;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    rdhei_ctx *ctx = P->ctx;
    int cus = 0;
    HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device));
    const std::string key = tune_key(P, cus);
    auto it = ctx->tuned.find(key);
    if (it != ctx->tuned.end() && !(flags & RDHEI_TUNE_FORCE)) {
        rc = plan_apply(P, it->second);
        if (rc) return rc;
        rc = plan_issue(P, st);
        if (rc) return rc;
        HIPCHK(hipStreamSynchronize(st));
        return RDHEI_OK;
    }
    const int samples = std::max<int>(reps, 5);
    const LayoutOpts base = P->opts;
    // layout variants: the hiding mode of embed/extract plans (whole images
    // where the batch has them, steps in one pass, counted steps), the quads
    // per work unit of encrypt/recover plans with band pairs of more than one
    // quad
    std::vector<TuneRecord> variants;
    {
        TuneRecord v0;
        v0.hide_mode = base.hide_mode;
        v0.qseg = base.qseg;
        v0.wg_image = base.wg_image;
        variants.push_back(v0);
        const bool hide = P->op == RDHEI_OP_EMBED || P->op == RDHEI_OP_EXTRACT;
        bool eligible = false;
        uint32_t max_nq = 0;
        for (const rdhei_job &q : P->src) {
            eligible = eligible || whole_eligible(P->op, q);
            if (q.height % kTile == 0 && q.width % kTile == 0) max_nq = std::max<uint32_t>(max_nq, (uint32_t)(q.width / kTile + 1) / 2);
        }
        // whole images (where the batch allows), steps in one pass, counted steps
        if (hide)
            for (int hm : {1, 3, 2}) {
                if (hm == v0.hide_mode || (hm == 1 && !eligible)) continue;
                TuneRecord v = v0;
                v.hide_mode = hm;
                variants.push_back(v);
            }
        // encryption / recovery by stages or one workgroup per image (where the batch allows)
        const bool img_ok = wg_image_ok(P->op, P->src.data(), (int)P->src.size(), base.per_pixel);
        if (img_ok) {
            TuneRecord v = v0;
            v.wg_image = P->layout.images ? 1 : 2;
            variants.push_back(v);
        }
        // quads per work unit (stage-wise encryption and recovery)
        if (!hide && max_nq > 1)
            for (int qs : {2, 4, 8, 16}) {
                if (qs == v0.qseg || (uint32_t)qs / 2 >= max_nq) continue;   // longer than every band pair: same as a shorter one
                TuneRecord v = v0;
                v.qseg = qs;
                if (img_ok) v.wg_image = 1;
                variants.push_back(v);
            }
    }
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    // one timed run of stage k at the plan's current grid choice
    auto time_stage = [&](size_t k, float &ms) -> int {
        if (hipEventRecord(e0, st) != hipSuccess) return RDHEI_EDEVICE;
        int r = rdhei_plan_run_stage(P, (int32_t)k, stream);
        if (r) return r;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return RDHEI_EDEVICE;
        return RDHEI_OK;
    };
    const int cand[] = {0, cus, 2 * cus, 4 * cus, 8 * cus, 16 * cus, 32 * cus};
    TuneRecord best_v;
    float best_total = 0.f, best_spread = 0.f;
    for (size_t vi = 0; vi < variants.size() && !rc; ++vi) {
        TuneRecord v = variants[vi];
        v.grids.clear();
        rc = plan_apply(P, v);
        if (rc) break;
        // the stages read what the stages before them wrote: bring the
        // plan's buffers to a consistent state first (every stage is idempotent)
        rc = plan_issue(P, st);
        if (rc) break;
        float total = 0.f, spread = 0.f;
        for (size_t k = 0; k < P->stages.size() && !rc; ++k) {
            // per candidate: the median and the spread (max - min) of `samples`
            // timed runs after one warm-up; a candidate replaces the current
            // choice only when its median is lower by more than the two
            // spreads together (and by 2 % at least)
            float cm = 0.f, cs = 0.f;
            int cg = 0;
            bool have = false;
            for (int g : cand) {
                P->stage_grid[k] = g;
                rc = rdhei_plan_run_stage(P, (int32_t)k, stream);
                if (rc) break;
                std::vector<float> t((size_t)samples);
                for (int r = 0; r < samples && !rc; ++r) rc = time_stage(k, t[(size_t)r]);
                if (rc) break;
                std::sort(t.begin(), t.end());
                const float med = t[t.size() / 2], spr = t.back() - t.front();
                if (!have || med < cm - std::max(0.02f * cm, 0.5f * (cs + spr))) {
                    cm = med;
                    cs = spr;
                    cg = g;
                    have = true;
                }
            }
            P->stage_grid[k] = cg;
            v.grids.push_back(cg);
            total += cm;
            spread += cs;
        }
        if (rc) break;
        if (vi == 0 || total < best_total - std::max(0.02f * best_total, 0.5f * (best_spread + spread))) {
            best_total = total;
            best_spread = spread;
            best_v = v;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    rc = plan_apply(P, best_v);
    if (rc) return rc;
    ctx->tuned[key] = best_v;
    tune_save(ctx);
    // leave the buffers as one run with the chosen shapes leaves them
    rc = plan_issue(P, st);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(st));
    return RDHEI_OK;
}

int rdhei_plan_tuned(rdhei_plan *P, int32_t *hide_mode, int32_t *qseg, int32_t *wg_image) {
    if (!P) return RDHEI_EINVAL;
    if (hide_mode) *hide_mode = P->opts.hide_mode;
    if (qseg) *qseg = P->opts.qseg;
    if (wg_image) *wg_image = P->opts.wg_image;
    return RDHEI_OK;
}

int rdhei_ctx_set_tune_file(rdhei_ctx *ctx, const char *path) {
    if (!ctx) return RDHEI_EINVAL;
    ctx->tune_file = path ? path : "";
    if (ctx->tune_file.empty()) return RDHEI_OK;
    return tune_load(ctx);
}

void rdhei_plan_destroy(rdhei_plan *P) {
    if (!P) return;
    (void)hipSetDevice(P->ctx->device);
    (void)hipDeviceSynchronize();
    if (P->exec) (void)hipGraphExecDestroy(P->exec);
    if (P->graph) (void)hipGraphDestroy(P->graph);
    P->jobs.release();
    P->ws.release();
    P->single.release();
    delete P;
}

int rdhei_lmr_compress(const uint8_t *eta_bits, const uint8_t *l_bits, int32_t M, int32_t N, uint8_t *stream,
                       int64_t capacity_bytes, int64_t *stream_bits) {
    if (!eta_bits || !l_bits || !stream || !stream_bits || M < 1 || N < 1 || capacity_bytes < 8) return RDHEI_EINVAL;
    return lmr_compress_impl(eta_bits, l_bits, M, N, stream, capacity_bytes, stream_bits);
}

int rdhei_lmr_decompress(const uint8_t *stream, int64_t stream_bytes, int32_t M, int32_t N, uint8_t *eta_bits,
                         uint8_t *l_bits) {
    if (!stream || !eta_bits || !l_bits || M < 1 || N < 1 || stream_bytes < 8) return RDHEI_EINVAL;
    return lmr_decompress_impl(stream, stream_bytes, M, N, eta_bits, l_bits);
}

const char *rdhei_strerror(int code) {
    switch (code) {
        case RDHEI_OK: return "ok";
        case RDHEI_EINVAL: return "invalid argument";
        case RDHEI_ECAPACITY: return "message longer than the capacity";
        case RDHEI_ENOFIT: return "LMR maps do not compress into the MSB plane";
        case RDHEI_ENOMEM: return "out of memory";
        case RDHEI_EDEVICE: return "HIP runtime error";
        case RDHEI_ECORRUPT: return "malformed LMR map stream";
        default: return "unknown error";
    }
}

const char *rdhei_last_error(void) { return g_err.c_str(); }

const char *rdhei_version(void) { return "rdhei 0.1 gfx950"; }

}  // extern "C"

/*
 * rdhei.h -- C ABI of the MI355X (gfx950) EMR-/LMR-RDHEI library.
 *
 * Method: Zhang & Luo, "Vector-based Efficient Data Hiding in Encrypted Images
 * via Multi-MSB Replacement" (arXiv 2302.07992).  The three roles of the
 * reserving-room-before-encryption scheme (Sec. I, RRBE figure; Sec. III):
 *   content owner  -> rdhei_encrypt   (key K1: location map, rotation, XOR)
 *   data hider     -> rdhei_embed     (key K2: multi-MSB replacement)
 *   recipient      -> rdhei_extract   (key K2) and/or rdhei_recover (key K1)
 *
 * Conventions shared by every entry point
 *   - Images are 8-bit grey, row-major, height M rows by width N columns,
 *     M*N bytes, in DEVICE memory owned by the caller.  The fast tiled path
 *     is taken when M and N are multiples of 64 and buffers are 16-byte
 *     aligned; every other shape runs a per-pixel path with identical output.
 *   - Messages are bit strings packed MSB-first into bytes (bit t is bit
 *     7 - t%8 of byte t/8), in DEVICE memory owned by the caller, 16-byte
 *     aligned and padded to a multiple of 16 bytes (at least
 *     ceil(nbits/128)*16 bytes): the kernels move whole 16-byte blocks.
 *   - The method (EMR or LMR) and the image size are public: the data hider
 *     and the recipient pass them to every call along with the meta record.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Calls are
 *     stream-ordered and return before the GPU work finishes, except where a
 *     function says it synchronises (the LMR entry points, which run a host
 *     stage).
 *   - Return value: RDHEI_OK (0) or a negative RDHEI_E* code.  Argument
 *     errors are reported before anything is launched.  Conditions only the
 *     device can see (message longer than the capacity computed on the
 *     device) are written to meta->status and the affected image is left
 *     unmodified by that stage.
 *   - A context owns device workspace; two calls that use one context must be
 *     ordered on one stream (use one context per concurrent stream).  The
 *     library never frees caller memory.
 *
 * Keystream (Sec. III-A, secret key generation, asks for a cryptographically
 * secure stream cipher); one of two counter-based families, chosen per context
 * with RDHEI_OPT_KEYSTREAM.  A stream is named by (key, nonce, domain): domain
 * 1 = image keystream s (K1), domain 2 = message keystream (K2); the nonce is
 * a per-image 64-bit value the content owner passes to encryption, recorded
 * in the meta record and used by every role of that image for both streams,
 * so that images encrypted under one key never share a keystream or a
 * rotation (use a distinct nonce per image and key).  Streams stay below 2^36
 * bytes (images of at most 2^31 pixels).
 *   - RDHEI_KEYSTREAM_PHILOX (default): byte idx is little-endian byte idx%16
 *     of Philox4x32-10 (Salmon et al., SC'11) with counter (idx/16, nonce high
 *     word, domain, nonce low word) and key (key low word, key high word).
 *   - RDHEI_KEYSTREAM_CHACHA20: byte idx is byte idx%64 of the ChaCha20 block
 *     (Bernstein 2008; the 32-bit-counter, 96-bit-nonce layout of RFC 8439)
 *     with the 256-bit key (key as 8 little-endian bytes, then 24 zero
 *     bytes), block counter idx/64 and nonce words (domain, nonce low word,
 *     nonce high word): exactly the RFC 8439 keystream for that key and nonce
 *     from counter 0.
 */
#ifndef RDHEI_H
#define RDHEI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RDHEI_OK         0
#define RDHEI_EINVAL    -1   /* bad size, pointer, method or parameter       */
#define RDHEI_ECAPACITY -2   /* message longer than the image's capacity      */
#define RDHEI_ENOFIT    -3   /* LMR: no candidate map compresses into M*N bits */
#define RDHEI_ENOMEM    -4   /* device or host allocation failed              */
#define RDHEI_EDEVICE   -5   /* HIP runtime error (see rdhei_last_error)      */
#define RDHEI_ECORRUPT  -6   /* LMR: map stream in the MSB plane is malformed */

#define RDHEI_EMR 0          /* Sec. III-A: map in the LSB plane, b in [2,7]   */
#define RDHEI_LMR 1          /* Sec. III-B: maps compressed into the MSB plane */
#define RDHEI_DEMR 2         /* dynamic b (Sec. V, future work): EMR with one b
                                per 64x64 tile; batch entry points only, sides
                                multiples of 64, see rdhei_job.btab           */

/* Public side information of one encrypted image (64 bytes, plain data).
 * The paper carries b and the message length implicitly; this record makes
 * them explicit.  Written by rdhei_encrypt (on the device), read by the other
 * three entry points (on the device). */
typedef struct rdhei_meta {
    int32_t height;          /* M                                              */
    int32_t width;           /* N                                              */
    int32_t method;          /* RDHEI_EMR or RDHEI_LMR                         */
    int32_t b;               /* MSBs compared per pixel (EMR 2..7, LMR 2..8;
                                DEMR: 0, the b of each tile is in its table) */
    int32_t min_level;       /* rotation block sizes 2^min_level..2^max_level  */
    int32_t max_level;
    int64_t redundant;       /* Z_b: pixels labelled 0 (redundant)             */
    int64_t capacity_bits;   /* b*Z_b (EMR), (b-1)*Z_b (LMR), sum over tiles of
                                b_t*Z_{b_t}(t) (DEMR)                          */
    int64_t map_bits;        /* LMR: bits of the map stream in the MSB plane   */
    int32_t status;          /* RDHEI_OK or the device-side error of a stage   */
    int32_t reserved;
    uint64_t nonce;          /* keystream nonce given to rdhei_encrypt          */
} rdhei_meta;

typedef struct rdhei_ctx rdhei_ctx;
typedef struct rdhei_plan rdhei_plan;

/* Context on HIP device `device` (workspace arena, kernels' tile choice). */
int  rdhei_ctx_create(rdhei_ctx **out, int device);
void rdhei_ctx_destroy(rdhei_ctx *ctx);

/* Content owner (Sec. III-A encoding phase; Sec. III-B encoding phase).
 * Reads d_img (M x N), writes the encrypted image d_enc (M x N; must not
 * alias d_img) and *d_meta (device memory), which records `nonce`: the
 * per-image keystream nonce of K1's image stream and K2's message stream.
 * EMR: location map for the b in [2,7] maximising b*Z_b (optimal-b equation),
 * rotation of image and map by key-driven block turns at block sizes
 * 2^1..2^n (rotation equation), XOR with s (encryption equation), map into
 * the LSB plane.  Asynchronous.
 * LMR: b in [2,8], rotation at 2^4..2^n, first-MSB map, both maps compressed
 * on the host and written into the MSB plane (candidates tried in order of
 * (b-1)*Z_b; RDHEI_ENOFIT when none fits).  Synchronises `stream`. */
int rdhei_encrypt(rdhei_ctx *ctx, const uint8_t *d_img, uint8_t *d_enc, int32_t M, int32_t N,
                  uint64_t k1, uint64_t nonce, int32_t method, rdhei_meta *d_meta, void *stream);

/* Data hider (Sec. III-A / III-B data hiding phase).  d_marked holds I_e on
 * entry and I_e' on return (in place).  The first nbits bits of d_msg are
 * XORed with K2's keystream and written, in raster order, into the
 * replaceable bits of the redundant pixels (EMR: bits 7..8-b of pixels with
 * LSB 0; LMR: bits 6..8-b of pixels the decompressed map marks 0).  nbits < 0
 * means "the full capacity".  Unused replaceable bits are left unchanged.
 * d_msg is read in whole 16-byte blocks: it must hold ceil(n/128)*16 bytes,
 * n = nbits (the capacity when nbits < 0).
 * A message longer than the capacity sets d_meta->status = RDHEI_ECAPACITY
 * and leaves the image unchanged.
 * EMR: asynchronous; LMR: synchronises (host map decompression). */
int rdhei_embed(rdhei_ctx *ctx, uint8_t *d_marked, int32_t M, int32_t N, int32_t method,
                rdhei_meta *d_meta, const uint8_t *d_msg, int64_t nbits, uint64_t k2, void *stream);

/* Recipient with K2 (Sec. III-A/B decoding with K2).  Writes the first nbits
 * message bits to d_msg (nbits < 0: the capacity), zero-filled to a whole
 * number of 32-bit words; d_msg must hold ceil(nbits/128)*16 bytes. */
int rdhei_extract(rdhei_ctx *ctx, const uint8_t *d_marked, int32_t M, int32_t N, int32_t method,
                  rdhei_meta *d_meta, uint8_t *d_msg, int64_t nbits, uint64_t k2, void *stream);

/* Recipient with K1 (Sec. III-A/B decoding with K1).  Writes the recovered
 * image to d_img (M x N; must not alias d_marked).  EMR output differs from
 * the original only in bit 0 (expected PSNR about 51.14 dB); LMR output is
 * exact.  EMR: asynchronous; LMR: synchronises. */
int rdhei_recover(rdhei_ctx *ctx, const uint8_t *d_marked, int32_t M, int32_t N, int32_t method,
                  rdhei_meta *d_meta, uint8_t *d_img, uint64_t k1, void *stream);

/* ---- Batches: many independent images per launch ------------------------ */

#define RDHEI_OP_ENCRYPT 0
#define RDHEI_OP_EMBED   1
#define RDHEI_OP_EXTRACT 2
#define RDHEI_OP_RECOVER 3

/* One image of a batch.  All pointers are device memory; sizes may differ
 * between images.  in/out/msg follow the single-image call of the op:
 * ENCRYPT: in = I, out = I_e;  EMBED: out = I_e (modified in place), msg in;
 * EXTRACT: in = I_e', msg out;  RECOVER: in = I_e', out = I'.
 * nonce: ENCRYPT only, the image's keystream nonce (recorded in its meta;
 * the other ops read it from there).
 * btab: RDHEI_DEMR only (NULL otherwise), device memory of (height/64) *
 * (width/64) bytes: the b of every 64x64 tile in encrypted-tile order
 * (row-major over the encrypted image), public side information like the
 * meta.  ENCRYPT writes it; EMBED, EXTRACT and RECOVER read it.  Dynamic b
 * (the conclusion's suggestion; this library's reading): a pixel (i, j),
 * j >= 1, is redundant when its b_t most significant bits equal those of its
 * left neighbour, t its tile (the location-map rule of Sec. III-A carried over
 * tile borders); b_t in [2,7] is the first b reaching the largest b * Z_b(t)
 * over the tile's own counts; data hiding replaces the top b_t bits of the
 * tile's redundant pixels; recovery copies, left to right, the top b_t bits of
 * the restored left neighbour into each pixel labelled 0. */
typedef struct rdhei_job {
    const uint8_t *in;
    uint8_t *out;
    uint8_t *msg;
    rdhei_meta *meta;
    uint64_t key;
    uint64_t nonce;
    int64_t nbits;           /* EMBED/EXTRACT: bits, or < 0 for the capacity   */
    int32_t height, width;
    int32_t method;          /* plans and direct batches: RDHEI_EMR, RDHEI_DEMR */
    int32_t reserved;
    uint8_t *btab;           /* RDHEI_DEMR: the tile b table (see above)        */
} rdhei_job;

/* Plan flags. */
#define RDHEI_PLAN_GRAPH     0   /* batched launches, captured once in a hipGraph */
#define RDHEI_PLAN_EAGER     1   /* batched launches issued directly             */
#define RDHEI_PLAN_PER_IMAGE 2   /* the same kernels launched image by image      */

/* Build a reusable plan for one EMR op over `njobs` images (host array,
 * copied).  The plan owns its device job table and workspace.  A GRAPH plan
 * captures its launches on the first run and replays them afterwards; the
 * job pointers are fixed at creation.  Plans are independent of each other
 * and of their context's single-image workspace. */
int  rdhei_plan_create(rdhei_ctx *ctx, int32_t op, const rdhei_job *jobs, int32_t njobs, int32_t flags,
                       rdhei_plan **out);
int  rdhei_plan_run(rdhei_plan *plan, void *stream);
void rdhei_plan_destroy(rdhei_plan *plan);
/* Workgroup cap of the plan's grid-stride launches (0 = one workgroup per
 * work unit), e.g. as chosen by the autotuner. */
int  rdhei_plan_set_grid(rdhei_plan *plan, int32_t max_workgroups);

/* A plan's batched sequence is a list of stages (kernels or kernel groups in
 * the paper's phase order).  These run or name one stage on its own, for
 * profiling; a stage reads what the earlier stages of a full run left in the
 * plan's workspace. */
int         rdhei_plan_stage_count(rdhei_plan *plan);
const char *rdhei_plan_stage_name(rdhei_plan *plan, int32_t k);
int         rdhei_plan_run_stage(rdhei_plan *plan, int32_t k, void *stream);

/* Launch-shape autotuner.  For each layout variant of the plan -- the hiding
 * mode of EMBED/EXTRACT plans (one wave per image where the batch allows it,
 * 4096-pixel steps in one pass, counted 4096-pixel steps), for ENCRYPT and
 * RECOVER plans by stages or one workgroup per image (where the batch allows
 * it) and, by stages, the quads per work unit (2, 4, 8, 16) -- it times every
 * stage at several
 * workgroup counts (the launcher's default -- what fits on the device at once
 * -- and 1, 2, 4, 8, 16 and 32 workgroups per compute unit), max(reps, 5)
 * timed runs each after a warm-up.  A candidate replaces the current choice
 * only when its median run is shorter by more than half the two spreads
 * (max - min of the runs) together, and by 2 % at least; variants compete the
 * same way on the sum of their stages' medians, the plan's own variant first.
 * Choices are cached in the context by device (architecture and compute
 * units), op, keystream family and size class (log2 of the plan's pixels and
 * images), written to the context's tune file if it has one
 * (rdhei_ctx_set_tune_file), and reused by later plans of the same key unless
 * RDHEI_TUNE_FORCE is set.  Tuning reruns the stages on the plan's own
 * buffers (every stage is idempotent), may lay the plan out again (same
 * results, other work units), and leaves the buffers as one run of the plan
 * does; it synchronises `stream`.  PER_IMAGE plans are left as they are.
 * rdhei_plan_set_grid clears the tuned counts. */
#define RDHEI_TUNE_FORCE 1
int rdhei_plan_autotune(rdhei_plan *plan, int32_t reps, int32_t flags, void *stream);
/* The plan's layout variant: hiding mode (RDHEI_OPT_HIDE_MODE values), quads
 * per work unit and workgroup-per-image mode (RDHEI_OPT_WG_PER_IMAGE values);
 * any pointer may be NULL. */
int rdhei_plan_tuned(rdhei_plan *plan, int32_t *hide_mode, int32_t *qseg, int32_t *wg_image);
/* Persist the autotuner's choices: entries of the JSON file at `path` (if it
 * exists) are loaded into the context now, and the file is rewritten after
 * every autotune.  NULL or "" keeps choices in memory only.  RDHEI_EINVAL for
 * a malformed file. */
int rdhei_ctx_set_tune_file(rdhei_ctx *ctx, const char *path);
/* Workgroup count stage k runs with (0: the launcher's default), or < 0 on error. */
int rdhei_plan_stage_grid(rdhei_plan *plan, int32_t k);

/* One EMR op over a batch of images, launched directly on `stream` (no plan,
 * no graph): for batches whose composition changes from call to call, such
 * as a serving loop.
 *   d_workspace  device scratch of at least rdhei_workspace_size() bytes,
 *                256-byte aligned, owned by the caller and in use until the
 *                launches on `stream` finish; NULL: the context's own
 *                workspace, grown when needed (growing synchronises the
 *                device; RDHEI_OPT_RESERVE_WS sizes it up front).
 * The job table goes up through a ring of 16 pinned staging buffers, so the
 * call blocks only when it runs more than 16 calls ahead of the GPU.  Calls
 * on one context must use one stream. */
int rdhei_workspace_size(rdhei_ctx *ctx, int32_t op, const rdhei_job *jobs, int32_t njobs, int64_t *bytes);
int rdhei_run_batch(rdhei_ctx *ctx, int32_t op, const rdhei_job *jobs, int32_t njobs, void *d_workspace,
                    int64_t workspace_bytes, void *stream);

/* Several EMR ops of one batch in order on `stream` (for example encrypt then
 * embed of a server's new requests, extract and recover of its returning
 * ones), all sharing one workspace: what rdhei_run_batch does for each op in
 * turn, with one table upload and one call for all of them.  ops[i] runs over
 * jobs[i][0 .. njobs[i]-1]; 1 <= n_ops <= 8; an op reads what the ops before
 * it in the list wrote, in stream order.  rdhei_roles_workspace_size gives the
 * workspace bytes (the largest of the ops'); d_workspace as for
 * rdhei_run_batch (NULL: the context's own).  Errors as rdhei_run_batch, with
 * nothing launched when any op's table is invalid. */
int rdhei_roles_workspace_size(rdhei_ctx *ctx, int32_t n_ops, const int32_t *ops, const rdhei_job *const *jobs,
                               const int32_t *njobs, int64_t *bytes);
int rdhei_run_roles(rdhei_ctx *ctx, int32_t n_ops, const int32_t *ops, const rdhei_job *const *jobs,
                    const int32_t *njobs, void *d_workspace, int64_t workspace_bytes, void *stream);

/* rdhei_run_batch without allocation, for callers that cannot allocate device
 * memory (code under stream capture, tight serving loops, hosts that forbid
 * hipMalloc): the job tables and the workspace live in a static device array
 * of 64 MiB that the library holds on every GPU it runs on until the process
 * ends; no hipMalloc, hipFree or pinned host allocation is made.  Same ops,
 * jobs and results as rdhei_run_batch (EMR only).  A batch whose tables and
 * workspace exceed 64 MiB is rejected with RDHEI_ENOMEM before anything is
 * launched (rdhei_last_error gives the bytes it needs); for scale, one
 * 512 x 512 encryption takes about 23 KB, a 16384 x 16384 image about 26 MB.
 * Every call on a GPU shares that GPU's array: calls whose launches overlap on
 * one GPU (different streams, or different contexts on one device) race and
 * must be ordered by the caller; calls on one stream are ordered.  The array
 * keeps the last call's contents; each call initialises what it reads. */
int rdhei_run_batch_static(rdhei_ctx *ctx, int32_t op, const rdhei_job *jobs, int32_t njobs, void *stream);

/* Context options. */
#define RDHEI_OPT_PER_PIXEL  1   /* 1: force the per-pixel path for every shape  */
#define RDHEI_OPT_MAX_GRID   2   /* workgroup cap of grid-stride launches         */
#define RDHEI_OPT_RESERVE_WS 3   /* allocate this many workspace bytes now        */
#define RDHEI_OPT_HIDE_MODE  4   /* embed/extract: 0 one wave walks each image
                                    of up to 1 Mpx once a batch holds enough of
                                    them to fill the device, other images go by
                                    4096-pixel steps, counted, scanned, then
                                    hidden (three passes); 1 one wave per image
                                    wherever allowed; 2 always counted steps;
                                    3 steps in one pass, each taking its rank
                                    from a look-back over the steps before it
                                    (pays where images have few steps; slow for
                                    large ones).  Results are identical.         */
#define RDHEI_OPT_LMR_MIN_LEVEL 5 /* LMR rotation blocks 2^v..2^n, v in 1..4
                                    (default 4, the method's; Table
                                    LMR_block_size compares 1..4).  Every role
                                    of an image must use the same value; it is
                                    recorded in meta.min_level.                  */
#define RDHEI_OPT_KEYSTREAM 6    /* keystream family of every role on the
                                    context: RDHEI_KEYSTREAM_PHILOX (default)
                                    or RDHEI_KEYSTREAM_CHACHA20.  Like the
                                    keys, the parties of an image must agree
                                    on it; it is not recorded in the meta.
                                    Calls made after it is set use it; a plan
                                    keeps the family it was created with.      */
#define RDHEI_OPT_QUAD_SEG  7    /* encryption and EMR recovery: 2x2 tile quads
                                    per work unit along a band pair (1..64,
                                    default 4); results are identical        */
#define RDHEI_OPT_WG_PER_IMAGE 8 /* EMR and DEMR encryption and recovery of
                                    batches whose images are all tiled (sides
                                    multiples of 64) with at most 1024 tiles
                                    each: 0 one workgroup per image once the
                                    batch has four images per compute unit,
                                    else by stages; 1 by stages (every tile's
                                    label statistics or keystream codes, then
                                    per-image finalisation, then the
                                    permuting pass, each launch spread over
                                    all tiles); 2 one workgroup per image does
                                    all of an image in one launch (encryption
                                    reads the image the second time soon
                                    after the first; the vector-bound code
                                    work of some images overlaps the memory-
                                    bound pass of others).  Other batches go
                                    by stages.  Results are identical.       */
#define RDHEI_KEYSTREAM_PHILOX   0
#define RDHEI_KEYSTREAM_CHACHA20 1
int rdhei_ctx_set_option(rdhei_ctx *ctx, int32_t option, int64_t value);

/* ---- LMR over a batch of images (Sec. III-B) ---------------------------------
 * One call per role, every device stage batched over the images and the map
 * coder run on `threads` host threads (0: all hardware threads).
 *   RDHEI_OP_ENCRYPT  jobs {in = I, out = I_e, meta, key = K1}: statistics, then
 *                     for each image the candidate b in order of (b-1)*Z_b whose
 *                     compressed rotated maps fit the MSB plane, then the
 *                     encryption carrying that stream in bit 7.  An image that
 *                     fits no candidate gets meta.status RDHEI_ENOFIT and its
 *                     output is not written; the call still returns RDHEI_OK.
 *   RDHEI_OP_EMBED / RDHEI_OP_EXTRACT / RDHEI_OP_RECOVER: jobs as for the EMR
 *                     batch ops; the maps are read back from each marked image's
 *                     MSB plane and decoded on the host first.  Images whose
 *                     meta is not usable are skipped; a stream that does not
 *                     decode sets meta.status RDHEI_ECORRUPT.
 * times (optional, 3 doubles): seconds spent in device stages and copies, in
 * the host coder, and in the whole call.  Synchronises `stream`. */
int rdhei_lmr_batch(rdhei_ctx *ctx, int32_t op, const rdhei_job *jobs, int32_t njobs, int32_t threads,
                    double *times, void *stream);

/* ---- LMR host stage: bi-level map coder (Sec. III-B, map compression) ---- */
/* The paper compresses the rotated first-MSB map and the rotated location map
 * with JBIG-KIT.  This library uses its own context-modelled binary
 * arithmetic coder.  Inputs are host bit planes (M*N bits, MSB-first packed,
 * raster order).  The stream is: 32-bit big-endian byte length of the eta
 * part, 32-bit big-endian byte length of the l part, eta part, l part.
 * rdhei_lmr_compress writes at most `capacity_bytes` bytes and returns
 * RDHEI_ENOFIT if the stream would be longer; *stream_bits receives its length
 * in bits.  rdhei_lmr_decompress returns RDHEI_ECORRUPT on a malformed stream. */
int rdhei_lmr_compress(const uint8_t *eta_bits, const uint8_t *l_bits, int32_t M, int32_t N,
                       uint8_t *stream, int64_t capacity_bytes, int64_t *stream_bits);
int rdhei_lmr_decompress(const uint8_t *stream, int64_t stream_bytes, int32_t M, int32_t N,
                         uint8_t *eta_bits, uint8_t *l_bits);

/* ---- Image metrics (Sec. IV: Table EMR_results and the security analysis) ----
 * Per pair of 8-bit images (a, b), eight doubles written to d_out[8*i + k]:
 *   k = 0, 1  Shannon entropy (bits) and chi-square test of a (Sec. IV-B
 *             equations: chi2 = 256 * M * N * sum_v (P_v - 1/256)^2);
 *   k = 2, 3  the same for b;
 *   k = 4     NPCR: percentage of positions where a and b differ (Sec. IV-B;
 *             the printed indicator is inverted, the metric counts changes);
 *   k = 5     UACI: mean |a - b| as a percentage of 255 (Sec. IV-B);
 *   k = 6     PSNR = 10 log10(255^2 / MSE) dB, +inf for identical images;
 *   k = 7     SSIM: mean over every 7x7 window inside the image of the
 *             structural similarity with sample (co)variances, K1 = 0.01,
 *             K2 = 0.03, L = 255 (the paper names no variant), computed only
 *             with RDHEI_METRIC_SSIM.
 * Values 2..7 are NaN when b is NULL; SSIM is NaN without the flag or when
 * an image side is below 7.  a, b: device images, row-major height x width,
 * caller-owned, read only (16-byte aligned images take vector loads).  d_out:
 * device memory of 8 * njobs doubles, caller-owned.  The job array is host
 * memory, copied.  Asynchronous on `stream`; errors: RDHEI_EINVAL for a
 * NULL a or d_out, sizes below 1 or unknown flags. */
typedef struct {
    const uint8_t *a;
    const uint8_t *b;
    int32_t height, width;
} rdhei_metric_job;
#define RDHEI_METRIC_COUNT 8
#define RDHEI_METRIC_SSIM  1
int rdhei_metrics(rdhei_ctx *ctx, const rdhei_metric_job *jobs, int32_t njobs, int32_t flags, double *d_out,
                  void *stream);

/* ---- Per-tile b (the conclusion's dynamic b) -----------------------------------
 * The conclusion suggests a b that varies over the image.  This call computes
 * the choice of this library's dynamic-b reading, one b per 64x64 tile,
 * without encrypting: for tile t of an image, Z_b(t) = pixels of the tile,
 * image column 0 excepted, whose b most significant bits equal those of their
 * left neighbour (for a tile's first column the neighbour lies in the tile to
 * its left: the location-map rule of Sec. III-A carried over tile borders),
 * b = 2..7; b_t = the first b reaching the largest b * Z_b(t), as the global b
 * is chosen; the image's capacity = sum over tiles of b_t * Z_{b_t}(t) bits.
 *   jobs        image in .a (.b unused), height and width positive multiples of
 *               64, .a 16-byte aligned
 *   d_tile_b    device, one byte per tile of every image: images in job order,
 *               tiles row-major
 *   d_capacity  device, one int64 per image
 * Asynchronous on `stream`.  Errors (nothing launched): RDHEI_EINVAL for NULL
 * pointers, njobs < 1, a side that is not a positive multiple of 64, an
 * unaligned image or more than 2^31 tiles. */
int rdhei_tile_b(rdhei_ctx *ctx, const rdhei_metric_job *jobs, int32_t njobs, uint8_t *d_tile_b, int64_t *d_capacity,
                 void *stream);

/* ---- Diagnostics ---------------------------------------------------------- */
const char *rdhei_strerror(int code);
/* Text of the last HIP error seen by this thread (empty if none). */
const char *rdhei_last_error(void);
/* Library version string. */
const char *rdhei_version(void);

#ifdef __cplusplus
}
#endif
#endif /* RDHEI_H */

/*
 * Plain, single-threaded CPU oracle for EMR-RDHEI and LMR-RDHEI
 * (Zhang & Luo, "Vector-based Efficient Data Hiding in Encrypted Images via
 * Multi-MSB Replacement", arXiv 2302.07992).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or constant generator
 * with the HIP path.  It runs every step the way the paper states it:
 * the Omega glide once per candidate b, the block rotation level by level with
 * the whole image materialised after each level, embedding with a running bit
 * counter, and the omega glide for recovery.  No closed forms, no blocking.
 *
 * Conventions the paper leaves open are fixed as follows (each is a reading of
 * a silent or ambiguous passage; the product follows the same readings):
 *   - keystream: Philox4x32-10 (Salmon et al., SC'11); byte idx of the stream
 *     (key, nonce, domain) is little-endian byte (idx & 15) of the block with
 *     counter (idx>>4, nonce high word, domain, nonce low word) and key
 *     (K low, K high), for idx < 2^36.  Domain 1 = image keystream s (key K1),
 *     domain 2 = message keystream (key K2); the nonce is a per-image value
 *     the content owner picks and the side information carries, so that two
 *     images under one key never share a stream.  The paper asks only for a
 *     secure stream cipher (Sec. III-A, "Secret key generation").  The second
 *     family, selected with or_set_keystream(1), is ChaCha20: byte idx is byte
 *     idx%64 of the ChaCha20 block (IETF layout) with key (K as 8
 *     little-endian bytes, 24 zero bytes), counter idx/64 and nonce words
 *     (domain, nonce low word, nonce high word), for idx < 2^38.
 *   - a pixel is redundant (label 0) when its b MSBs equal those of the
 *     tracker (the text of Sec. III-A wins over the indicator printed in the
 *     gliding equation).
 *   - optimal b: the first b reaching the largest b*Z_b (ties -> smaller b).
 *   - n = floor(log2(min(M, N))); only full 2^m x 2^m blocks are rotated.
 *   - a rotation code r turns the block r quarter turns counter-clockwise
 *     (out[a][c] = in[c][k-1-a] per turn); decoding turns (4-r) mod 4.
 *   - payload bits fill pixels in raster order of the encrypted image, the
 *     most significant replaceable bit first; message bytes are read
 *     MSB-first; the message is XORed with the K2 stream bit by bit.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Keystream (Sec. III-A "Secret key generation"): Philox4x32-10.            */
/* ------------------------------------------------------------------------ */

void or_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* ChaCha20 block function (Bernstein 2008; IETF layout: state words 0-3 the
 * constant "expand 32-byte k", 4-11 the key, 12 the block counter, 13-15 the
 * nonce).  Twenty rounds, alternately on the columns and the diagonals of the
 * 4x4 state, then the input state added word by word; the 64 output bytes
 * are the 16 words little-endian. */
static uint32_t or_rotl32(uint32_t v, int n) { return (v << n) | (v >> (32 - n)); }

static void or_quarter_round(uint32_t *x, int a, int b, int c, int d)
{
    x[a] += x[b]; x[d] ^= x[a]; x[d] = or_rotl32(x[d], 16);
    x[c] += x[d]; x[b] ^= x[c]; x[b] = or_rotl32(x[b], 12);
    x[a] += x[b]; x[d] ^= x[a]; x[d] = or_rotl32(x[d], 8);
    x[c] += x[d]; x[b] ^= x[c]; x[b] = or_rotl32(x[b], 7);
}

void or_chacha20_block(const uint32_t key[8], uint32_t counter, const uint32_t nonce[3], uint8_t out[64])
{
    uint32_t in[16], x[16];
    in[0] = 0x61707865u; in[1] = 0x3320646eu; in[2] = 0x79622d32u; in[3] = 0x6b206574u;
    for (int i = 0; i < 8; ++i) in[4 + i] = key[i];
    in[12] = counter;
    in[13] = nonce[0]; in[14] = nonce[1]; in[15] = nonce[2];
    memcpy(x, in, sizeof x);
    for (int round = 0; round < 20; round += 2) {
        or_quarter_round(x, 0, 4, 8, 12);     /* columns */
        or_quarter_round(x, 1, 5, 9, 13);
        or_quarter_round(x, 2, 6, 10, 14);
        or_quarter_round(x, 3, 7, 11, 15);
        or_quarter_round(x, 0, 5, 10, 15);    /* diagonals */
        or_quarter_round(x, 1, 6, 11, 12);
        or_quarter_round(x, 2, 7, 8, 13);
        or_quarter_round(x, 3, 4, 9, 14);
    }
    for (int i = 0; i < 16; ++i) {
        uint32_t v = x[i] + in[i];
        for (int k = 0; k < 4; ++k) out[4 * i + k] = (uint8_t)(v >> (8 * k));
    }
}

/* Keystream family of every later or_keystream call: 0 Philox4x32-10, 1
 * ChaCha20 (see the header note). */
static int or_family = 0;

void or_set_keystream(int family) { or_family = family; }

/* Bytes [first, first+count) of the stream (key, nonce, domain).  Streams are
 * at most 2^36 bytes long (Philox's block index fills one counter word). */
void or_keystream(uint64_t key, uint64_t nonce, uint32_t domain, uint64_t first, uint64_t count, uint8_t *out)
{
    if (first + count > ((uint64_t)1 << 36)) abort();
    uint32_t k[2] = {(uint32_t)key, (uint32_t)(key >> 32)};
    if (or_family == 1) {
        uint32_t ck[8] = {k[0], k[1], 0u, 0u, 0u, 0u, 0u, 0u};
        uint8_t block[64];
        uint64_t have = ~(uint64_t)0;      /* index of the block in `block` */
        for (uint64_t t = 0; t < count; ++t) {
            uint64_t idx = first + t;
            uint64_t c = idx >> 6;
            if (c != have) {
                uint32_t nw[3] = {domain, (uint32_t)nonce, (uint32_t)(nonce >> 32)};
                or_chacha20_block(ck, (uint32_t)c, nw, block);
                have = c;
            }
            out[t] = block[idx & 63];
        }
        return;
    }
    for (uint64_t t = 0; t < count; ++t) {
        uint64_t idx = first + t;
        uint64_t blk = idx >> 4;
        uint32_t ctr[4] = {(uint32_t)blk, (uint32_t)(nonce >> 32), domain, (uint32_t)nonce};
        uint32_t w[4];
        or_philox4x32_10(ctr, k, w);
        unsigned within = (unsigned)(idx & 15);
        out[t] = (uint8_t)(w[within >> 2] >> (8 * (within & 3)));
    }
}

/* ------------------------------------------------------------------------ */
/* Location maps (Sec. III-A "Optimal location map generation", Eqs. for the */
/* initialisation, the glide and the map update).                            */
/* ------------------------------------------------------------------------ */

/* Location map for one b by gliding the tracker omega along each row.
 * L[i][0] = 1; for j >= 1 the pixel is redundant (0) when its b MSBs match
 * the tracker; the tracker takes the pixel whenever the pixel is
 * non-redundant.  Returns Z_b, the number of zeros. */
int64_t or_location_map(const uint8_t *I, int32_t M, int32_t N, int b, uint8_t *L)
{
    int64_t zeros = 0;
    int shift = 8 - b;
    for (int32_t i = 0; i < M; ++i) {
        uint8_t omega = I[(int64_t)i * N];
        L[(int64_t)i * N] = 1;
        for (int32_t j = 1; j < N; ++j) {
            uint8_t phi = I[(int64_t)i * N + j];
            if ((phi >> shift) == (omega >> shift)) {
                L[(int64_t)i * N + j] = 0;
                ++zeros;
            } else {
                L[(int64_t)i * N + j] = 1;
                omega = phi;
            }
        }
    }
    return zeros;
}

/* Z_b for b = bmin..bmax (Z[b - bmin]), each from its own glide. */
void or_redundancy_counts(const uint8_t *I, int32_t M, int32_t N, int bmin, int bmax, int64_t *Z)
{
    uint8_t *L = (uint8_t *)malloc((size_t)M * (size_t)N + 1);
    for (int b = bmin; b <= bmax; ++b)
        Z[b - bmin] = or_location_map(I, M, N, b, L);
    free(L);
}

/* Eq. for the optimal b: the b maximising b * Z_b / (M N), first on ties. */
int or_select_b(const int64_t *Z, int bmin, int bmax)
{
    int best = bmin;
    for (int b = bmin + 1; b <= bmax; ++b)
        if ((int64_t)b * Z[b - bmin] > (int64_t)best * Z[best - bmin])
            best = b;
    return best;
}

/* ------------------------------------------------------------------------ */
/* Block rotation (Sec. III-A "Rotation and image encryption", rotation       */
/* equation; decoding: Sec. III-A decoding with K1, de-rotation equation).   */
/* ------------------------------------------------------------------------ */

int or_max_level(int32_t M, int32_t N)
{
    int32_t m = M < N ? M : N;
    int n = 0;
    while (((int64_t)2 << n) <= m) ++n;   /* largest n with 2^n <= min(M,N) */
    return n;
}

/* Rotation code of the full block (C1, C2) of side 2^m: (sum of s) mod 4. */
static int block_code(const uint8_t *s, int32_t N, int m, int32_t C1, int32_t C2)
{
    int32_t k = (int32_t)1 << m;
    uint64_t sum = 0;
    for (int32_t a = 0; a < k; ++a)
        for (int32_t c = 0; c < k; ++c)
            sum += s[((int64_t)C1 * k + a) * N + (int64_t)C2 * k + c];
    return (int)(sum % 4);
}

/* One level: every full 2^m block of X (M x N) turned `turns(code)` quarter
 * turns counter-clockwise, written into a fresh copy of the image. */
static void rotate_level(uint8_t *X, int32_t M, int32_t N, const uint8_t *s, int m, int inverse)
{
    int32_t k = (int32_t)1 << m;
    size_t bytes = (size_t)M * (size_t)N;
    uint8_t *next = (uint8_t *)malloc(bytes + 1);
    uint8_t *blk = (uint8_t *)malloc((size_t)k * (size_t)k);
    uint8_t *tmp = (uint8_t *)malloc((size_t)k * (size_t)k);
    memcpy(next, X, bytes);
    for (int32_t C1 = 0; C1 < M / k; ++C1) {
        for (int32_t C2 = 0; C2 < N / k; ++C2) {
            int r = block_code(s, N, m, C1, C2);
            int turns = inverse ? (4 - r) % 4 : r;
            for (int32_t a = 0; a < k; ++a)
                for (int32_t c = 0; c < k; ++c)
                    blk[a * k + c] = X[((int64_t)C1 * k + a) * N + (int64_t)C2 * k + c];
            for (int t = 0; t < turns; ++t) {
                for (int32_t a = 0; a < k; ++a)
                    for (int32_t c = 0; c < k; ++c)
                        tmp[a * k + c] = blk[c * k + (k - 1 - a)];
                memcpy(blk, tmp, (size_t)k * (size_t)k);
            }
            for (int32_t a = 0; a < k; ++a)
                for (int32_t c = 0; c < k; ++c)
                    next[((int64_t)C1 * k + a) * N + (int64_t)C2 * k + c] = blk[a * k + c];
        }
    }
    memcpy(X, next, bytes);
    free(next); free(blk); free(tmp);
}

/* Encoding: levels min_level..n ascending.  Decoding: n..min_level with the
 * opposite turn. */
void or_rotate(uint8_t *X, int32_t M, int32_t N, const uint8_t *s, int min_level, int inverse)
{
    int n = or_max_level(M, N);
    if (!inverse) {
        for (int m = min_level; m <= n; ++m) rotate_level(X, M, N, s, m, 0);
    } else {
        for (int m = n; m >= min_level; --m) rotate_level(X, M, N, s, m, 1);
    }
}

/* ------------------------------------------------------------------------ */
/* EMR-RDHEI                                                                 */
/* ------------------------------------------------------------------------ */

typedef struct or_meta {
    int32_t b;
    int32_t min_level;
    int32_t max_level;
    int32_t pad;
    int64_t redundant;
    int64_t capacity_bits;
} or_meta;

/* Encoding phase (Sec. III-A): location map for the optimal b in [2,7],
 * rotation of I and l with K1's keystream, XOR encryption, and the rotated
 * map written into the LSB plane. */
void or_emr_encrypt(const uint8_t *I, int32_t M, int32_t N, uint64_t k1, uint64_t nonce, uint8_t *Ie,
                    or_meta *meta)
{
    size_t MN = (size_t)M * (size_t)N;
    int64_t Z[6];
    or_redundancy_counts(I, M, N, 2, 7, Z);
    int b = or_select_b(Z, 2, 7);
    uint8_t *l = (uint8_t *)malloc(MN + 1);
    or_location_map(I, M, N, b, l);

    uint8_t *s = (uint8_t *)malloc(MN + 1);
    or_keystream(k1, nonce, 1, 0, MN, s);

    uint8_t *Irot = (uint8_t *)malloc(MN + 1);
    memcpy(Irot, I, MN);
    or_rotate(Irot, M, N, s, 1, 0);
    or_rotate(l, M, N, s, 1, 0);

    for (size_t p = 0; p < MN; ++p) {
        uint8_t enc = (uint8_t)(s[p] ^ Irot[p]);
        Ie[p] = (uint8_t)((enc & 0xFE) | (l[p] & 1));
    }
    meta->b = b;
    meta->min_level = 1;
    meta->max_level = or_max_level(M, N);
    meta->redundant = Z[b - 2];
    meta->capacity_bits = (int64_t)b * Z[b - 2];
    free(l); free(s); free(Irot);
}

static int get_bit(const uint8_t *bytes, int64_t t) { return (bytes[t >> 3] >> (7 - (t & 7))) & 1; }
static void put_bit(uint8_t *bytes, int64_t t, int v)
{
    if (v) bytes[t >> 3] |= (uint8_t)(0x80 >> (t & 7));
    else   bytes[t >> 3] &= (uint8_t)~(0x80 >> (t & 7));
}

/* Data hiding (Sec. III-A "Data hiding phase" for EMR, Sec. III-B for LMR):
 * the message is encrypted with K2's stream and written into the replaceable
 * bits (top `nrep` bits below `top`) of every pixel that the rotated location
 * map marks 0, in raster order, using a running bit counter.  `lmap` is the
 * rotated location map (1 byte per pixel).  Returns the number of bits
 * written, or -1 if the message does not fit. */
int64_t or_hide(uint8_t *X, int32_t M, int32_t N, const uint8_t *lmap, int top, int nrep,
                const uint8_t *msg, int64_t nbits, uint64_t k2, uint64_t nonce)
{
    size_t MN = (size_t)M * (size_t)N;
    int64_t cap = 0;
    for (size_t p = 0; p < MN; ++p) cap += (lmap[p] == 0) ? nrep : 0;
    if (nbits > cap) return -1;
    int64_t nbytes = (nbits + 7) / 8;
    uint8_t *ks = (uint8_t *)malloc((size_t)nbytes + 1);
    or_keystream(k2, nonce, 2, 0, (uint64_t)nbytes, ks);
    int64_t t = 0;
    for (size_t p = 0; p < MN && t < nbits; ++p) {
        if (lmap[p] != 0) continue;
        for (int u = 0; u < nrep && t < nbits; ++u, ++t) {
            int bit = get_bit(msg, t) ^ get_bit(ks, t);
            int pos = top - u;
            X[p] = (uint8_t)((X[p] & ~(1u << pos)) | ((unsigned)bit << pos));
        }
    }
    free(ks);
    return t;
}

/* Extraction (Sec. III-A decoding with K2): concatenate the replaceable bits
 * of the pixels marked 0, raster order, and decrypt with K2's stream. */
int64_t or_reveal(const uint8_t *X, int32_t M, int32_t N, const uint8_t *lmap, int top, int nrep,
                  uint8_t *msg, int64_t nbits, uint64_t k2, uint64_t nonce)
{
    size_t MN = (size_t)M * (size_t)N;
    int64_t nbytes = (nbits + 7) / 8;
    uint8_t *ks = (uint8_t *)malloc((size_t)nbytes + 1);
    or_keystream(k2, nonce, 2, 0, (uint64_t)nbytes, ks);
    memset(msg, 0, (size_t)nbytes);
    int64_t t = 0;
    for (size_t p = 0; p < MN && t < nbits; ++p) {
        if (lmap[p] != 0) continue;
        for (int u = 0; u < nrep && t < nbits; ++u, ++t) {
            int bit = (X[p] >> (top - u)) & 1;
            put_bit(msg, t, bit ^ get_bit(ks, t));
        }
    }
    free(ks);
    return t;
}

/* EMR data hiding: the rotated map is the LSB plane of I_e; b MSBs replaced. */
int64_t or_emr_embed(uint8_t *Ie, int32_t M, int32_t N, int b, const uint8_t *msg, int64_t nbits, uint64_t k2,
                     uint64_t nonce)
{
    size_t MN = (size_t)M * (size_t)N;
    uint8_t *l = (uint8_t *)malloc(MN + 1);
    for (size_t p = 0; p < MN; ++p) l[p] = Ie[p] & 1;
    int64_t r = or_hide(Ie, M, N, l, 7, b, msg, nbits, k2, nonce);
    free(l);
    return r;
}

int64_t or_emr_extract(const uint8_t *Ie, int32_t M, int32_t N, int b, uint8_t *msg, int64_t nbits, uint64_t k2,
                       uint64_t nonce)
{
    size_t MN = (size_t)M * (size_t)N;
    uint8_t *l = (uint8_t *)malloc(MN + 1);
    for (size_t p = 0; p < MN; ++p) l[p] = Ie[p] & 1;
    int64_t r = or_reveal(Ie, M, N, l, 7, b, msg, nbits, k2, nonce);
    free(l);
    return r;
}

/* Recovery glide (Sec. III-A decoding with K1, last paragraph): omega starts
 * from column 0 and keeps the replaceable bits of the last pixel marked 1;
 * every pixel marked 0 takes them.  `mask` selects the replaceable bits. */
static void recovery_glide(uint8_t *D, const uint8_t *l, int32_t M, int32_t N, uint8_t mask)
{
    for (int32_t i = 0; i < M; ++i) {
        uint8_t omega = D[(int64_t)i * N] & mask;
        for (int32_t j = 1; j < N; ++j) {
            int64_t p = (int64_t)i * N + j;
            if (l[p] == 1) omega = D[p] & mask;
            else D[p] = (uint8_t)((D[p] & (uint8_t)~mask) | omega);
        }
    }
}

/* EMR image recovery: l from the LSBs, XOR decryption, de-rotation of the
 * decrypted image and the map in descending level order, then the glide. */
void or_emr_recover(const uint8_t *Ie, int32_t M, int32_t N, int b, uint64_t k1, uint64_t nonce, uint8_t *out)
{
    size_t MN = (size_t)M * (size_t)N;
    uint8_t *s = (uint8_t *)malloc(MN + 1);
    uint8_t *l = (uint8_t *)malloc(MN + 1);
    or_keystream(k1, nonce, 1, 0, MN, s);
    for (size_t p = 0; p < MN; ++p) {
        l[p] = Ie[p] & 1;
        out[p] = (uint8_t)(Ie[p] ^ s[p]);
    }
    or_rotate(out, M, N, s, 1, 1);
    or_rotate(l, M, N, s, 1, 1);
    recovery_glide(out, l, M, N, (uint8_t)(0xFF << (8 - b)));
    free(s); free(l);
}

/* ------------------------------------------------------------------------ */
/* Dynamic b (Sec. V, future work).  The paper suggests tracing more         */
/* redundant bits with a b that varies over the image and defines nothing    */
/* further.  Reading: one b per 64 x 64 tile (sides multiples of 64).  A     */
/* pixel (i, j), j >= 1, is redundant when its b_t MSBs equal those of its   */
/* left neighbour (i, j-1), t its tile -- with one b for the whole image that */
/* is exactly the set the Omega glide marks (Sec. III-A), here carried over   */
/* tile borders.  b_t is chosen by the optimal-b rule on the tile's own      */
/* counts.  Everything else is the EMR method: rotation, XOR, the map in the  */
/* LSB plane, data hiding into the top b MSBs of redundant pixels, where b is */
/* that of the pixel's tile.  The b table is side information in encrypted-  */
/* tile order (the data hider has no K1 to follow tiles through the          */
/* rotation).                                                                */
/* ------------------------------------------------------------------------ */

#define OR_TILE 64

/* Z_b(t) for b = 2..7 (Z[6 t + b - 2], tiles row-major) by the left-neighbour
 * rule, and b_t: the first b reaching the largest b * Z_b(t). */
void or_demr_tile_b(const uint8_t *I, int32_t M, int32_t N, uint8_t *tile_b, int64_t *Z)
{
    int32_t tx_n = N / OR_TILE, ty_n = M / OR_TILE;
    for (int32_t ty = 0; ty < ty_n; ++ty) {
        for (int32_t tx = 0; tx < tx_n; ++tx) {
            int64_t *z = Z + 6 * ((int64_t)ty * tx_n + tx);
            for (int b = 2; b <= 7; ++b) {
                int64_t n = 0;
                for (int32_t i = ty * OR_TILE; i < (ty + 1) * OR_TILE; ++i)
                    for (int32_t j = tx * OR_TILE; j < (tx + 1) * OR_TILE; ++j) {
                        if (j == 0) continue;
                        uint8_t v = I[(int64_t)i * N + j], w = I[(int64_t)i * N + j - 1];
                        if ((v >> (8 - b)) == (w >> (8 - b))) ++n;
                    }
                z[b - 2] = n;
            }
            tile_b[(int64_t)ty * tx_n + tx] = (uint8_t)or_select_b(z, 2, 7);
        }
    }
}

/* Per-pixel b from a tile table (tiles row-major). */
static void expand_tile_b(const uint8_t *tile_b, int32_t M, int32_t N, uint8_t *bmap)
{
    int32_t tx_n = N / OR_TILE;
    for (int32_t i = 0; i < M; ++i)
        for (int32_t j = 0; j < N; ++j)
            bmap[(int64_t)i * N + j] = tile_b[(int64_t)(i / OR_TILE) * tx_n + j / OR_TILE];
}

/* Encoding with a b per tile: labels by the rule above, rotation of I, the
 * map and the per-pixel b with K1's keystream, XOR, the map in the LSB plane.
 * btab_enc receives the b table in encrypted-tile order (read from the
 * rotated per-pixel b, which is constant on every encrypted tile because
 * levels above 2^6 move whole tiles); returns -1 if it is not (never for
 * sides that are multiples of 64). */
int or_demr_encrypt(const uint8_t *I, int32_t M, int32_t N, uint64_t k1, uint64_t nonce, uint8_t *Ie,
                    uint8_t *btab_enc, or_meta *meta)
{
    size_t MN = (size_t)M * (size_t)N;
    int32_t tx_n = N / OR_TILE, ty_n = M / OR_TILE;
    size_t T = (size_t)tx_n * (size_t)ty_n;
    uint8_t *tb = (uint8_t *)malloc(T + 1);
    int64_t *Z = (int64_t *)malloc(6 * T * sizeof(int64_t) + 8);
    or_demr_tile_b(I, M, N, tb, Z);
    int64_t red = 0, cap = 0;
    for (size_t t = 0; t < T; ++t) {
        red += Z[6 * t + tb[t] - 2];
        cap += (int64_t)tb[t] * Z[6 * t + tb[t] - 2];
    }
    uint8_t *bmap = (uint8_t *)malloc(MN + 1);
    expand_tile_b(tb, M, N, bmap);
    uint8_t *l = (uint8_t *)malloc(MN + 1);
    for (int32_t i = 0; i < M; ++i)
        for (int32_t j = 0; j < N; ++j) {
            int64_t p = (int64_t)i * N + j;
            int sh = 8 - bmap[p];
            l[p] = (uint8_t)(j == 0 || (I[p] >> sh) != (I[p - 1] >> sh));
        }
    uint8_t *s = (uint8_t *)malloc(MN + 1);
    or_keystream(k1, nonce, 1, 0, MN, s);
    uint8_t *Irot = (uint8_t *)malloc(MN + 1);
    memcpy(Irot, I, MN);
    or_rotate(Irot, M, N, s, 1, 0);
    or_rotate(l, M, N, s, 1, 0);
    or_rotate(bmap, M, N, s, 1, 0);
    for (size_t p = 0; p < MN; ++p) Ie[p] = (uint8_t)(((s[p] ^ Irot[p]) & 0xFE) | (l[p] & 1));
    int rc = 0;
    for (int32_t ty = 0; ty < ty_n; ++ty)
        for (int32_t tx = 0; tx < tx_n; ++tx) {
            uint8_t v = bmap[(int64_t)ty * OR_TILE * N + (int64_t)tx * OR_TILE];
            btab_enc[(int64_t)ty * tx_n + tx] = v;
            for (int32_t i = ty * OR_TILE; i < (ty + 1) * OR_TILE; ++i)
                for (int32_t j = tx * OR_TILE; j < (tx + 1) * OR_TILE; ++j)
                    if (bmap[(int64_t)i * N + j] != v) rc = -1;
        }
    meta->b = 0;
    meta->min_level = 1;
    meta->max_level = or_max_level(M, N);
    meta->redundant = red;
    meta->capacity_bits = cap;
    free(tb); free(Z); free(bmap); free(l); free(s); free(Irot);
    return rc;
}

/* Data hiding / extraction with the b of each pixel's (encrypted) tile: the
 * message, XORed with K2's stream, fills the top b bits of the pixels whose
 * LSB is 0, raster order, most significant first (a running bit counter). */
int64_t or_demr_embed(uint8_t *Ie, int32_t M, int32_t N, const uint8_t *btab_enc, const uint8_t *msg, int64_t nbits,
                      uint64_t k2, uint64_t nonce)
{
    size_t MN = (size_t)M * (size_t)N;
    uint8_t *bmap = (uint8_t *)malloc(MN + 1);
    expand_tile_b(btab_enc, M, N, bmap);
    int64_t cap = 0;
    for (size_t p = 0; p < MN; ++p) cap += (Ie[p] & 1) == 0 ? bmap[p] : 0;
    if (nbits > cap) { free(bmap); return -1; }
    int64_t nbytes = (nbits + 7) / 8;
    uint8_t *ks = (uint8_t *)malloc((size_t)nbytes + 1);
    or_keystream(k2, nonce, 2, 0, (uint64_t)nbytes, ks);
    int64_t t = 0;
    for (size_t p = 0; p < MN && t < nbits; ++p) {
        if ((Ie[p] & 1) != 0) continue;
        for (int u = 0; u < bmap[p] && t < nbits; ++u, ++t) {
            int bit = get_bit(msg, t) ^ get_bit(ks, t);
            Ie[p] = (uint8_t)((Ie[p] & ~(1u << (7 - u))) | ((unsigned)bit << (7 - u)));
        }
    }
    free(ks); free(bmap);
    return t;
}

int64_t or_demr_extract(const uint8_t *Ie, int32_t M, int32_t N, const uint8_t *btab_enc, uint8_t *msg, int64_t nbits,
                        uint64_t k2, uint64_t nonce)
{
    size_t MN = (size_t)M * (size_t)N;
    uint8_t *bmap = (uint8_t *)malloc(MN + 1);
    expand_tile_b(btab_enc, M, N, bmap);
    int64_t nbytes = (nbits + 7) / 8;
    uint8_t *ks = (uint8_t *)malloc((size_t)nbytes + 1);
    or_keystream(k2, nonce, 2, 0, (uint64_t)nbytes, ks);
    memset(msg, 0, (size_t)nbytes);
    int64_t t = 0;
    for (size_t p = 0; p < MN && t < nbits; ++p) {
        if ((Ie[p] & 1) != 0) continue;
        for (int u = 0; u < bmap[p] && t < nbits; ++u, ++t)
            put_bit(msg, t, ((Ie[p] >> (7 - u)) & 1) ^ get_bit(ks, t));
    }
    free(ks); free(bmap);
    return t;
}

/* Recovery with K1: l from the LSBs, XOR decryption, de-rotation of the image,
 * the map and the per-pixel b (spread from the table in the encrypted
 * domain), then left to right along each row: a pixel labelled 0 takes the
 * top b MSBs (b of its tile) of its left neighbour as restored. */
void or_demr_recover(const uint8_t *Ie, int32_t M, int32_t N, const uint8_t *btab_enc, uint64_t k1, uint64_t nonce,
                     uint8_t *out)
{
    size_t MN = (size_t)M * (size_t)N;
    uint8_t *s = (uint8_t *)malloc(MN + 1);
    uint8_t *l = (uint8_t *)malloc(MN + 1);
    uint8_t *bmap = (uint8_t *)malloc(MN + 1);
    or_keystream(k1, nonce, 1, 0, MN, s);
    expand_tile_b(btab_enc, M, N, bmap);
    for (size_t p = 0; p < MN; ++p) {
        l[p] = Ie[p] & 1;
        out[p] = (uint8_t)(Ie[p] ^ s[p]);
    }
    or_rotate(out, M, N, s, 1, 1);
    or_rotate(l, M, N, s, 1, 1);
    or_rotate(bmap, M, N, s, 1, 1);
    for (int32_t i = 0; i < M; ++i)
        for (int32_t j = 1; j < N; ++j) {
            int64_t p = (int64_t)i * N + j;
            if (l[p] != 0) continue;
            uint8_t mask = (uint8_t)(0xFF << (8 - bmap[p]));
            out[p] = (uint8_t)((out[p - 1] & mask) | (out[p] & (uint8_t)~mask));
        }
    free(s); free(l); free(bmap);
}

/* ------------------------------------------------------------------------ */
/* LMR-RDHEI (Sec. III-B).  The map compression is an external step here:    */
/* the caller hands in the compressed stream; this file never compresses.    */
/* ------------------------------------------------------------------------ */

/* Maps for LMR with a given b (b in [2,8]) and min_level: the rotated
 * location map and the rotated first-MSB map eta = (I AND 128) mod 127, one
 * byte per pixel each. */
void or_lmr_rotated_maps(const uint8_t *I, int32_t M, int32_t N, int b, int min_level, uint64_t k1, uint64_t nonce,
                         uint8_t *l_rot, uint8_t *eta_rot)
{
    size_t MN = (size_t)M * (size_t)N;
    uint8_t *s = (uint8_t *)malloc(MN + 1);
    or_keystream(k1, nonce, 1, 0, MN, s);
    or_location_map(I, M, N, b, l_rot);
    for (size_t p = 0; p < MN; ++p) eta_rot[p] = (uint8_t)((I[p] & 128) % 127);
    or_rotate(l_rot, M, N, s, min_level, 0);
    or_rotate(eta_rot, M, N, s, min_level, 0);
    free(s);
}

/* LMR encryption with a given stream for the first-MSB plane: rotate I,
 * XOR with s, then bit 7 of pixel p (raster order) := stream bit p for
 * p < stream_bits. */
void or_lmr_encrypt(const uint8_t *I, int32_t M, int32_t N, int min_level, uint64_t k1, uint64_t nonce,
                    const uint8_t *stream, int64_t stream_bits, uint8_t *Ie)
{
    size_t MN = (size_t)M * (size_t)N;
    uint8_t *s = (uint8_t *)malloc(MN + 1);
    or_keystream(k1, nonce, 1, 0, MN, s);
    memcpy(Ie, I, MN);
    or_rotate(Ie, M, N, s, min_level, 0);
    for (size_t p = 0; p < MN; ++p) Ie[p] = (uint8_t)(Ie[p] ^ s[p]);
    for (int64_t p = 0; p < stream_bits && p < (int64_t)MN; ++p)
        Ie[p] = (uint8_t)((Ie[p] & 0x7F) | (get_bit(stream, p) << 7));
    free(s);
}

/* LMR data hiding / extraction: (b-1) bits at bits 6..8-b of every pixel the
 * (decompressed, rotated) location map marks 0. */
int64_t or_lmr_embed(uint8_t *Ie, int32_t M, int32_t N, int b, const uint8_t *l_rot,
                     const uint8_t *msg, int64_t nbits, uint64_t k2, uint64_t nonce)
{
    return or_hide(Ie, M, N, l_rot, 6, b - 1, msg, nbits, k2, nonce);
}

int64_t or_lmr_extract(const uint8_t *Ie, int32_t M, int32_t N, int b, const uint8_t *l_rot,
                       uint8_t *msg, int64_t nbits, uint64_t k2, uint64_t nonce)
{
    return or_reveal(Ie, M, N, l_rot, 6, b - 1, msg, nbits, k2, nonce);
}

/* LMR recovery (Sec. III-B decoding with K1): XOR decryption, de-rotation of
 * the image and both maps, bit 7 from eta, then the glide over bits
 * 6..8-b guided by l. */
void or_lmr_recover(const uint8_t *Ie, int32_t M, int32_t N, int b, int min_level, uint64_t k1, uint64_t nonce,
                    const uint8_t *l_rot, const uint8_t *eta_rot, uint8_t *out)
{
    size_t MN = (size_t)M * (size_t)N;
    uint8_t *s = (uint8_t *)malloc(MN + 1);
    uint8_t *l = (uint8_t *)malloc(MN + 1);
    uint8_t *eta = (uint8_t *)malloc(MN + 1);
    or_keystream(k1, nonce, 1, 0, MN, s);
    memcpy(l, l_rot, MN);
    memcpy(eta, eta_rot, MN);
    for (size_t p = 0; p < MN; ++p) out[p] = (uint8_t)(Ie[p] ^ s[p]);
    or_rotate(out, M, N, s, min_level, 1);
    or_rotate(l, M, N, s, min_level, 1);
    or_rotate(eta, M, N, s, min_level, 1);
    for (size_t p = 0; p < MN; ++p) out[p] = (uint8_t)((out[p] & 0x7F) | ((eta[p] & 1) << 7));
    uint8_t mask = (uint8_t)((0xFF << (8 - b)) & 0x7F);
    recovery_glide(out, l, M, N, mask);
    free(s); free(l); free(eta);
}

/* ------------------------------------------------------------------------ */
/* LMR map compression (Sec. III-B "Maps generation, rotation, and           */
/* compression").  The paper uses JBIG-KIT; the library defines its own      */
/* bi-level coder and this is a second, plain implementation of that         */
/* definition:                                                               */
/*   pixels in raster order; context of ten already-coded neighbours         */
/*   (row-2: j-1, j, j+1; row-1: j-2 .. j+2; row: j-2, j-1; first listed is  */
/*   the highest bit; outside the plane = 0); per context a 12-bit           */
/*   probability of a 0, starting at 2048, moved by 1/32 of the distance     */
/*   to 0 or 4096 after each bit; a 32-bit range coder (bound =              */
/*   (range >> 12) * p; 0 keeps the low part; renormalise by bytes while     */
/*   range < 2^24; carries ripple into the bytes already written; four      */
/*   bytes of low flush the end).  Container: 32-bit big-endian byte counts  */
/*   of the eta part and the l part, then the two parts.                     */
/* ------------------------------------------------------------------------ */

static int plane_at(const uint8_t *P, int32_t M, int32_t N, int64_t i, int64_t j)
{
    if (i < 0 || i >= M || j < 0 || j >= N) return 0;
    return P[i * N + j] ? 1 : 0;
}

static int plane_context(const uint8_t *P, int32_t M, int32_t N, int64_t i, int64_t j)
{
    int c = 0;
    c = (c << 1) | plane_at(P, M, N, i - 2, j - 1);
    c = (c << 1) | plane_at(P, M, N, i - 2, j);
    c = (c << 1) | plane_at(P, M, N, i - 2, j + 1);
    c = (c << 1) | plane_at(P, M, N, i - 1, j - 2);
    c = (c << 1) | plane_at(P, M, N, i - 1, j - 1);
    c = (c << 1) | plane_at(P, M, N, i - 1, j);
    c = (c << 1) | plane_at(P, M, N, i - 1, j + 1);
    c = (c << 1) | plane_at(P, M, N, i - 1, j + 2);
    c = (c << 1) | plane_at(P, M, N, i, j - 2);
    c = (c << 1) | plane_at(P, M, N, i, j - 1);
    return c;
}

/* Encode a plane (one byte 0/1 per pixel) into out; returns the byte count,
 * or -1 if it would exceed cap. */
int64_t or_plane_encode(const uint8_t *P, int32_t M, int32_t N, uint8_t *out, int64_t cap)
{
    uint32_t prob[1024];
    for (int c = 0; c < 1024; ++c) prob[c] = 2048;
    uint64_t low = 0;
    uint32_t range = 0xFFFFFFFFu;
    int64_t n = 0;
    for (int64_t i = 0; i < M; ++i) {
        for (int64_t j = 0; j < N; ++j) {
            int c = plane_context(P, M, N, i, j);
            int bit = P[i * N + j] ? 1 : 0;
            uint32_t bound = (range >> 12) * prob[c];
            if (bit == 0) {
                range = bound;
                prob[c] += (4096 - prob[c]) >> 5;
            } else {
                low += bound;
                range -= bound;
                prob[c] -= prob[c] >> 5;
            }
            if (low >= ((uint64_t)1 << 32)) {          /* carry into written bytes */
                low -= (uint64_t)1 << 32;
                for (int64_t k = n - 1; k >= 0; --k) {
                    out[k] = (uint8_t)(out[k] + 1);
                    if (out[k] != 0) break;
                }
            }
            while (range < ((uint32_t)1 << 24)) {
                if (n >= cap) return -1;
                out[n++] = (uint8_t)(low >> 24);
                low = (low << 8) & 0xFFFFFFFFull;
                range <<= 8;
            }
        }
    }
    for (int k = 0; k < 4; ++k) {
        if (n >= cap) return -1;
        out[n++] = (uint8_t)(low >> 24);
        low = (low << 8) & 0xFFFFFFFFull;
    }
    return n;
}

/* Decode a plane of M x N bits from in[0..len) (bytes past the end read 0). */
void or_plane_decode(const uint8_t *in, int64_t len, int32_t M, int32_t N, uint8_t *P)
{
    uint32_t prob[1024];
    for (int c = 0; c < 1024; ++c) prob[c] = 2048;
    int64_t pos = 0;
    uint32_t code = 0, range = 0xFFFFFFFFu;
    for (int k = 0; k < 4; ++k) code = (code << 8) | (pos < len ? in[pos] : 0), ++pos;
    for (int64_t i = 0; i < M; ++i) {
        for (int64_t j = 0; j < N; ++j) {
            int c = plane_context(P, M, N, i, j);
            uint32_t bound = (range >> 12) * prob[c];
            int bit;
            if (code < bound) {
                bit = 0;
                range = bound;
                prob[c] += (4096 - prob[c]) >> 5;
            } else {
                bit = 1;
                code -= bound;
                range -= bound;
                prob[c] -= prob[c] >> 5;
            }
            P[i * N + j] = (uint8_t)bit;
            while (range < ((uint32_t)1 << 24)) {
                code = (code << 8) | (pos < len ? in[pos] : 0);
                ++pos;
                range <<= 8;
            }
        }
    }
}

/* Container of the two compressed maps; returns its length in bytes or -1
 * when it exceeds cap bytes. */
int64_t or_lmr_compress(const uint8_t *eta, const uint8_t *l, int32_t M, int32_t N, uint8_t *out, int64_t cap)
{
    if (cap < 8) return -1;
    int64_t ne = or_plane_encode(eta, M, N, out + 8, cap - 8);
    if (ne < 0) return -1;
    int64_t nl = or_plane_encode(l, M, N, out + 8 + ne, cap - 8 - ne);
    if (nl < 0) return -1;
    out[0] = (uint8_t)(ne >> 24); out[1] = (uint8_t)(ne >> 16); out[2] = (uint8_t)(ne >> 8); out[3] = (uint8_t)ne;
    out[4] = (uint8_t)(nl >> 24); out[5] = (uint8_t)(nl >> 16); out[6] = (uint8_t)(nl >> 8); out[7] = (uint8_t)nl;
    return 8 + ne + nl;
}

int or_lmr_decompress(const uint8_t *in, int64_t len, int32_t M, int32_t N, uint8_t *eta, uint8_t *l)
{
    if (len < 8) return -1;
    int64_t ne = ((int64_t)in[0] << 24) | ((int64_t)in[1] << 16) | ((int64_t)in[2] << 8) | in[3];
    int64_t nl = ((int64_t)in[4] << 24) | ((int64_t)in[5] << 16) | ((int64_t)in[6] << 8) | in[7];
    if (8 + ne + nl > len) return -1;
    or_plane_decode(in + 8, ne, M, N, eta);
    or_plane_decode(in + 8 + ne, nl, M, N, l);
    return 0;
}

/* LMR encoding phase (Sec. III-B): b in [2,8]; candidates in order of the
 * LMR capacity (b-1)*Z_b (ties: smaller b first); for each, rotate the maps
 * with blocks 2^min_level..2^n (the method uses 2^4; Table LMR_block_size
 * also starts at 2^1, 2^2 and 2^3), compress, and keep the first whose
 * stream fits the M*N-bit MSB plane (the "next most optimal location map"
 * fallback).  Returns 0 and fills Ie/meta/stream, or -1 for a bad case. */
int or_lmr_encode(const uint8_t *I, int32_t M, int32_t N, uint64_t k1, uint64_t nonce, int32_t min_level, uint8_t *Ie,
                  or_meta *meta, uint8_t *stream, int64_t *stream_bits)
{
    size_t MN = (size_t)M * (size_t)N;
    int64_t Z[7];
    or_redundancy_counts(I, M, N, 2, 8, Z);
    int order[7];
    for (int k = 0; k < 7; ++k) order[k] = 2 + k;
    for (int a = 1; a < 7; ++a) {            /* stable insertion sort, descending capacity */
        int v = order[a], k = a - 1;
        while (k >= 0 && (int64_t)(order[k] - 1) * Z[order[k] - 2] < (int64_t)(v - 1) * Z[v - 2]) {
            order[k + 1] = order[k];
            --k;
        }
        order[k + 1] = v;
    }
    uint8_t *l_rot = (uint8_t *)malloc(MN + 1), *eta_rot = (uint8_t *)malloc(MN + 1);
    int64_t cap = (int64_t)(MN / 8);
    int chosen = 0;
    int64_t len = -1;
    for (int k = 0; k < 7 && !chosen; ++k) {
        int b = order[k];
        or_lmr_rotated_maps(I, M, N, b, min_level, k1, nonce, l_rot, eta_rot);
        len = or_lmr_compress(eta_rot, l_rot, M, N, stream, cap);
        if (len >= 0) chosen = b;
    }
    free(l_rot); free(eta_rot);
    meta->min_level = min_level;
    meta->max_level = or_max_level(M, N);
    if (!chosen) {
        meta->b = 0; meta->redundant = 0; meta->capacity_bits = 0;
        *stream_bits = 0;
        return -1;
    }
    meta->b = chosen;
    meta->redundant = Z[chosen - 2];
    meta->capacity_bits = (int64_t)(chosen - 1) * Z[chosen - 2];
    *stream_bits = 8 * len;
    or_lmr_encrypt(I, M, N, min_level, k1, nonce, stream, 8 * len, Ie);
    return 0;
}

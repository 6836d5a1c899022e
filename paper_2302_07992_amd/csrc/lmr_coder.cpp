// Bi-level map coder for LMR-RDHEI (host stage).  The paper compresses the
// rotated first-MSB map and the rotated location map with JBIG-KIT so that
// both fit in the MSB plane (Sec. III-B, maps generation, rotation and
// compression).  This is the library's own lossless coder for such planes:
// an adaptive binary arithmetic coder driven by a 10-pixel context of already
// coded neighbours (two rows above and two pixels to the left).
//
// Coder definition (both directions follow it exactly):
//   context  c = x(i-2,j-1) x(i-2,j) x(i-2,j+1) x(i-1,j-2) x(i-1,j-1) x(i-1,j)
//               x(i-1,j+1) x(i-1,j+2) x(i,j-2) x(i,j-1)   (first = bit 9);
//               pixels outside the plane count as 0
//   model    p[c] = P(bit = 0) in 1/4096, starts at 2048; after coding a 0,
//            p += (4096 - p) >> 5, after a 1, p -= p >> 5
//   coder    32-bit range coder: bound = (range >> 12) * p; a 0 keeps
//            [low, low + bound), a 1 keeps [low + bound, low + range);
//            while range < 2^24 the top byte of low is emitted and range,
//            low shift left by 8; a carry out of low adds one to the bytes
//            already emitted; the end flushes the 4 bytes of low.
//   stream   u32 BE byte length of the eta part, u32 BE byte length of the
//            l part, eta part, l part.
#include <cstdint>
#include <cstring>
#include <vector>

#include "../../include/rdhei.h"

namespace rdhei {
namespace {

// Bit j of row i of a plane stored MSB-first, 0 outside the plane.
struct PlaneView {
    const uint8_t *bits;
    int32_t M, N;
    inline uint32_t at(int64_t i, int64_t j) const {
        if (i < 0 || j < 0 || j >= N) return 0;
        const int64_t p = i * N + j;
        return (bits[p >> 3] >> (7 - (p & 7))) & 1u;
    }
};

// The context of pixel (i, j), kept as three sliding windows: w2 = bits
// x(i-2, j-1..j+1), w1 = x(i-1, j-2..j+2), w0 = x(i, j-2..j-1) (first pixel
// in the highest bit).  Moving to j + 1 shifts one new pixel into each.
struct Context {
    uint32_t w2 = 0, w1 = 0, w0 = 0;
    void start_row(const PlaneView &v, int64_t i) {
        w2 = (v.at(i - 2, 0) << 1) | v.at(i - 2, 1);
        w1 = (v.at(i - 1, 0) << 2) | (v.at(i - 1, 1) << 1) | v.at(i - 1, 2);
        w0 = 0;
    }
    uint32_t value() const { return (w2 << 7) | (w1 << 2) | w0; }
    // after pixel (i, j) with value `bit`
    void advance(const PlaneView &v, int64_t i, int64_t j, uint32_t bit) {
        w2 = ((w2 << 1) | v.at(i - 2, j + 2)) & 7u;
        w1 = ((w1 << 1) | v.at(i - 1, j + 3)) & 31u;
        w0 = ((w0 << 1) | bit) & 3u;
    }
};

class Encoder {
   public:
    explicit Encoder(std::vector<uint8_t> &out) : out_(out) {}
    void put(uint32_t bit, uint16_t &p) {
        const uint32_t bound = (range_ >> 12) * p;
        if (!bit) {
            range_ = bound;
            p = (uint16_t)(p + ((4096u - p) >> 5));
        } else {
            low_ += bound;
            range_ -= bound;
            p = (uint16_t)(p - (p >> 5));
        }
        if (low_ >> 32) carry();
        while (range_ < (1u << 24)) {
            out_.push_back((uint8_t)(low_ >> 24));
            low_ = (low_ << 8) & 0xFFFFFFFFull;
            range_ <<= 8;
        }
    }
    void finish() {
        for (int k = 0; k < 4; ++k) {
            out_.push_back((uint8_t)(low_ >> 24));
            low_ = (low_ << 8) & 0xFFFFFFFFull;
        }
    }

   private:
    void carry() {
        low_ &= 0xFFFFFFFFull;
        for (size_t k = out_.size(); k-- > 0;) {
            if (++out_[k] != 0) break;
        }
    }
    std::vector<uint8_t> &out_;
    uint64_t low_ = 0;
    uint32_t range_ = 0xFFFFFFFFu;
};

class Decoder {
   public:
    Decoder(const uint8_t *in, int64_t n) : in_(in), n_(n) {
        for (int k = 0; k < 4; ++k) code_ = (code_ << 8) | next();
    }
    uint32_t get(uint16_t &p) {
        const uint32_t bound = (range_ >> 12) * p;
        uint32_t bit;
        if (code_ < bound) {
            range_ = bound;
            p = (uint16_t)(p + ((4096u - p) >> 5));
            bit = 0;
        } else {
            code_ -= bound;
            range_ -= bound;
            p = (uint16_t)(p - (p >> 5));
            bit = 1;
        }
        while (range_ < (1u << 24)) {
            code_ = (code_ << 8) | next();
            range_ <<= 8;
        }
        return bit;
    }
    bool overrun() const { return pos_ > n_ + 4; }

   private:
    uint32_t next() { return pos_ < n_ ? in_[pos_++] : (++pos_, 0u); }
    const uint8_t *in_;
    int64_t n_;
    int64_t pos_ = 0;
    uint32_t code_ = 0;
    uint32_t range_ = 0xFFFFFFFFu;
};

void encode_plane(const uint8_t *bits, int32_t M, int32_t N, std::vector<uint8_t> &out) {
    std::vector<uint16_t> p(1024, 2048);
    Encoder enc(out);
    PlaneView v{bits, M, N};
    Context c;
    for (int64_t i = 0; i < M; ++i) {
        c.start_row(v, i);
        for (int64_t j = 0; j < N; ++j) {
            const uint32_t bit = v.at(i, j);
            enc.put(bit, p[c.value()]);
            c.advance(v, i, j, bit);
        }
    }
    enc.finish();
}

bool decode_plane(const uint8_t *in, int64_t n, int32_t M, int32_t N, uint8_t *bits) {
    std::vector<uint16_t> p(1024, 2048);
    Decoder dec(in, n);
    const uint64_t MN = (uint64_t)M * N;
    memset(bits, 0, (size_t)((MN + 7) / 8));
    PlaneView v{bits, M, N};
    Context c;
    for (int64_t i = 0; i < M; ++i) {
        c.start_row(v, i);
        for (int64_t j = 0; j < N; ++j) {
            const uint32_t bit = dec.get(p[c.value()]);
            const int64_t q = i * N + j;
            if (bit) bits[q >> 3] |= (uint8_t)(0x80u >> (q & 7));
            c.advance(v, i, j, bit);
        }
    }
    return !dec.overrun();
}

void put_be32(uint8_t *d, uint32_t v) {
    d[0] = (uint8_t)(v >> 24); d[1] = (uint8_t)(v >> 16); d[2] = (uint8_t)(v >> 8); d[3] = (uint8_t)v;
}
uint32_t get_be32(const uint8_t *d) {
    return ((uint32_t)d[0] << 24) | ((uint32_t)d[1] << 16) | ((uint32_t)d[2] << 8) | d[3];
}

}  // namespace

int lmr_compress_impl(const uint8_t *eta_bits, const uint8_t *l_bits, int32_t M, int32_t N, uint8_t *stream,
                      int64_t capacity_bytes, int64_t *stream_bits) {
    std::vector<uint8_t> e, l;
    e.reserve(4096);
    l.reserve(4096);
    encode_plane(eta_bits, M, N, e);
    encode_plane(l_bits, M, N, l);
    const int64_t total = 8 + (int64_t)e.size() + (int64_t)l.size();
    *stream_bits = 8 * total;
    if (total > capacity_bytes) return RDHEI_ENOFIT;
    put_be32(stream, (uint32_t)e.size());
    put_be32(stream + 4, (uint32_t)l.size());
    memcpy(stream + 8, e.data(), e.size());
    memcpy(stream + 8 + e.size(), l.data(), l.size());
    return RDHEI_OK;
}

int lmr_decompress_impl(const uint8_t *stream, int64_t stream_bytes, int32_t M, int32_t N, uint8_t *eta_bits,
                        uint8_t *l_bits) {
    const int64_t ne = get_be32(stream), nl = get_be32(stream + 4);
    if (8 + ne + nl > stream_bytes) return RDHEI_ECORRUPT;
    if (!decode_plane(stream + 8, ne, M, N, eta_bits)) return RDHEI_ECORRUPT;
    if (!decode_plane(stream + 8 + ne, nl, M, N, l_bits)) return RDHEI_ECORRUPT;
    return RDHEI_OK;
}

}  // namespace rdhei

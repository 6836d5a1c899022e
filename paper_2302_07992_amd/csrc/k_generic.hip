// Per-pixel path for shapes the tiled path does not cover (any M x N): the
// rotation codes of every level stored as one byte per block, and the block
// turns applied level by level per pixel.  Same output as the tiled path.
#include "device.hpp"

namespace rdhei {

// Offset of level m (>= 1) in the all-level code array.
__host__ __device__ inline uint64_t gen_off(int M, int N, int m) {
    uint64_t off = 0;
    for (int k = 1; k < m; ++k) off += (uint64_t)(M >> k) * (uint64_t)(N >> k);
    return off;
}

// Level 1: code of each full 2x2 block = (sum of its four keystream bytes) mod 4.
// Also clears the image's statistics record.
template <int KS>
__global__ void k_gen_level1(const Job *__restrict__ jobs, int j, uint8_t *__restrict__ ws) {
    const Job &J = jobs[j];
    const uint64_t nz = job_nonce(J);
    const uint32_t gx = (uint32_t)(J.N >> 1), gy = (uint32_t)(J.M >> 1);
    const uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q == 0) {
        uint32_t *st = reinterpret_cast<uint32_t *>(ws + J.ws_stats);
        for (int k = 0; k < kStatWords; ++k) st[k] = 0;
    }
    if (q >= (uint64_t)gx * gy) return;
    const uint32_t Y = (uint32_t)(q / gx), X = (uint32_t)(q % gx);
    const uint64_t p = (uint64_t)(2 * Y) * (uint64_t)J.N + 2 * X;
    const uint32_t sum = stream_byte<KS>(J.key, nz, kDomainImage, p) + stream_byte<KS>(J.key, nz, kDomainImage, p + 1) +
                         stream_byte<KS>(J.key, nz, kDomainImage, p + J.N) +
                         stream_byte<KS>(J.key, nz, kDomainImage, p + J.N + 1);
    ws[J.ws_codes + gen_off(J.M, J.N, 1) + q] = (uint8_t)(sum & 3u);
}

// Level m from level m-1: the four children of a full block are full blocks.
__global__ void k_gen_level_up(const Job *__restrict__ jobs, int j, uint8_t *__restrict__ ws, int m) {
    const Job &J = jobs[j];
    const uint32_t gx = (uint32_t)(J.N >> m), gy = (uint32_t)(J.M >> m);
    const uint32_t cx = (uint32_t)(J.N >> (m - 1));
    const uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (uint64_t)gx * gy) return;
    const uint32_t Y = (uint32_t)(q / gx), X = (uint32_t)(q % gx);
    const uint8_t *c = ws + J.ws_codes + gen_off(J.M, J.N, m - 1) + (uint64_t)(2 * Y) * cx + 2 * X;
    ws[J.ws_codes + gen_off(J.M, J.N, m) + q] = (uint8_t)((c[0] + c[1] + c[cx] + c[cx + 1]) & 3);
}

// Z_b (b = 2..8): pixels with a left neighbour and lambda >= b.
__global__ void k_gen_stats(const Job *__restrict__ jobs, int j, uint8_t *__restrict__ ws) {
    const Job &J = jobs[j];
    __shared__ uint32_t h[7];
    if (threadIdx.x < 7) h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t total = (uint64_t)J.M * (uint64_t)J.N;
    const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < total && (p % (uint64_t)J.N) != 0) {
        const uint32_t x = (uint32_t)(J.in[p] ^ J.in[p - 1]);
        const uint32_t lam = __clz((x << 24) | 0x00800000u);
        if (lam >= 2) atomicAdd(&h[lam - 2], 1u);
    }
    __syncthreads();
    if (threadIdx.x < 7) {
        uint32_t z = 0;
        for (int k = (int)threadIdx.x; k < 7; ++k) z += h[k];
        if (z) atomicAdd(reinterpret_cast<uint32_t *>(ws + J.ws_stats) + threadIdx.x, z);
    }
}

// Forward rotation of original position (y, x): levels min_level..n ascending.
__device__ inline void gen_forward(const Job &J, const uint8_t *codes, uint32_t y, uint32_t x,
                                   uint32_t &oy, uint32_t &ox) {
    uint32_t cy = y, cx = x;
    for (int m = J.min_level; m <= J.max_level; ++m) {
        const uint32_t gy = (uint32_t)(J.M >> m), gx = (uint32_t)(J.N >> m);
        const uint32_t BY = y >> m, BX = x >> m;
        if (BY < gy && BX < gx) {
            const uint32_t r = codes[gen_off(J.M, J.N, m) + (uint64_t)BY * gx + BX] & 3u;
            const uint32_t mask = (1u << m) - 1u;
            uint32_t ly = cy & mask, lx = cx & mask;
            turn_bits(r, ly, lx, mask);
            cy = (cy & ~mask) | ly;
            cx = (cx & ~mask) | lx;
        }
    }
    oy = cy;
    ox = cx;
}

template <int MODE, int KS>
__global__ void k_gen_encrypt(const Job *__restrict__ jobs, int j, uint8_t *__restrict__ ws) {
    const Job &J = jobs[j];
    const uint64_t nz = job_nonce(J);
    const uint64_t total = (uint64_t)J.M * (uint64_t)J.N;
    const uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= total) return;
    if (MODE == ENC_EMR && J.meta->status != RDHEI_OK) return;
    const int b = J.fixed_b > 0 ? J.fixed_b : J.meta->b;
    const uint32_t y = (uint32_t)(q / (uint64_t)J.N), x = (uint32_t)(q % (uint64_t)J.N);
    uint32_t py, px;
    gen_forward(J, ws + J.ws_codes, y, x, py, px);
    const uint64_t p = (uint64_t)py * (uint64_t)J.N + px;
    const uint32_t v = J.in[q];
    uint32_t l = 1;
    if (x > 0) l = ((v ^ (uint32_t)J.in[q - 1]) >> (8 - b)) != 0u;
    if (MODE == ENC_LMR_MAPS) {
        ws[J.ws_bytes + p] = (uint8_t)((l << 1) | (v >> 7));
        return;
    }
    const uint32_t s = stream_byte<KS>(J.key, nz, kDomainImage, p);
    uint32_t e;
    if (MODE == ENC_EMR) {
        e = ((v ^ s) & 0xFEu) | l;
    } else {
        e = v ^ s;
        if ((int64_t)p < J.stream_bits) {
            const uint32_t bit = (J.stream[p >> 3] >> (7 - (p & 7))) & 1u;
            e = (e & 0x7Fu) | (bit << 7);
        }
    }
    J.out[p] = (uint8_t)e;
}

// Pack the byte-per-pixel LMR maps into two MSB-first bit planes (out: l, msg: eta).
__global__ void k_gen_pack(const Job *__restrict__ jobs, int j, const uint8_t *__restrict__ ws) {
    const Job &J = jobs[j];
    const uint64_t total = (uint64_t)J.M * (uint64_t)J.N;
    const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (8 * k >= total) return;
    uint32_t lb = 0, eb = 0;
    for (int t = 0; t < 8; ++t) {
        const uint64_t p = 8 * k + t;
        const uint32_t v = p < total ? ws[J.ws_bytes + p] : 0u;
        lb |= ((v >> 1) & 1u) << (7 - t);
        eb |= (v & 1u) << (7 - t);
    }
    J.out[k] = (uint8_t)lb;
    J.msg[k] = (uint8_t)eb;
}

// One thread per row: gather, decrypt, glide.
template <int METHOD, int KS>
__global__ void k_gen_recover(const Job *__restrict__ jobs, int j, const uint8_t *__restrict__ ws) {
    const Job &J = jobs[j];
    const uint64_t nz = job_nonce(J);
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (uint32_t)J.M) return;
    const int b = J.meta->b;
    const uint32_t mask = METHOD == RDHEI_EMR ? ((0xFFu << (8 - b)) & 0xFFu) : ((0xFFu << (8 - b)) & 0x7Fu);
    uint32_t omega = 0;
    for (uint32_t x = 0; x < (uint32_t)J.N; ++x) {
        uint32_t py, px;
        gen_forward(J, ws + J.ws_codes, i, x, py, px);
        const uint64_t p = (uint64_t)py * (uint64_t)J.N + px;
        const uint32_t e = J.in[p];
        uint32_t D = e ^ stream_byte<KS>(J.key, nz, kDomainImage, p);
        uint32_t l;
        if (METHOD == RDHEI_EMR) {
            l = e & 1u;
        } else {
            l = (J.lbits[p >> 3] >> (7 - (p & 7))) & 1u;
            D = (D & 0x7Fu) | (((J.etabits[p >> 3] >> (7 - (p & 7))) & 1u) << 7);
        }
        if (l || x == 0) omega = D & mask;
        else D = (D & ~mask) | omega;
        J.out[(uint64_t)i * (uint64_t)J.N + x] = (uint8_t)D;
    }
}

static inline unsigned blocks(uint64_t n, unsigned t) { return (unsigned)((n + t - 1) / t); }

void launch_generic_levels(const Launch &L, int j, const Job &h) {
    const uint64_t n1 = h.max_level >= 1 ? (uint64_t)(h.M >> 1) * (uint64_t)(h.N >> 1) : 1;
    with_keystream(L.keystream, [&](auto K) {
        hipLaunchKernelGGL(k_gen_level1<decltype(K)::value>, dim3(blocks(n1 ? n1 : 1, 256)), dim3(256), 0, L.stream,
                           L.jobs, j, L.ws);
    });
    for (int m = 2; m <= h.max_level; ++m) {
        const uint64_t n = (uint64_t)(h.M >> m) * (uint64_t)(h.N >> m);
        hipLaunchKernelGGL(k_gen_level_up, dim3(blocks(n, 256)), dim3(256), 0, L.stream, L.jobs, j, L.ws, m);
    }
}

void launch_generic_stats(const Launch &L, int j, const Job &h) {
    const uint64_t n = (uint64_t)h.M * (uint64_t)h.N;
    hipLaunchKernelGGL(k_gen_stats, dim3(blocks(n, 256)), dim3(256), 0, L.stream, L.jobs, j, L.ws);
}

void launch_generic_encrypt(const Launch &L, int j, const Job &h, int mode) {
    const uint64_t n = (uint64_t)h.M * (uint64_t)h.N;
    const dim3 g(blocks(n, 256)), b(256);
    with_keystream(L.keystream, [&](auto K) {
        constexpr int KS = decltype(K)::value;
        if (mode == ENC_EMR) hipLaunchKernelGGL((k_gen_encrypt<ENC_EMR, KS>), g, b, 0, L.stream, L.jobs, j, L.ws);
        else if (mode == ENC_LMR) hipLaunchKernelGGL((k_gen_encrypt<ENC_LMR, KS>), g, b, 0, L.stream, L.jobs, j, L.ws);
        else hipLaunchKernelGGL((k_gen_encrypt<ENC_LMR_MAPS, KS>), g, b, 0, L.stream, L.jobs, j, L.ws);
    });
    if (mode == ENC_LMR_MAPS)
        hipLaunchKernelGGL(k_gen_pack, dim3(blocks((n + 7) / 8, 256)), b, 0, L.stream, L.jobs, j, L.ws);
}

void launch_generic_recover(const Launch &L, int j, const Job &h) {
    const dim3 g(blocks((uint64_t)h.M, 64)), b(64);
    with_keystream(L.keystream, [&](auto K) {
        constexpr int KS = decltype(K)::value;
        if (h.method == RDHEI_EMR) hipLaunchKernelGGL((k_gen_recover<RDHEI_EMR, KS>), g, b, 0, L.stream, L.jobs, j, L.ws);
        else hipLaunchKernelGGL((k_gen_recover<RDHEI_LMR, KS>), g, b, 0, L.stream, L.jobs, j, L.ws);
    });
}

uint64_t generic_code_bytes(int M, int N, int n) { return gen_off(M, N, n + 1); }

}  // namespace rdhei

// Image metrics of Sec. IV (quality of the reconstruction, security of the
// encrypted and marked images) over a batch of image pairs (a, b):
//   entropy and chi-square test of a and of b (Sec. IV-B equations),
//   NPCR, UACI and PSNR of the pair (Sec. IV-B equations; NPCR counts the
//   positions where the two images differ),
//   SSIM of the pair: mean over every 7x7 window inside the image of the
//   structural similarity with sample (co)variances, K1 = 0.01, K2 = 0.03,
//   L = 255 (uniform window; the paper names no variant).
// Everything but the final divisions and logarithms is exact integer
// arithmetic: level counts, differing pixels, sum |a - b|, sum (a - b)^2 and
// the window sums of a, b, a^2, b^2, ab.
#include "device.hpp"
#include "internal.hpp"

namespace rdhei {

// Job of unit u: the last job whose first unit is at most u (wave-uniform).
template <bool SSIM>
__device__ __forceinline__ int metric_job(const MetricJob *jobs, int njobs, uint32_t u) {
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        const uint32_t f = SSIM ? jobs[mid].ssim_first : jobs[mid].sum_first;
        if (f <= u) lo = mid;
        else hi = mid - 1;
    }
    return (int)uni((uint32_t)lo);
}

__global__ void k_metric_zero(MetricAcc *acc, uint32_t words16) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < words16) reinterpret_cast<uint4 *>(acc)[i] = make_uint4(0, 0, 0, 0);
}

// ---- level counts and pixel differences -----------------------------------
// One workgroup per kMetricChunk-pixel run of an image (grid-stride).  Each
// wave counts levels into its own LDS histograms; the run's counts then go
// to the job's counters with one atomic add per level.  Per four pixels: bytes that differ from the XOR,
// sum |a-b| with one sum-of-absolute-differences, sum (a-b)^2 as a.a + b.b -
// 2 a.b with three 4-byte dot products.
__device__ __forceinline__ void diff4(uint32_t x, uint32_t y, uint32_t &nd, uint32_t &sa, uint32_t &s2, uint32_t &sxy) {
    const uint32_t d = x ^ y;
    nd += (uint32_t)__popc((((d & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | d) & 0x80808080u);
    sa = __builtin_amdgcn_sad_u8(x, y, sa);
    s2 = __builtin_amdgcn_udot4(x, x, __builtin_amdgcn_udot4(y, y, s2, false), false);
    sxy = __builtin_amdgcn_udot4(x, y, sxy, false);
}

__global__ __launch_bounds__(kThreads) void k_metric_sums(const MetricJob *__restrict__ jobs, int njobs,
                                                           MetricAcc *__restrict__ acc, uint32_t units) {
    constexpr int kW = kThreads / 64;
    __shared__ uint32_t hist[kW][2][256];
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
    uint32_t *ha = hist[wave][0], *hb = hist[wave][1];
    for (uint32_t u = blockIdx.x; u < units; u += gridDim.x) {
        const int j = metric_job<false>(jobs, njobs, u);
        const MetricJob &J = jobs[j];
        const uint64_t MN = (uint64_t)J.M * (uint64_t)J.N;
        const uint64_t p0 = (uint64_t)(u - J.sum_first) * kMetricChunk;
        const uint64_t p1 = p0 + kMetricChunk < MN ? p0 + kMetricChunk : MN;
        const bool pair = J.b != nullptr;
        for (uint32_t i = tid; i < kW * 2 * 256; i += kThreads) (&hist[0][0][0])[i] = 0;
        __syncthreads();
        uint32_t nd = 0, sa = 0, s2 = 0, sxy = 0;
        auto count4 = [&](uint32_t x, uint32_t y) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                atomicAdd(&ha[(x >> (8 * k)) & 0xFFu], 1u);
                if (pair) atomicAdd(&hb[(y >> (8 * k)) & 0xFFu], 1u);
            }
            if (pair) diff4(x, y, nd, sa, s2, sxy);
        };
        uint64_t q0 = p0;
        if (J.vec) {
            // whole 16-byte groups (p0 is a multiple of 16), consecutive lanes on
            // consecutive groups, the next group loaded ahead; then the tail
            const uint64_t g1 = p0 + (p1 - p0) / 16 * 16;
            uint64_t q = p0 + 16 * (uint64_t)tid;
            uint4 x = make_uint4(0, 0, 0, 0), y = make_uint4(0, 0, 0, 0);
            if (q < g1) {
                x = gload<uint4>(J.a + q);
                if (pair) y = gload<uint4>(J.b + q);
            }
            for (; q < g1; q += 16 * (uint64_t)kThreads) {
                const uint4 cx = x, cy = y;
                const uint64_t qn = q + 16 * (uint64_t)kThreads;
                if (qn < g1) {
                    x = gload<uint4>(J.a + qn);
                    if (pair) y = gload<uint4>(J.b + qn);
                }
                count4(cx.x, cy.x);
                count4(cx.y, cy.y);
                count4(cx.z, cy.z);
                count4(cx.w, cy.w);
            }
            q0 = g1;
        }
        for (uint64_t q = q0 + tid; q < p1; q += kThreads) {   // bytes one by one
            const uint32_t x = J.a[q], y = pair ? J.b[q] : 0u;
            atomicAdd(&ha[x], 1u);
            if (pair) {
                atomicAdd(&hb[y], 1u);
                nd += x != y;
                sa += x > y ? x - y : y - x;
                s2 += x * x + y * y;
                sxy += x * y;
            }
        }
        __syncthreads();
        MetricAcc &A = acc[j];
        for (uint32_t v = tid; v < 256; v += kThreads) {
            uint32_t ca = 0, cb = 0;
#pragma unroll
            for (int w = 0; w < kW; ++w) {
                ca += hist[w][0][v];
                cb += hist[w][1][v];
            }
            if (ca) atomicAdd(&A.ha[v], ca);
            if (cb) atomicAdd(&A.hb[v], cb);
        }
        if (pair) {
            // this run's sums (each lane's fit 32 bits: at most 1,024 pixels of 255^2)
            unsigned long long n64 = nd, a64 = sa, q64 = (unsigned long long)s2 - 2ull * sxy;
            for (int off = 32; off > 0; off >>= 1) {
                n64 += __shfl_down(n64, off, 64);
                a64 += __shfl_down(a64, off, 64);
                q64 += __shfl_down(q64, off, 64);
            }
            if (lane == 0) {
                atomicAdd(&A.ndiff, n64);
                atomicAdd(&A.sabs, a64);
                atomicAdd(&A.ssq, q64);
            }
        }
        __syncthreads();   // the next run clears the histograms
    }
}

// ---- SSIM ------------------------------------------------------------------
// One workgroup per tile of kSsimRows x kSsimCols window anchors (grid-
// stride): the tile's pixels of both images (anchors plus 6 rows and
// columns) go to LDS; thread t owns anchor column t, runs down the rows with
// the last seven rows' horizontal sums in registers (one ring slot per row
// of a 7-row group) and a running vertical sum, and scores each window from
// its exact integer sums with one double division.
__device__ __forceinline__ double ssim_window(int32_t sa, int32_t sb, int32_t saa, int32_t sbb, int32_t sab) {
    // With n = 49 pixels the means are s/n and the sample (co)variances
    // (n s_xy - s_x s_y) / (n (n - 1)); scaling the luminance factor by n^2
    // and the contrast-structure factor by n (n - 1) leaves integers (below
    // 2^31 for 8-bit pixels) plus the constants C1 n^2 and C2 n (n - 1).
    constexpr int32_t n = kSsimWin * kSsimWin;
    constexpr double C1n = (0.01 * 255.0) * (0.01 * 255.0) * (double)(n * n);
    constexpr double C2n = (0.03 * 255.0) * (0.03 * 255.0) * (double)(n * (n - 1));
    const int32_t pab = sa * sb;
    const double l_num = (double)(2 * pab) + C1n, l_den = (double)(sa * sa + sb * sb) + C1n;
    const double c_num = (double)(2 * (n * sab - pab)) + C2n;
    const double c_den = (double)((n * saa - sa * sa) + (n * sbb - sb * sb)) + C2n;
    return (l_num * c_num) / (l_den * c_den);
}

__global__ __launch_bounds__(kThreads) void k_metric_ssim(const MetricJob *__restrict__ jobs, int njobs,
                                                           MetricAcc *__restrict__ acc, uint32_t tiles) {
    constexpr int kPR = kSsimRows + kSsimWin - 1, kPC = kSsimCols + kSsimWin - 1, kStride = (kPC + 3) / 4 * 4 + 4;
    static_assert(kSsimCols == kThreads, "one anchor column per thread");
    __shared__ __align__(16) uint8_t pa[kPR * kStride], pb[kPR * kStride];
    const uint32_t tid = threadIdx.x, lane = tid & 63u;
    for (uint32_t u = blockIdx.x; u < tiles; u += gridDim.x) {
        const int j = metric_job<true>(jobs, njobs, u);
        const MetricJob &J = jobs[j];
        const int AR = J.M - kSsimWin + 1, AC = J.N - kSsimWin + 1;   // anchors per column / row
        const int tcols = (AC + kSsimCols - 1) / kSsimCols;
        const int v = (int)(u - J.ssim_first);
        const int r0 = v / tcols * kSsimRows, c0 = v % tcols * kSsimCols;
        const int rows = (AR - r0 < kSsimRows ? AR - r0 : kSsimRows) + kSsimWin - 1;   // pixel rows of the tile
        __syncthreads();   // the previous tile's readers are done
        if (J.vec && (J.N & 3) == 0) {
            // 4-byte words (rows and the tile's first column are 4-aligned)
            constexpr int kPW = (kPC + 3) / 4;
            for (int i = (int)tid; i < kPR * kPW; i += kThreads) {
                const int y = i / kPW, x = 4 * (i % kPW);
                const bool in = y < rows && c0 + x < J.N;   // a word is inside the row or outside it
                const uint64_t off = (uint64_t)(r0 + y) * (uint64_t)J.N + (uint64_t)(c0 + x);
                const uint32_t wa = in ? *reinterpret_cast<const uint32_t *>(J.a + off) : 0u;
                const uint32_t wb = in ? *reinterpret_cast<const uint32_t *>(J.b + off) : 0u;
                *reinterpret_cast<uint32_t *>(pa + y * kStride + x) = wa;
                *reinterpret_cast<uint32_t *>(pb + y * kStride + x) = wb;
            }
        } else {
            for (int i = (int)tid; i < kPR * kPC; i += kThreads) {
                const int y = i / kPC, x = i % kPC;
                const bool in = y < rows && c0 + x < J.N;
                const uint64_t off = (uint64_t)(r0 + y) * (uint64_t)J.N + (uint64_t)(c0 + x);
                pa[y * kStride + x] = in ? J.a[off] : 0;
                pb[y * kStride + x] = in ? J.b[off] : 0;
            }
        }
        __syncthreads();
        const bool col = c0 + (int)tid < AC;
        int32_t ra[kSsimWin], rb[kSsimWin], raa[kSsimWin], rbb[kSsimWin], rab[kSsimWin];
        int32_t sa = 0, sb = 0, saa = 0, sbb = 0, sab = 0;
        double part = 0.0;
        for (int y0 = 0; y0 < rows; y0 += kSsimWin) {
#pragma unroll
            for (int k = 0; k < kSsimWin; ++k) {
                const int y = y0 + k;
                if (y < rows) {   // uniform over the workgroup
                    // bytes tid .. tid + 6 of the row as two words (the second
                    // masked to three bytes), from three aligned LDS words
                    const uint32_t *wa = reinterpret_cast<const uint32_t *>(pa + y * kStride) + (tid >> 2);
                    const uint32_t *wb = reinterpret_cast<const uint32_t *>(pb + y * kStride) + (tid >> 2);
                    const uint32_t sh = (tid & 3u) * 8u;
                    const uint32_t a0 = __builtin_amdgcn_alignbit(wa[1], wa[0], sh);
                    const uint32_t a1 = __builtin_amdgcn_alignbit(wa[2], wa[1], sh) & 0x00FFFFFFu;
                    const uint32_t b0 = __builtin_amdgcn_alignbit(wb[1], wb[0], sh);
                    const uint32_t b1 = __builtin_amdgcn_alignbit(wb[2], wb[1], sh) & 0x00FFFFFFu;
                    // byte sums by sum-of-absolute-differences against 0, the
                    // products by 4-byte dot products
                    const int32_t ha = (int32_t)__builtin_amdgcn_sad_u8(a0, 0u, __builtin_amdgcn_sad_u8(a1, 0u, 0u));
                    const int32_t hb = (int32_t)__builtin_amdgcn_sad_u8(b0, 0u, __builtin_amdgcn_sad_u8(b1, 0u, 0u));
                    const int32_t haa = (int32_t)__builtin_amdgcn_udot4(a0, a0, __builtin_amdgcn_udot4(a1, a1, 0u, false), false);
                    const int32_t hbb = (int32_t)__builtin_amdgcn_udot4(b0, b0, __builtin_amdgcn_udot4(b1, b1, 0u, false), false);
                    const int32_t hab = (int32_t)__builtin_amdgcn_udot4(a0, b0, __builtin_amdgcn_udot4(a1, b1, 0u, false), false);
                    if (y >= kSsimWin) {   // row y - 7 leaves the window
                        sa -= ra[k];
                        sb -= rb[k];
                        saa -= raa[k];
                        sbb -= rbb[k];
                        sab -= rab[k];
                    }
                    ra[k] = ha;
                    rb[k] = hb;
                    raa[k] = haa;
                    rbb[k] = hbb;
                    rab[k] = hab;
                    sa += ha;
                    sb += hb;
                    saa += haa;
                    sbb += hbb;
                    sab += hab;
                    if (y >= kSsimWin - 1 && col) part += ssim_window(sa, sb, saa, sbb, sab);
                }
            }
        }
        for (int off = 32; off > 0; off >>= 1) part += __shfl_down(part, off, 64);
        if (lane == 0) atomicAdd(&acc[j].ssim, part);
    }
}

// ---- per-job results -------------------------------------------------------
// One wave per job: lane l takes levels 4l .. 4l + 3 of the entropy and
// chi-square sums, a shuffle tree adds the lanes up, lane 0 writes
// out[8 j + k]: entropy(a), chi2(a), entropy(b), chi2(b), NPCR, UACI, PSNR,
// SSIM (NaN where b is absent, SSIM not asked for or the image is smaller
// than the window; PSNR infinite for identical images).
__device__ __forceinline__ void level_terms(const uint32_t *h, double MN, uint32_t lane, double &H, double &X) {
    H = 0.0;
    X = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t c = h[4 * lane + (uint32_t)k];
        const double p = (double)c / MN;
        if (c) H -= p * log2(p);
        const double d = p - 1.0 / 256.0;
        X += d * d;
    }
    for (int off = 32; off > 0; off >>= 1) {
        H += __shfl_down(H, off, 64);
        X += __shfl_down(X, off, 64);
    }
}

__global__ __launch_bounds__(kThreads) void k_metric_final(const MetricJob *__restrict__ jobs, int njobs,
                                                            const MetricAcc *__restrict__ acc, int with_ssim,
                                                            double *__restrict__ out) {
    const int j = (int)(blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6));
    if (j >= njobs) return;   // whole waves
    const uint32_t lane = threadIdx.x & 63u;
    const MetricJob &J = jobs[j];
    const MetricAcc &A = acc[j];
    const double MN = (double)J.M * (double)J.N;
    const double nan = __builtin_nan("");
    double *o = out + 8 * (uint64_t)j;
    double Ha, Xa, Hb = 0.0, Xb = 0.0;
    level_terms(A.ha, MN, lane, Ha, Xa);
    if (J.b) level_terms(A.hb, MN, lane, Hb, Xb);
    if (lane != 0) return;
    o[0] = Ha;
    o[1] = 256.0 * MN * Xa;
    if (!J.b) {
        for (int k = 2; k < 8; ++k) o[k] = nan;
        return;
    }
    o[2] = Hb;
    o[3] = 256.0 * MN * Xb;
    o[4] = 100.0 * (double)A.ndiff / MN;
    o[5] = 100.0 * (double)A.sabs / (255.0 * MN);
    o[6] = A.ssq == 0 ? __builtin_inf() : 10.0 * log10(255.0 * 255.0 / ((double)A.ssq / MN));
    const bool win = J.M >= kSsimWin && J.N >= kSsimWin;
    o[7] = with_ssim && win ? A.ssim / ((double)(J.M - kSsimWin + 1) * (double)(J.N - kSsimWin + 1)) : nan;
}

void launch_metrics(const MetricJob *jobs, int njobs, MetricAcc *acc, uint32_t sum_units, uint32_t ssim_tiles,
                    int with_ssim, double *out, hipStream_t st) {
    const uint32_t words16 = (uint32_t)((uint64_t)njobs * sizeof(MetricAcc) / 16);
    hipLaunchKernelGGL(k_metric_zero, dim3((words16 + 255) / 256), dim3(256), 0, st, acc, words16);
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const uint32_t cap = (uint32_t)(cus > 0 ? cus : 1) * 16u;
    if (sum_units)
        hipLaunchKernelGGL(k_metric_sums, dim3(sum_units < cap ? sum_units : cap), dim3(kThreads), 0, st, jobs, njobs,
                           acc, sum_units);
    if (with_ssim && ssim_tiles)
        hipLaunchKernelGGL(k_metric_ssim, dim3(ssim_tiles < cap ? ssim_tiles : cap), dim3(kThreads), 0, st, jobs,
                           njobs, acc, ssim_tiles);
    constexpr int kJobsPerBlock = kThreads / 64;
    hipLaunchKernelGGL(k_metric_final, dim3((njobs + kJobsPerBlock - 1) / kJobsPerBlock), dim3(kThreads), 0, st, jobs,
                       njobs, acc, with_ssim, out);
}

}  // namespace rdhei

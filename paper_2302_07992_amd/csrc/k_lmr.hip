// Batch helpers around the LMR host coder (Sec. III-B): gather every image's
// label counts and meta record into contiguous arrays for one copy to the
// host, scatter host-built meta records back, and pack the map stream that an
// LMR marked image carries in bit 7 of its first map_bits pixels.
#include "device.hpp"

namespace rdhei {

// Z_b (b = 2..8) of each image, left in the workspace by the finalisation.
__global__ void k_gather_z(const Job *__restrict__ jobs, int njobs, const uint8_t *__restrict__ ws,
                           int64_t *__restrict__ out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= njobs) return;
    const Job &J = jobs[j];
    const int64_t *z = reinterpret_cast<const int64_t *>(ws + stat_z_offset(J));
    for (int k = 0; k < 7; ++k) out[7 * j + k] = z[k];
}

__global__ void k_gather_meta(const Job *__restrict__ jobs, int njobs, rdhei_meta *__restrict__ out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < njobs) out[j] = *jobs[j].meta;
}

__global__ void k_scatter_meta(const Job *__restrict__ jobs, int njobs, const rdhei_meta *__restrict__ in) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < njobs) *jobs[j].meta = in[j];
}

// Image blockIdx.y: bit 7 of pixels [0, map_bits) packed MSB-first at
// out + off[j]; images whose record is not usable are skipped.
__global__ void k_msb_plane(const Job *__restrict__ jobs, const uint64_t *__restrict__ off, uint8_t *__restrict__ out) {
    const Job &J = jobs[blockIdx.y];
    const rdhei_meta *m = J.meta;
    const int64_t bits = m->map_bits;
    const int64_t MN = (int64_t)J.M * J.N;
    if (m->status != RDHEI_OK || bits < 64 || bits > MN) return;
    const uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;   // output byte
    if ((int64_t)(8 * q) >= bits) return;
    uint32_t v = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k)
        if ((int64_t)(8 * q + k) < bits) v |= (uint32_t)((J.in[8 * q + k] >> 7) & 1u) << (7 - k);
    out[off[blockIdx.y] + q] = (uint8_t)v;
}

void launch_gather_z(const Launch &L, int64_t *out) {
    if (!L.njobs) return;
    hipLaunchKernelGGL(k_gather_z, dim3((L.njobs + 255) / 256), dim3(256), 0, L.stream, L.jobs, L.njobs, L.ws, out);
}

void launch_gather_meta(const Launch &L, rdhei_meta *out) {
    if (!L.njobs) return;
    hipLaunchKernelGGL(k_gather_meta, dim3((L.njobs + 255) / 256), dim3(256), 0, L.stream, L.jobs, L.njobs, out);
}

void launch_scatter_meta(const Launch &L, const rdhei_meta *in) {
    if (!L.njobs) return;
    hipLaunchKernelGGL(k_scatter_meta, dim3((L.njobs + 255) / 256), dim3(256), 0, L.stream, L.jobs, L.njobs, in);
}

void launch_msb_plane(const Launch &L, const uint64_t *off, uint8_t *out, uint64_t max_bytes) {
    if (!L.njobs || !max_bytes) return;
    hipLaunchKernelGGL(k_msb_plane, dim3((unsigned)((max_bytes + 255) / 256), (unsigned)L.njobs), dim3(256), 0,
                       L.stream, L.jobs, off, out);
}

}  // namespace rdhei

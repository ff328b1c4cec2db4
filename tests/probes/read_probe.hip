// Counter calibration probe: reads a buffer of known size once, either with
// wave-uniform (scalar) loads of 64 bytes -- the way the traversal reads
// records and particle runs -- or with per-lane 16-byte vector loads, so that
// a hardware counter of bytes fetched from memory (rocprofv3 FETCH_SIZE) can
// be scaled to bytes for both kinds of load.  Each workgroup (one wavefront)
// reads its own contiguous slice; results go out with per-lane vector stores.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

// slice of n16 uint4 per workgroup, n16 a multiple of 4
__global__ __launch_bounds__(64) void k_scalar_read(const uint4 *__restrict__ src, uint64_t n16,
                                                    uint32_t *__restrict__ out) {
    const uint4 *__restrict__ p = src + (uint64_t)blockIdx.x * n16;
    uint32_t acc = 0;
    for (uint64_t i = 0; i < n16; i += 4) {
        const uint4 a = p[i], b = p[i + 1], c = p[i + 2], d = p[i + 3];
        acc += (a.x ^ a.y ^ a.z ^ a.w) + (b.x ^ b.y ^ b.z ^ b.w) + (c.x ^ c.y ^ c.z ^ c.w) + (d.x ^ d.y ^ d.z ^ d.w);
    }
    out[(uint64_t)blockIdx.x * 64 + threadIdx.x] = acc + threadIdx.x;
}

__global__ __launch_bounds__(64) void k_vector_read(const uint4 *__restrict__ src, uint64_t n16,
                                                    uint32_t *__restrict__ out) {
    const uint4 *__restrict__ p = src + (uint64_t)blockIdx.x * n16;
    uint32_t acc = 0;
    for (uint64_t i = threadIdx.x; i < n16; i += 64) {
        const uint4 a = p[i];
        acc += a.x ^ a.y ^ a.z ^ a.w;
    }
    out[(uint64_t)blockIdx.x * 64 + threadIdx.x] = acc;
}

}  // namespace

extern "C" {

// Reads bytes (a multiple of 64 * blocks) of src with `blocks` workgroups;
// out holds 64 * blocks uint32.  kind 0: scalar loads, 1: vector loads.
__attribute__((visibility("default"))) int read_probe(int kind, const void *src, uint64_t bytes, uint32_t blocks,
                                                      uint32_t *out) {
    if (!src || !out || blocks == 0 || bytes % (64ull * blocks) != 0) return -1;
    const uint64_t n16 = bytes / 16 / blocks;
    if (kind == 0)
        hipLaunchKernelGGL(k_scalar_read, dim3(blocks), dim3(64), 0, 0, (const uint4 *)src, n16, out);
    else
        hipLaunchKernelGGL(k_vector_read, dim3(blocks), dim3(64), 0, 0, (const uint4 *)src, n16, out);
    return hipDeviceSynchronize() == hipSuccess ? 0 : -2;
}

}  // extern "C"

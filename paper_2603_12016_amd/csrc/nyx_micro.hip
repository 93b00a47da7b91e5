// nyx_micro.hip -- measurement kernels used next to the GLCM path: the
// machine ceilings its roofline is read against.
//
//   nyx_micro_copy        plain device copy of a byte range (16-byte vector
//                         loads and stores).  Its hardware counters calibrate
//                         FETCH_SIZE / WRITE_SIZE, and its rate is the
//                         measured copy bandwidth.
//   nyx_micro_read        read-only stream with a per-block reduction: the
//                         measured read bandwidth.
//   nyx_micro_lds_atomic  conflict-free LDS atomic adds (ds_add_u32), every
//                         lane of a wave on its own bank: the chip-wide LDS
//                         atomic rate the accumulation is compared with.
//
// Not part of the feature path; linked into its own library.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

__global__ __launch_bounds__(256) void k_copy(const uint4 *__restrict__ src, uint4 *__restrict__ dst, uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

__global__ __launch_bounds__(256) void k_read(const uint4 *__restrict__ src, uint64_t n, uint32_t *sink) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint32_t acc = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint4 v = src[i];
        acc ^= v.x ^ v.y ^ v.z ^ v.w;
    }
    __shared__ uint32_t red[256];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (uint32_t s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] ^= red[threadIdx.x + s];
        __syncthreads();
    }
    // one word per block: keeps the loads live
    if (threadIdx.x == 0) sink[blockIdx.x] = red[0];
}

// Each lane adds to word (lane + 32 * j) of its wave's slice: lanes 0..31
// and 32..63 hit 32 distinct banks in each half-wave step.  Four independent
// streams per lane keep several atomics in flight.
__global__ __launch_bounds__(256) void k_lds_atomic(uint32_t iters, uint32_t *out) {
    __shared__ uint32_t cnt[256 * 4];
    for (uint32_t i = threadIdx.x; i < 256u * 4u; i += blockDim.x) cnt[i] = 0u;
    __syncthreads();
    const uint32_t base = (threadIdx.x & ~63u) * 4u + (threadIdx.x & 63u);
    for (uint32_t it = 0; it < iters; ++it) {
        __hip_atomic_fetch_add(&cnt[base], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        __hip_atomic_fetch_add(&cnt[base + 64u], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        __hip_atomic_fetch_add(&cnt[base + 128u], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        __hip_atomic_fetch_add(&cnt[base + 192u], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    __syncthreads();
    uint32_t s = 0;
    for (uint32_t i = threadIdx.x; i < 256u * 4u; i += blockDim.x) s += cnt[i];
    __shared__ uint32_t red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (uint32_t i = 0; i < blockDim.x; ++i) t += red[i];
        out[blockIdx.x] = t;   // = 4 * iters * blockDim.x when every add landed
    }
}

uint32_t grid_for(uint64_t n) {
    uint64_t g = (n + 255u) / 256u;
    if (g > 256u * 64u) g = 256u * 64u;
    return g ? (uint32_t)g : 1u;
}

}  // namespace

extern "C" {

// dst and src: device pointers, 16-byte aligned; bytes a multiple of 16.
int nyx_micro_copy(const void *src, void *dst, uint64_t bytes, void *stream) {
    if (!src || !dst || bytes % 16u || (uintptr_t)src % 16u || (uintptr_t)dst % 16u) return 1;
    const uint64_t n = bytes / 16u;
    hipLaunchKernelGGL(k_copy, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream,
                       reinterpret_cast<const uint4 *>(src), reinterpret_cast<uint4 *>(dst), n);
    return hipGetLastError() == hipSuccess ? 0 : 2;
}

// sink: device buffer of at least 16384 u32.
int nyx_micro_read(const void *src, uint64_t bytes, uint32_t *sink, void *stream) {
    if (!src || !sink || bytes % 16u || (uintptr_t)src % 16u) return 1;
    const uint64_t n = bytes / 16u;
    hipLaunchKernelGGL(k_read, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream,
                       reinterpret_cast<const uint4 *>(src), n, sink);
    return hipGetLastError() == hipSuccess ? 0 : 2;
}

// out: device buffer of `blocks` u32; each block performs 4 * iters * 256 adds.
int nyx_micro_lds_atomic(uint32_t blocks, uint32_t iters, uint32_t *out, void *stream) {
    if (!out || blocks == 0) return 1;
    hipLaunchKernelGGL(k_lds_atomic, dim3(blocks), dim3(256), 0, (hipStream_t)stream, iters, out);
    return hipGetLastError() == hipSuccess ? 0 : 2;
}

}  // extern "C"

// Random-access and atomic ceilings of the device: the rates the hash-table
// stages are compared with. Counting is bound by the probes and counter
// updates of Alg. 1 rather than by streaming (Sec. 3.3.1 measures the probe
// behaviour of the GPU table), so the measurement reports inserts per second
// next to what the hardware sustains for the same access kinds:
//   LDS_CAS   64-bit compare-and-swap with return at random slots of an LDS
//             table (the claim step of an LDS table insert);
//   LDS_ADD   32-bit add without return at random LDS words (the count step);
//   HBM_ADD   32-bit device-scope add without return at random 64-byte lines;
//   HBM_CAS   64-bit device-scope compare-and-swap with return at random lines
//             (the claim step of an HBM table insert);
//   HBM_LOAD  64-bit device-coherent load from random lines;
//   ONE_ADDR  device-scope add with return on a single word, one per wave
//             (a shared work-queue cursor).
// Positions come from a per-thread xorshift generator, so nothing here is
// data-dependent and every launch stays inside its buffers.
#include "../../include/gerbil.h"
#include "common.h"
#include "internal.h"

namespace gerbil {
namespace {

constexpr uint32_t kCeilBlock = 1024;
constexpr uint32_t kLdsCasSlots = 16384;   // 128 KB of 64-bit slots
constexpr uint32_t kLdsAddWords = 32768;   // 128 KB of 32-bit words

__device__ __forceinline__ uint32_t xorshift32(uint32_t& x) {
    x ^= x << 13;
    x ^= x >> 17;
    x ^= x << 5;
    return x;
}

__device__ __forceinline__ uint32_t thread_seed() {
    const uint32_t g = blockIdx.x * kCeilBlock + threadIdx.x;
    return ((g * 2654435761u) ^ 0x9E3779B9u ^ (g >> 7)) | 1u;
}

__global__ void __launch_bounds__(kCeilBlock) k_ceil_lds_cas(uint32_t iters, uint64_t* sink) {
    extern __shared__ __align__(16) uint8_t lds_raw[];
    uint64_t* t = (uint64_t*)lds_raw;
    for (uint32_t i = threadIdx.x; i < kLdsCasSlots; i += kCeilBlock) t[i] = GERBIL_EMPTY;
    __syncthreads();
    uint32_t x = thread_seed();
    uint64_t acc = 0;
    for (uint32_t i = 0; i < iters; i++) {
        const uint32_t sl = xorshift32(x) & (kLdsCasSlots - 1);
        uint64_t exp = GERBIL_EMPTY;
        __hip_atomic_compare_exchange_strong(t + sl, &exp, (uint64_t)x, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_WORKGROUP);
        acc += exp;
    }
    sink[blockIdx.x * kCeilBlock + threadIdx.x] = acc;
}

__global__ void __launch_bounds__(kCeilBlock) k_ceil_lds_add(uint32_t iters, uint64_t* sink) {
    extern __shared__ __align__(16) uint8_t lds_raw[];
    uint32_t* t = (uint32_t*)lds_raw;
    for (uint32_t i = threadIdx.x; i < kLdsAddWords; i += kCeilBlock) t[i] = 0;
    __syncthreads();
    uint32_t x = thread_seed();
    for (uint32_t i = 0; i < iters; i++)
        __hip_atomic_fetch_add(t + (xorshift32(x) & (kLdsAddWords - 1)), 1u, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
    __syncthreads();
    uint64_t acc = 0;
    for (uint32_t i = threadIdx.x; i < kLdsAddWords; i += kCeilBlock) acc += t[i];
    sink[blockIdx.x * kCeilBlock + threadIdx.x] = acc;
}

__global__ void __launch_bounds__(kCeilBlock) k_ceil_hbm(uint32_t kind, uint8_t* buf, uint64_t n_lines,
                                                         uint32_t iters, uint64_t* sink) {
    uint32_t x = thread_seed();
    uint64_t acc = 0;
    for (uint32_t i = 0; i < iters; i++) {
        // two draws give 64 random bits, reduced onto the lines
        const uint64_t r = ((uint64_t)xorshift32(x) << 32) | xorshift32(x);
        const uint64_t line = (uint64_t)(((unsigned __int128)r * n_lines) >> 64);
        uint8_t* p = buf + line * 64;
        if (kind == GERBIL_CEIL_HBM_ADD) {
            __hip_atomic_fetch_add((uint32_t*)p, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else if (kind == GERBIL_CEIL_HBM_CAS) {
            acc += cas_dev((uint64_t*)p, (uint64_t)i, r);
        } else {
            acc += ld_dev((const uint64_t*)p);
        }
    }
    sink[blockIdx.x * kCeilBlock + threadIdx.x] = acc;
}

__global__ void __launch_bounds__(kCeilBlock) k_ceil_one_addr(uint64_t* word, uint32_t iters, uint64_t* sink) {
    uint64_t acc = 0;
    if (__lane_id() == 0)
        for (uint32_t i = 0; i < iters; i++) acc += add_dev(word, 1ull);
    sink[blockIdx.x * kCeilBlock + threadIdx.x] = acc;
}

}  // namespace
}  // namespace gerbil

using namespace gerbil;

extern "C" int32_t gerbil_ceiling(uint32_t kind, void* buf, uint64_t buf_bytes, uint32_t grid, uint32_t iters,
                                  uint64_t* sink, hipStream_t stream) {
    if (!sink || grid == 0 || grid > (1u << 20) || iters == 0) return GERBIL_EINVAL;
    const bool hbm = kind == GERBIL_CEIL_HBM_ADD || kind == GERBIL_CEIL_HBM_CAS || kind == GERBIL_CEIL_HBM_LOAD ||
                     kind == GERBIL_CEIL_ONE_ADDR;
    if (kind > GERBIL_CEIL_ONE_ADDR) return GERBIL_EINVAL;
    if (hbm && (!buf || buf_bytes < 64 || (buf_bytes & 63) || ((uintptr_t)buf & 63))) return GERBIL_EINVAL;
    hipError_t e = hipSuccess;
    switch (kind) {
        case GERBIL_CEIL_LDS_CAS:
            // the attribute is set on every call (no process-wide flag to race on)
            e = hipFuncSetAttribute((const void*)k_ceil_lds_cas, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    8 * kLdsCasSlots);
            if (e == hipSuccess)
                hipLaunchKernelGGL(k_ceil_lds_cas, dim3(grid), dim3(kCeilBlock), 8 * kLdsCasSlots, stream, iters, sink);
            break;
        case GERBIL_CEIL_LDS_ADD:
            e = hipFuncSetAttribute((const void*)k_ceil_lds_add, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    4 * kLdsAddWords);
            if (e == hipSuccess)
                hipLaunchKernelGGL(k_ceil_lds_add, dim3(grid), dim3(kCeilBlock), 4 * kLdsAddWords, stream, iters, sink);
            break;
        case GERBIL_CEIL_ONE_ADDR:
            hipLaunchKernelGGL(k_ceil_one_addr, dim3(grid), dim3(kCeilBlock), 0, stream, (uint64_t*)buf, iters, sink);
            break;
        default:
            hipLaunchKernelGGL(k_ceil_hbm, dim3(grid), dim3(kCeilBlock), 0, stream, kind, (uint8_t*)buf,
                               buf_bytes / 64, iters, sink);
            break;
    }
    if (e == hipSuccess) e = hipGetLastError();
    return e == hipSuccess ? GERBIL_OK : GERBIL_EDEVICE;
}

// HyperLogLog sketches of the distinct k-mers of every bin, from the k-mer
// occurrences of its super-mers: the alternative the table-size estimate
// of Sec. 3.4.1 is compared with. The work items are chunks of kHllChunk
// super-mers of one bin, so a large bin is spread over many workgroups. A
// workgroup keeps the 2^p registers of its item's bin in LDS; each thread
// walks one super-mer, rolling its window one base at a time, hashes every
// canonical key and raises register (top p bits of the hash) to the rank of
// the first set bit of the remaining bits. The item's registers are then
// merged into the bin's with atomic maxima (the registers start at zero), so
// the result does not depend on how the bin was split.
#include "../../include/gerbil.h"
#include "common.h"
#include "internal.h"

namespace gerbil {
namespace {

constexpr uint32_t kHllBlock = 256;
constexpr uint64_t kHllSeed = 0x5bd1e9955bd1e995ull;   // not the table seed: an independent hash

// Advance a window by one base b: fw drops its first base and appends b; rc
// drops its last base and takes the complement of b in front. The last word
// holds r bases, right-aligned.
template <int W>
__device__ __forceinline__ void roll_kmer(uint64_t (&fw)[W], uint64_t (&rc)[W], uint32_t r, uint64_t b) {
#pragma unroll
    for (int i = 0; i + 1 < W; i++) {
        const uint32_t top = i + 2 < W ? 62u : 2u * r - 2u;   // the first base of word i + 1
        fw[i] = (fw[i] << 2) | ((fw[i + 1] >> top) & 3ull);
    }
    const uint64_t lmask = r == 32 ? ~0ull : ((1ull << (2 * r)) - 1ull);
    fw[W - 1] = ((fw[W - 1] << 2) | b) & lmask;
#pragma unroll
    for (int i = W - 1; i >= 1; i--) {
        const uint32_t top = i == W - 1 ? 2u * r - 2u : 62u;
        rc[i] = (rc[i] >> 2) | ((rc[i - 1] & 3ull) << top);
    }
    rc[0] = (rc[0] >> 2) | ((3ull - b) << (W == 1 ? 2u * r - 2u : 62u));
}

constexpr uint32_t kHllChunk = 2048;   // super-mers per work item

template <int W>
__global__ void __launch_bounds__(kHllBlock) k_hll(const uint64_t* __restrict__ packed, uint64_t n_bytes,
                                                   const uint64_t* __restrict__ desc,
                                                   const uint64_t* __restrict__ bin_off, uint32_t n_bins, uint32_t k,
                                                   uint32_t canonical, uint32_t p, uint32_t* __restrict__ regs) {
    extern __shared__ uint32_t lds[];
    const uint32_t m = 1u << p, tid = threadIdx.x;
    uint32_t* R = lds;              // [m] registers of the current item's bin
    uint32_t* pre = lds + m;        // [n_bins + 1] first work item of every bin
    uint32_t* part = pre + n_bins + 1;   // [kHllBlock] scan scratch
    // work items per bin and their prefix: thread t takes bins [t*per, (t+1)*per)
    const uint32_t per = (n_bins + kHllBlock - 1) / kHllBlock;
    uint32_t sum = 0;
    for (uint32_t e = 0; e < per; e++) {
        const uint32_t b = tid * per + e;
        if (b < n_bins) sum += (uint32_t)((bin_off[b + 1] - bin_off[b] + kHllChunk - 1) / kHllChunk);
    }
    part[tid] = sum;
    __syncthreads();
    for (uint32_t off = 1; off < kHllBlock; off <<= 1) {
        const uint32_t y = tid >= off ? part[tid - off] : 0u;
        __syncthreads();
        part[tid] += y;
        __syncthreads();
    }
    uint32_t run = tid ? part[tid - 1] : 0u;
    for (uint32_t e = 0; e < per; e++) {
        const uint32_t b = tid * per + e;
        if (b < n_bins) {
            pre[b] = run;
            run += (uint32_t)((bin_off[b + 1] - bin_off[b] + kHllChunk - 1) / kHllChunk);
        }
    }
    if (tid == kHllBlock - 1) pre[n_bins] = part[kHllBlock - 1];
    __syncthreads();
    const uint32_t total = pre[n_bins];
    const uint32_t r = k - 32u * (W - 1);
    for (uint32_t item = blockIdx.x; item < total; item += gridDim.x) {
        uint32_t lo = 0, hi = n_bins;   // the bin of the item: last b with pre[b] <= item
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (pre[mid] <= item) lo = mid; else hi = mid;
        }
        const uint32_t b = lo;
        const uint64_t d0 = bin_off[b] + (uint64_t)(item - pre[b]) * kHllChunk;
        const uint64_t d1 = d0 + kHllChunk < bin_off[b + 1] ? d0 + kHllChunk : bin_off[b + 1];
        for (uint32_t j = tid; j < m; j += kHllBlock) R[j] = 0;
        __syncthreads();
        for (uint64_t d = d0 + tid; d < d1; d += kHllBlock) {
            const uint64_t dd = desc[d];
            const int64_t start = (int64_t)(dd >> 24);
            const uint32_t nk = (uint32_t)(dd & 0xFFFFFFu);
            if (nk == 0 || start < 0 || (uint64_t)start + nk - 1 + k > n_bytes) continue;   // never read out of range
            uint64_t fw[W], rc[W];
            extract_kmer<W>(packed, start, k, fw, rc);
            for (uint32_t t = 0; t < nk; t++) {
                if (t) {   // the next window: one more base from the packed stream
                    const uint64_t pos = (uint64_t)start + t + k - 1;
                    roll_kmer<W>(fw, rc, r, (packed[pos >> 5] >> (62 - 2 * (pos & 31))) & 3ull);
                }
                uint64_t key[W];
                canonical_of<W>(fw, rc, key, canonical);
                const uint64_t h = key_hash<W>(key, kHllSeed);
                const uint32_t idx = (uint32_t)(h >> (64 - p));
                const uint32_t rho = (uint32_t)__clzll((h << p) | (1ull << (p - 1))) + 1u;
                atomicMax(&R[idx], rho);
            }
        }
        __syncthreads();
        for (uint32_t j = tid; j < m; j += kHllBlock)
            if (R[j]) atomicMax(&regs[((uint64_t)b << p) + j], R[j]);
        __syncthreads();   // R is cleared for the next item
    }
}

template <int W>
hipError_t hll_w(const uint64_t* packed, uint64_t n_bytes, const uint64_t* desc, const uint64_t* bin_off,
                 uint32_t n_bins, uint32_t k, uint32_t canonical, uint32_t p, uint32_t* regs, hipStream_t s) {
    const size_t lds = ((size_t)1 << p) * 4 + ((size_t)n_bins + 1) * 4 + (size_t)kHllBlock * 4;
    if (hipFuncSetAttribute((const void*)k_hll<W>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return hipErrorInvalidValue;
    hipError_t e = launch_fill_u32(regs, (uint64_t)n_bins << p, 0u, s);   // merged by atomic maxima
    if (e != hipSuccess) return e;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        cus = 1;
    const uint32_t grid = 4u * (uint32_t)cus;   // every item is taken by some workgroup (grid stride)
    hipLaunchKernelGGL(k_hll<W>, dim3(grid), dim3(kHllBlock), lds, s, packed, n_bytes, desc, bin_off, n_bins, k,
                       canonical, p, regs);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_hll(const uint64_t* packed, uint64_t n_bytes, const uint64_t* desc, const uint64_t* bin_off,
                      uint32_t n_bins, uint32_t k, uint32_t canonical, uint32_t p, uint32_t* regs, hipStream_t s) {
    switch ((k + 31) / 32) {
        case 1: return hll_w<1>(packed, n_bytes, desc, bin_off, n_bins, k, canonical, p, regs, s);
        case 2: return hll_w<2>(packed, n_bytes, desc, bin_off, n_bins, k, canonical, p, regs, s);
        case 3: return hll_w<3>(packed, n_bytes, desc, bin_off, n_bins, k, canonical, p, regs, s);
        case 4: return hll_w<4>(packed, n_bytes, desc, bin_off, n_bins, k, canonical, p, regs, s);
        case 5: return hll_w<5>(packed, n_bytes, desc, bin_off, n_bins, k, canonical, p, regs, s);
        case 6: return hll_w<6>(packed, n_bytes, desc, bin_off, n_bins, k, canonical, p, regs, s);
        case 7: return hll_w<7>(packed, n_bytes, desc, bin_off, n_bins, k, canonical, p, regs, s);
        case 8: return hll_w<8>(packed, n_bytes, desc, bin_off, n_bins, k, canonical, p, regs, s);
        case 9: return hll_w<9>(packed, n_bytes, desc, bin_off, n_bins, k, canonical, p, regs, s);
        case 10: return hll_w<10>(packed, n_bytes, desc, bin_off, n_bins, k, canonical, p, regs, s);
        case 11: return hll_w<11>(packed, n_bytes, desc, bin_off, n_bins, k, canonical, p, regs, s);
        case 12: return hll_w<12>(packed, n_bytes, desc, bin_off, n_bins, k, canonical, p, regs, s);
        case 13: return hll_w<13>(packed, n_bytes, desc, bin_off, n_bins, k, canonical, p, regs, s);
        case 14: return hll_w<14>(packed, n_bytes, desc, bin_off, n_bins, k, canonical, p, regs, s);
        case 15: return hll_w<15>(packed, n_bytes, desc, bin_off, n_bins, k, canonical, p, regs, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace gerbil

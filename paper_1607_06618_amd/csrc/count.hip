// Plain schedule of the counting step: one launch sequence per bin (insert
// kernel, then the dump of its table), bins in order, one table reused; plus
// the emergency-area sort-and-count that runs after all bins. The table logic
// (Alg. 1, publication of multi-word keys, dump) is in table.h.
#include "table.h"

namespace gerbil {

constexpr uint32_t kMaxBlock = 1024;

// Insert the k-mers of descriptors [d0, d1) of one bin. A block loads one
// descriptor per thread, scans their k-mer counts, then every lane takes one
// k-mer at a time (so super-mers of different lengths balance within a block).
template <int W>
__global__ void __launch_bounds__(kMaxBlock) k_count_bin(CountArgs a, Table t, uint32_t nb, uint64_t d0, uint64_t d1) {
    __shared__ int64_t sstart[kMaxBlock];
    __shared__ uint32_t spre[kMaxBlock];
    __shared__ uint32_t wsum[17];
    const uint32_t tid = threadIdx.x, B = blockDim.x;
    for (uint64_t c0 = d0 + (uint64_t)blockIdx.x * B; c0 < d1; c0 += (uint64_t)gridDim.x * B) {
        uint64_t i = c0 + tid;
        uint32_t n = 0;
        int64_t st = 0;
        if (i < d1) {
            uint64_t d = a.desc[i];
            st = (int64_t)(d >> 24);
            n = (uint32_t)(d & 0xFFFFFFu);
        }
        uint32_t total;
        uint32_t pre = block_excl_scan(n, wsum, total);
        sstart[tid] = st;
        spre[tid] = pre;
        __syncthreads();
        for (uint32_t idx = tid; idx < total; idx += B) {
            // last descriptor whose prefix is <= idx
            uint32_t lo = 0, hi = B;
            while (hi - lo > 1) {
                uint32_t mid = (lo + hi) >> 1;
                if (spre[mid] <= idx) lo = mid; else hi = mid;
            }
            count_position<W>(a, t, nb, sstart[lo] + (int64_t)(idx - spre[lo]));
        }
        __syncthreads();
    }
}

// Dump a table: emit pairs with count >= threshold, histogram every count,
// and reset the slot for the next bin.
template <int W>
__global__ void __launch_bounds__(256) k_compact(CountArgs a, Table t, uint64_t n_slots) {
    __shared__ uint32_t lh[kLdsHist];
    const uint32_t tid = threadIdx.x;
    for (uint32_t b = tid; b < kLdsHist; b += blockDim.x) lh[b] = 0;
    __syncthreads();
    uint32_t wmax = 0;
    for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x; base < n_slots; base += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t slot = base + tid;
        compact_slot<W>(a, t, slot, slot < n_slots, lh, wmax);
    }
    flush_max(a.max_count, wmax);
    __syncthreads();
    for (uint32_t b = tid; b < kLdsHist; b += blockDim.x)
        if (lh[b]) add_dev(&a.hist[b], (uint64_t)lh[b]);
}

// ------------------------------------------------------ emergency area
template <int W>
__device__ __forceinline__ bool key_less(const uint64_t* x, const uint64_t* y) {
#pragma unroll
    for (int i = 0; i < W; i++)
        if (x[i] != y[i]) return x[i] < y[i];
    return false;
}
template <int W>
__device__ __forceinline__ bool key_eq(const uint64_t* x, const uint64_t* y) {
    bool e = true;
#pragma unroll
    for (int i = 0; i < W; i++) e &= x[i] == y[i];
    return e;
}

// Sort-and-count of the emergency area (Sec. 3.4.3). One workgroup: bitonic
// sort of the keys in place (padded to a power of two with all-ones keys,
// which no canonical key equals), then run-length counting. This path is
// expected to be empty at sensible load factors; it exists for exactness.
template <int W>
__global__ void __launch_bounds__(1024) k_overflow(CountArgs a) {
    const uint32_t tid = threadIdx.x, B = blockDim.x;
    uint64_t n = ld_dev(a.n_ovf);
    if (n > a.ovf_cap) n = a.ovf_cap;
    if (n == 0) return;
    uint64_t N = 1;
    while (N < n) N <<= 1;   // ovf capacity is a power of two, so N <= capacity
    uint64_t* K = a.ovf_keys;
    for (uint64_t i = n + tid; i < N; i += B)
        for (int w = 0; w < W; w++) K[i * W + w] = ~0ull;
    __syncthreads();
    for (uint64_t size = 2; size <= N; size <<= 1) {
        for (uint64_t stride = size >> 1; stride > 0; stride >>= 1) {
            for (uint64_t i = tid; i < N / 2; i += B) {
                uint64_t lo = 2 * stride * (i / stride) + (i % stride), hi = lo + stride;
                bool asc = (lo & size) == 0;
                uint64_t x[W], y[W];
#pragma unroll
                for (int w = 0; w < W; w++) { x[w] = K[lo * W + w]; y[w] = K[hi * W + w]; }
                bool swap = asc ? key_less<W>(y, x) : key_less<W>(x, y);
                if (swap) {
#pragma unroll
                    for (int w = 0; w < W; w++) { K[lo * W + w] = y[w]; K[hi * W + w] = x[w]; }
                }
            }
            __syncthreads();
        }
    }
    uint32_t wmax = 0;
    for (uint64_t base = 0; base < n; base += B) {
        uint64_t i = base + tid;
        bool is_start = i < n && (i == 0 || !key_eq<W>(K + i * W, K + (i - 1) * W));
        uint64_t c = 0;
        if (is_start) {
            uint64_t j = i + 1;
            while (j < n && key_eq<W>(K + j * W, K + i * W)) j++;
            c = j - i;
            add_dev(&a.hist[c < kHistInternal - 1 ? c : kHistInternal - 1], 1ull);
            if (c >= 0xFFFFFFFFull) set_status(a.status, ST_COUNT_SAT);
            uint32_t c32 = c > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)c;
            wmax = c32 > wmax ? c32 : wmax;
        }
        bool emit = is_start && c >= a.threshold;
        uint64_t pos = wave_reserve(a.n_out, emit);
        if (emit) {
            if (pos < a.cap) {
#pragma unroll
                for (int w = 0; w < W; w++) a.out_keys[pos * W + w] = K[i * W + w];
                a.out_counts[pos] = (uint32_t)c;
            } else {
                set_status(a.status, ST_OUT_CAP);
            }
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        uint32_t y = __shfl_xor(wmax, off);
        wmax = y > wmax ? y : wmax;
    }
    if (__lane_id() == 0 && wmax)
        __hip_atomic_fetch_max(a.max_count, (uint64_t)wmax, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------------ launchers
template <int W>
static hipError_t count_bin_w(const CountArgs& a, const Table& t, uint32_t nb, uint64_t d0, uint64_t d1,
                              uint32_t block, hipStream_t s) {
    uint64_t blocks = (d1 - d0 + block - 1) / block;
    uint32_t g = (uint32_t)(blocks < 65535 ? blocks : 65535);
    hipLaunchKernelGGL(k_count_bin<W>, dim3(g), dim3(block), 0, s, a, t, nb, d0, d1);
    return hipGetLastError();
}
template <int W>
static hipError_t compact_w(const CountArgs& a, const Table& t, uint32_t nb, hipStream_t s) {
    uint64_t n_slots = (uint64_t)nb * kBucket;
    uint64_t blocks = (n_slots + 255) / 256;
    uint32_t g = (uint32_t)(blocks < 8192 ? blocks : 8192);
    hipLaunchKernelGGL(k_compact<W>, dim3(g), dim3(256), 0, s, a, t, n_slots);
    return hipGetLastError();
}
template <int W>
static hipError_t overflow_w(const CountArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_overflow<W>, dim3(1), dim3(1024), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_count_bin(const CountArgs& a, const Table& t, uint32_t nb, uint64_t d0, uint64_t d1,
                            uint32_t block, hipStream_t s) {
    switch (a.W) {
        case 1: return count_bin_w<1>(a, t, nb, d0, d1, block, s);
        case 2: return count_bin_w<2>(a, t, nb, d0, d1, block, s);
        case 3: return count_bin_w<3>(a, t, nb, d0, d1, block, s);
        case 4: return count_bin_w<4>(a, t, nb, d0, d1, block, s);
        case 5: return count_bin_w<5>(a, t, nb, d0, d1, block, s);
        case 6: return count_bin_w<6>(a, t, nb, d0, d1, block, s);
        case 7: return count_bin_w<7>(a, t, nb, d0, d1, block, s);
        case 8: return count_bin_w<8>(a, t, nb, d0, d1, block, s);
        case 9: return count_bin_w<9>(a, t, nb, d0, d1, block, s);
        case 10: return count_bin_w<10>(a, t, nb, d0, d1, block, s);
        case 11: return count_bin_w<11>(a, t, nb, d0, d1, block, s);
        case 12: return count_bin_w<12>(a, t, nb, d0, d1, block, s);
        case 13: return count_bin_w<13>(a, t, nb, d0, d1, block, s);
        case 14: return count_bin_w<14>(a, t, nb, d0, d1, block, s);
        case 15: return count_bin_w<15>(a, t, nb, d0, d1, block, s);
    }
    return hipErrorInvalidValue;
}
hipError_t launch_compact(const CountArgs& a, const Table& t, uint32_t nb, hipStream_t s) {
    switch (a.W) {
        case 1: return compact_w<1>(a, t, nb, s);
        case 2: return compact_w<2>(a, t, nb, s);
        case 3: return compact_w<3>(a, t, nb, s);
        case 4: return compact_w<4>(a, t, nb, s);
        case 5: return compact_w<5>(a, t, nb, s);
        case 6: return compact_w<6>(a, t, nb, s);
        case 7: return compact_w<7>(a, t, nb, s);
        case 8: return compact_w<8>(a, t, nb, s);
        case 9: return compact_w<9>(a, t, nb, s);
        case 10: return compact_w<10>(a, t, nb, s);
        case 11: return compact_w<11>(a, t, nb, s);
        case 12: return compact_w<12>(a, t, nb, s);
        case 13: return compact_w<13>(a, t, nb, s);
        case 14: return compact_w<14>(a, t, nb, s);
        case 15: return compact_w<15>(a, t, nb, s);
    }
    return hipErrorInvalidValue;
}
hipError_t launch_overflow(const CountArgs& a, hipStream_t s) {
    switch (a.W) {
        case 1: return overflow_w<1>(a, s);
        case 2: return overflow_w<2>(a, s);
        case 3: return overflow_w<3>(a, s);
        case 4: return overflow_w<4>(a, s);
        case 5: return overflow_w<5>(a, s);
        case 6: return overflow_w<6>(a, s);
        case 7: return overflow_w<7>(a, s);
        case 8: return overflow_w<8>(a, s);
        case 9: return overflow_w<9>(a, s);
        case 10: return overflow_w<10>(a, s);
        case 11: return overflow_w<11>(a, s);
        case 12: return overflow_w<12>(a, s);
        case 13: return overflow_w<13>(a, s);
        case 14: return overflow_w<14>(a, s);
        case 15: return overflow_w<15>(a, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace gerbil

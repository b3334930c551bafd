// Plain schedule of the counting step: one launch sequence per bin (insert
// kernel, then the dump of its table), bins in order, one table reused; plus
// the counting of the emergency area that runs after all bins. The table logic
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
__device__ __forceinline__ bool key_eq(const uint64_t* x, const uint64_t* y) {
    bool e = true;
#pragma unroll
    for (int i = 0; i < W; i++) e &= x[i] == y[i];
    return e;
}

// Keys that did not fit in a table (theta probes failed, a sampled run
// overflowed, or the first word is the empty-slot marker) were appended to the
// emergency area (Sec. 3.4.3, where the paper sorts and compresses them). Here
// they are counted in an open-addressing table in HBM with at least twice as
// many slots as the area holds keys, so linear probing always ends at the key
// or at a free slot: exact, with no probe limit. A slot's state word holds the
// area index + 1 of the first occurrence that claimed it (by CAS on zero);
// another occurrence compares its key with that occurrence in the area, which
// no kernel writes any more, so nothing has to be published; every occurrence
// then adds one to its slot's count. Many workgroups insert; the table is then
// dumped (threshold, histogram). The table has next_pow2(2 n) slots for n keys,
// read on the device, so an empty area costs three launches that return at once.
constexpr uint32_t kOvfBlock = 256;

__device__ __forceinline__ uint64_t ovf_n(const CountArgs& a) {
    const uint64_t n = ld_dev(a.n_ovf);
    return n < a.ovf_cap ? n : a.ovf_cap;
}
__device__ __forceinline__ uint64_t ovf_slots(uint64_t n) {
    uint64_t t = 2;
    while (t < 2 * n) t <<= 1;
    return t;
}

__global__ void __launch_bounds__(kOvfBlock) k_ovf_clear(CountArgs a) {
    const uint64_t n = ovf_n(a);
    if (n == 0) return;
    const uint64_t T = ovf_slots(n);
    for (uint64_t i = (uint64_t)blockIdx.x * kOvfBlock + threadIdx.x; i < T; i += (uint64_t)gridDim.x * kOvfBlock) {
        a.ovf_state[i] = 0u;
        a.ovf_tcnt[i] = 0u;
    }
}

template <int W>
__global__ void __launch_bounds__(kOvfBlock) k_ovf_insert(CountArgs a) {
    const uint64_t n = ovf_n(a);
    if (n == 0) return;
    const uint64_t T = ovf_slots(n), mask = T - 1;
    for (uint64_t i = (uint64_t)blockIdx.x * kOvfBlock + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kOvfBlock) {
        const uint64_t* key = a.ovf_keys + i * W;
        uint64_t kw[W];
#pragma unroll
        for (int w = 0; w < W; w++) kw[w] = key[w];
        uint64_t s = key_hash<W>(kw, a.seed ^ 0x9E3779B97F4A7C15ull) & mask;
        for (uint64_t probe = 0; probe < T; probe++, s = (s + 1) & mask) {
            const uint32_t found = cas_dev(&a.ovf_state[s], 0u, (uint32_t)(i + 1));
            if (found == 0u || key_eq<W>(a.ovf_keys + (uint64_t)(found - 1) * W, kw)) {
                add_dev(&a.ovf_tcnt[s], 1u);
                break;
            }
        }
    }
}

template <int W>
__global__ void __launch_bounds__(kOvfBlock) k_ovf_dump(CountArgs a) {
    __shared__ uint32_t lh[kLdsHist];
    const uint32_t tid = threadIdx.x;
    const uint64_t n = ovf_n(a);
    if (n == 0) return;
    const uint64_t T = ovf_slots(n);
    for (uint32_t b = tid; b < kLdsHist; b += kOvfBlock) lh[b] = 0;
    __syncthreads();
    uint32_t wmax = 0;
    // every lane runs the same number of iterations (wave_reserve needs the whole wave)
    for (uint64_t base = (uint64_t)blockIdx.x * kOvfBlock; base < T; base += (uint64_t)gridDim.x * kOvfBlock) {
        const uint64_t s = base + tid;
        const uint32_t rep = s < T ? a.ovf_state[s] : 0u;
        const uint32_t c = rep ? a.ovf_tcnt[s] : 0u;
        if (c) {
            if (c < kLdsHist) atomicAdd(&lh[c], 1u);
            else add_dev(&a.hist[c < kHistInternal - 1 ? c : kHistInternal - 1], 1ull);
            wmax = c > wmax ? c : wmax;
        }
        const bool emit = c && c >= a.threshold;
        const uint64_t pos = wave_reserve(a.n_out, emit);
        if (emit) {
            if (pos < a.cap) {
                const uint64_t* key = a.ovf_keys + (uint64_t)(rep - 1) * W;
#pragma unroll
                for (int w = 0; w < W; w++) a.out_keys[pos * W + w] = key[w] ^ (w ? 0ull : stored_xor(a.canonical, a.k));
                a.out_counts[pos] = c;
            } else {
                set_status(a.status, ST_OUT_CAP);
            }
        }
    }
    flush_max(a.max_count, wmax);
    __syncthreads();
    for (uint32_t b = tid; b < kLdsHist; b += kOvfBlock)
        if (lh[b]) add_dev(&a.hist[b], (uint64_t)lh[b]);
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
// Grid of the emergency-area kernels: enough workgroups for the largest area;
// each returns at once when the area is empty.
static uint32_t ovf_grid(const CountArgs& a) {
    const uint64_t blocks = (2 * a.ovf_cap + kOvfBlock - 1) / kOvfBlock;
    return (uint32_t)(blocks < 2048 ? blocks : 2048);
}
template <int W>
static hipError_t overflow_w(const CountArgs& a, hipStream_t s) {
    const uint32_t g = ovf_grid(a);
    hipLaunchKernelGGL(k_ovf_clear, dim3(g), dim3(kOvfBlock), 0, s, a);
    hipLaunchKernelGGL(k_ovf_insert<W>, dim3(g), dim3(kOvfBlock), 0, s, a);
    hipLaunchKernelGGL(k_ovf_dump<W>, dim3(g), dim3(kOvfBlock), 0, s, a);
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

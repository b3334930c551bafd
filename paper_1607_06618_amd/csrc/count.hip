// Counting step (phase two): every bin is cut into canonical k-mers
// (Sec. 2.3.2 splitter, Sec. 2.4.2) which are inserted into an
// open-addressing hash table with double hashing (Sec. 2.2, Alg. 1): a key
// that matches a slot increments its counter, an empty slot takes the key
// with count 1, otherwise the next trial is probed; after theta trials the
// key goes to the emergency area (Sec. 3.4.3), which is sorted and
// run-length counted after the tables. Tables are dumped after their bin
// (Sec. 2.3.2 step 3): pairs with count >= threshold are emitted (App. A
// `-l`) and every count feeds the count-of-counts histogram.
//
// GPU table (prior art: Sec. 3.3.1 scans a 128-byte window per probe):
//   * slots are grouped in buckets of kBucket = 8; the probe words (word 0 of
//     each key) of a bucket are one 64-byte line, loaded by one lane at once,
//     so a probe scans 8 candidates whatever k is (probe words are stored
//     apart from the rest of the key, structure of arrays);
//   * trial t probes bucket fastrange(h1 + t*h2) with h2 odd (double hashing);
//   * a slot is claimed by CAS on word 0 (EMPTY = all ones: a canonical key
//     never has word 0 = all ones when k < 64; for k >= 64 such keys take the
//     emergency path). For W >= 2 the claimer then stores words 1..W-1 and
//     publishes the key by raising the counter from 0 to 1; a lane that finds
//     its word 0 in a claimed slot waits until the counter is non-zero before
//     comparing the other words. Claim, store and publish happen in one loop
//     iteration, so a waiting lane never waits on a lane of its own wave;
//   * counters are 32-bit (App. C); reaching 2^32-1 is an error.
//
// Exactness: slots are never freed while a bin is counted, so a key that
// fails theta trials found every probed bucket full of other keys and can
// never enter the table later; all of its occurrences go to the emergency
// area, which is therefore disjoint from the table contents.
#include "common.h"
#include "internal.h"

namespace gerbil {

constexpr uint32_t kSpinLimit = 1u << 22;   // bounded wait for an unpublished slot

// Publication of words 1..W-1 before the counter. The release fence makes
// the stores of the other words visible at agent scope before the counter
// increment; the matching acquire is on the reader's counter load.
__device__ __forceinline__ void publish_fence() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }
__device__ __forceinline__ uint32_t ld_cnt_acquire(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

template <int W>
__device__ __forceinline__ void overflow_push(const CountArgs& a, const uint64_t (&key)[W]) {
    uint64_t idx = add_dev(a.n_ovf, 1ull);
    if (idx < a.ovf_cap) {
#pragma unroll
        for (int i = 0; i < W; i++) a.ovf_keys[idx * W + i] = key[i];
    } else {
        set_status(a.status, ST_OVF_CAP);
    }
}

// Alg. 1 for one key. Returns false when theta trials failed (the caller
// sends the key to the emergency area).
template <int W>
__device__ __forceinline__ bool table_insert(const CountArgs& a, const Table& t, uint32_t nb,
                                             const uint64_t (&key)[W], uint64_t h) {
    if (W > 1 && key[0] == GERBIL_EMPTY) return false;
    const uint32_t h1 = (uint32_t)h, h2 = (uint32_t)(h >> 32) | 1u;
    for (uint32_t trial = 0; trial < a.theta; trial++) {
        const uint64_t bucket = fastrange32(h1 + trial * h2, nb);
        uint64_t* w0 = t.w0 + bucket * kBucket;
        uint32_t match = 0, empty = 0;
#pragma unroll
        for (uint32_t j = 0; j < kBucket; j++) {
            uint64_t v = ld_dev(w0 + j);
            match |= (uint32_t)(v == key[0]) << j;
            empty |= (uint32_t)(v == GERBIL_EMPTY) << j;
        }
        uint32_t spins = 0;
        while (match | empty) {
            const uint32_t j = __builtin_ctz(match | empty);
            const uint64_t slot = bucket * kBucket + j;
            if ((empty >> j) & 1u) {
                uint64_t old = cas_dev(w0 + j, GERBIL_EMPTY, key[0]);
                if (old == GERBIL_EMPTY) {
                    if (W > 1) {
#pragma unroll
                        for (int i = 1; i < W; i++) t.rest[(uint64_t)(i - 1) * t.stride + slot] = key[i];
                        publish_fence();
                    }
                    add_dev(t.cnt + slot, 1u);
                    return true;
                }
                empty &= ~(1u << j);
                if (old == key[0]) match |= 1u << j;
                continue;
            }
            // word 0 matches
            if (W == 1) {
                uint32_t old = add_dev(t.cnt + slot, 1u);
                if (old >= 0xFFFFFFFEu) set_status(a.status, ST_COUNT_SAT);
                return true;
            }
            uint32_t c = ld_cnt_acquire(t.cnt + slot);
            if (c == 0) {
                if (++spins > kSpinLimit) {
                    set_status(a.status, ST_SPIN);
                    return true;
                }
                __builtin_amdgcn_s_sleep(1);
                continue;
            }
            bool eq = true;
#pragma unroll
            for (int i = 1; i < W; i++) eq &= (t.rest[(uint64_t)(i - 1) * t.stride + slot] == key[i]);
            if (eq) {
                uint32_t old = add_dev(t.cnt + slot, 1u);
                if (old >= 0xFFFFFFFEu) set_status(a.status, ST_COUNT_SAT);
                return true;
            }
            match &= ~(1u << j);
        }
    }
    return false;
}

// Block-wide exclusive scan of one value per thread (blockDim.x <= 1024).
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* wsum, uint32_t& total) {
    const uint32_t lane = __lane_id(), wave = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    uint32_t incl = v;
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t y = __shfl_up(incl, off);
        if (lane >= (uint32_t)off) incl += y;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    if (wave == 0) {
        uint32_t s = lane < nw ? wsum[lane] : 0u;
        uint32_t si = s;
        for (int off = 1; off < 64; off <<= 1) {
            uint32_t y = __shfl_up(si, off);
            if (lane >= (uint32_t)off) si += y;
        }
        if (lane < nw) wsum[lane] = si - s;
        if (lane == 63) wsum[16] = si;
    }
    __syncthreads();
    total = wsum[16];
    uint32_t r = wsum[wave] + incl - v;
    __syncthreads();
    return r;
}

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
            int64_t p = sstart[lo] + (int64_t)(idx - spre[lo]);
            if (p < 0 || (uint64_t)p + a.k > a.n_bytes) {   // a corrupt descriptor must not read out of range
                set_status(a.status, ST_SPIN);
                continue;
            }
            uint64_t fw[W], rc[W], key[W];
            extract_kmer<W>(a.packed, p, a.k, fw, rc);
            canonical_of<W>(fw, rc, key);
            uint64_t h = key_hash<W>(key, a.seed);
            if (!table_insert<W>(a, t, nb, key, h)) overflow_push<W>(a, key);
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
        uint32_t c = slot < n_slots ? ld_dev(t.cnt + slot) : 0u;
        if (c) {
            if (c < kLdsHist) atomicAdd(&lh[c], 1u);
            else add_dev(&a.hist[c < kHistInternal - 1 ? c : kHistInternal - 1], 1ull);
            wmax = c > wmax ? c : wmax;
        }
        bool emit = c != 0 && c >= a.threshold;
        uint64_t pos = wave_reserve(a.n_out, emit);
        if (emit) {
            if (pos < a.cap) {
                a.out_keys[pos * W] = ld_dev(t.w0 + slot);
#pragma unroll
                for (int i = 1; i < W; i++) a.out_keys[pos * W + i] = t.rest[(uint64_t)(i - 1) * t.stride + slot];
                a.out_counts[pos] = c;
            } else {
                set_status(a.status, ST_OUT_CAP);
            }
        }
        if (c) {
            st_dev(t.w0 + slot, GERBIL_EMPTY);
            st_dev(t.cnt + slot, 0u);
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        uint32_t y = __shfl_xor(wmax, off);
        wmax = y > wmax ? y : wmax;
    }
    if (__lane_id() == 0 && wmax)
        __hip_atomic_fetch_max(a.max_count, (uint64_t)wmax, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
    }
    return hipErrorInvalidValue;
}

}  // namespace gerbil

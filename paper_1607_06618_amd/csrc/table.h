// Counting step (phase two): every bin is cut into canonical k-mers
// (Sec. 2.3.2 splitter, Sec. 2.4.2) which are inserted into an
// open-addressing hash table with double hashing (Sec. 2.2, Alg. 1): a key
// that matches a slot increments its counter, an empty slot takes the key
// with count 1, otherwise the next trial is probed; after theta trials the
// key goes to the emergency area (Sec. 3.4.3), counted after the tables in
// a table of its own. Tables are dumped after their bin
// (Sec. 2.3.2 step 3): pairs with count >= threshold are emitted (App. A
// `-l`) and every count feeds the count-of-counts histogram.
//
// GPU table (prior art: Sec. 3.3.1 scans a 128-byte window per probe):
//   * slots are grouped in buckets of kBucket = 8; the probe words (word 0 of
//     each key) of a bucket are one 64-byte line, loaded by one lane at once,
//     so a probe scans 8 candidates whatever k is (probe words are stored
//     apart from the rest of the key, structure of arrays);
//   * trial t probes bucket (b0 + t*s) mod nb with nb a power of two and s odd
//     (double hashing with a full period);
//   * a slot is claimed by CAS on word 0 (EMPTY = all ones). A key whose
//     stored word 0 is all ones takes the emergency path instead: a canonical
//     key (stored as is) has one only when it starts with 32 T's and k >= 64,
//     a `-d` key (word 0 stored XORed with GERBIL_DIRECT_XOR) only when it
//     starts with the one 32-mer that the XOR maps onto the marker. For W >= 2
//     the claimer then stores words 1..W-1 and
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
#pragma once
#include "common.h"
#include "internal.h"

namespace gerbil {

constexpr uint32_t kSpinLimit = 1u << 22;   // bounded wait for an unpublished slot

// Publication of words 1..W-1 before the counter. Every word a workgroup
// shares with another one is accessed with device-coherent (agent-scope
// atomic) loads and stores, which keep each location coherent across all
// CUs and XCDs. The claimer drains its stores (s_waitcnt vmcnt(0): each has
// been performed) before it raises the counter; a reader loads the other
// words only after it has seen a non-zero counter. No cache write-back or
// invalidation is needed on the hot path.
__device__ __forceinline__ void store_rest(uint64_t* p, uint64_t v) { st_dev(p, v); }
__device__ __forceinline__ uint64_t load_rest(const uint64_t* p) { return ld_dev(p); }
__device__ __forceinline__ void publish_fence() { drain_memory(); }
__device__ __forceinline__ void acquire_fence() { asm volatile("" ::: "memory"); }

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
    if (key[0] == GERBIL_EMPTY) return false;   // the empty-slot marker is never stored
    // nb is a power of two and the step is odd: the theta buckets are distinct
    const uint32_t mask = nb - 1;
    const uint32_t step = ((uint32_t)(h >> 32) | 1u) & mask | 1u;
    uint32_t bk = fastrange32((uint32_t)h, nb);
    for (uint32_t trial = 0; trial < a.theta; trial++, bk = (bk + step) & mask) {
        const uint64_t bucket = bk;
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
                        for (int i = 1; i < W; i++) store_rest(t.rest + (uint64_t)(i - 1) * t.stride + slot, key[i]);
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
            uint32_t c = ld_dev(t.cnt + slot);
            if (c == 0) {
                if (++spins > kSpinLimit) {
                    set_status(a.status, ST_SPIN);
                    return true;
                }
                __builtin_amdgcn_s_sleep(1);
                continue;
            }
            acquire_fence();
            bool eq = true;
#pragma unroll
            for (int i = 1; i < W; i++) eq &= (load_rest(t.rest + (uint64_t)(i - 1) * t.stride + slot) == key[i]);
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

// One slot of a dumped table: histogram the count (LDS buckets for small
// counts), emit the pair if count >= threshold, reset the slot. Every lane of
// the wave must call this (the output cursor is reserved per wave).
template <int W>
__device__ __forceinline__ void compact_slot(const CountArgs& a, const Table& t, uint64_t slot, bool active,
                                             uint32_t* lh, uint32_t& wmax) {
    uint32_t c = active ? ld_dev(t.cnt + slot) : 0u;
    if (c) {
        if (c < kLdsHist) atomicAdd(&lh[c], 1u);
        else add_dev(&a.hist[c < kHistInternal - 1 ? c : kHistInternal - 1], 1ull);
        wmax = c > wmax ? c : wmax;
    }
    bool emit = c != 0 && c >= a.threshold;
    uint64_t pos = wave_reserve(a.n_out, emit);
    if (emit) {
        if (pos < a.cap) {
            a.out_keys[pos * W] = ld_dev(t.w0 + slot) ^ stored_xor(a.canonical, a.k);
#pragma unroll
            for (int i = 1; i < W; i++) a.out_keys[pos * W + i] = load_rest(t.rest + (uint64_t)(i - 1) * t.stride + slot);
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

// Wave max of the largest count seen, then one atomic per wave.
__device__ __forceinline__ void flush_max(uint64_t* max_count, uint32_t wmax) {
    for (int off = 32; off > 0; off >>= 1) {
        uint32_t y = __shfl_xor(wmax, off);
        wmax = y > wmax ? y : wmax;
    }
    if (__lane_id() == 0 && wmax)
        __hip_atomic_fetch_max(max_count, (uint64_t)wmax, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The k-mer at position p: canonical key and hash, inserted or sent to the
// emergency area.
template <int W>
__device__ __forceinline__ void count_position(const CountArgs& a, const Table& t, uint32_t nb, int64_t p) {
    if (p < 0 || (uint64_t)p + a.k > a.n_bytes) {   // a corrupt descriptor must not read out of range
        set_status(a.status, ST_SPIN);
        return;
    }
    uint64_t fw[W], rc[W], key[W];
    extract_kmer<W>(a.packed, p, a.k, fw, rc);
    canonical_of<W>(fw, rc, key, a.canonical);
    key[0] ^= stored_xor(a.canonical, a.k);
    uint64_t h = key_hash<W>(key, a.seed);
    if (!table_insert<W>(a, t, nb, key, h)) overflow_push<W>(a, key);
}

}  // namespace gerbil

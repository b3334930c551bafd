// Device helpers shared by the gfx950 kernels of the counting path.
//
// Base code and packing (App. C): A=00, C=01, G=10, T=11. The read stream is
// packed 32 bases per 64-bit word, byte position i -> word i/32, with the
// first base of a word in bits 63:62. The packed array is preceded by one and
// followed by two zero words, so that any 32-base window starting in
// [-32, n_bytes) can be read without a bounds test.
//
// Key layout: W = ceil(k/32) words; words 0..W-2 hold 32 bases each (first
// base most significant), word W-1 holds the remaining r = k - 32(W-1) bases
// right-aligned. Numeric comparison word by word from word 0 is then the
// lexicographic order A<C<G<T used for canonical k-mers (Sec. 2.4.2).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define GERBIL_MAX_W 15         // longest key compiled: 15 words = k <= 480 (HBM tables)
#define GERBIL_MAX_LDS_W 8      // LDS tables: keys of up to 8 words (k <= 256)
#define GERBIL_EMPTY (~(uint64_t)0)    // probe word of an unclaimed slot

// Keys of k >= 32 counted as read (the `-d` mode of App. A) are stored with
// their first word XORed with this constant, and the XOR is undone on output. The all-T
// prefix (an all-ones word, the empty-slot marker), common in real reads as
// poly-A/poly-T tracts, is then an ordinary key; the stored word that equals
// the marker belongs to one fixed, irregular 32-mer, whose occurrences take
// the emergency area. Canonical keys are stored unchanged: a canonical key
// starts with 32 T's only if its reverse complement does too.
#define GERBIL_DIRECT_XOR 0x9E3779B97F4A7C15ull

// Device status bits (written with atomicOr, read back by the host).
#define ST_OUT_CAP 0x1u         // output pairs exceeded the caller's capacity
#define ST_OVF_CAP 0x2u         // emergency area exceeded its capacity
#define ST_SUPERM_CAP 0x4u      // super-mer descriptors exceeded capacity
#define ST_COUNT_SAT 0x8u       // a counter reached 2^32-1
#define ST_SPIN 0x10u           // a bounded wait gave up (device error)
#define ST_OFFSETS 0x20u        // offsets[n_reads] != n_bytes
#define ST_POOL 0x40u           // a bin needed a bigger table than the pool holds

namespace gerbil {

// 32 bases starting at global base position pos (pos >= -32).
__device__ __forceinline__ uint64_t window32(const uint64_t* __restrict__ P, int64_t pos) {
    int64_t q = pos >> 5;  // floor division (arithmetic shift)
    uint32_t r = (uint32_t)(pos & 31);
    // Both words are read unconditionally (the packed stream has a zero word
    // before and two after it), so the two loads are in flight together.
    uint64_t a = P[q];
    uint64_t b = P[q + 1];
    return r ? ((a << (2 * r)) | (b >> (64 - 2 * r))) : a;
}

// Reverse complement of 32 packed bases: reverse the order of the 2-bit
// groups and complement each (A<->T is 00<->11, C<->G is 01<->10: bitwise NOT).
__device__ __forceinline__ uint64_t revcomp32(uint64_t x) {
    x = __builtin_bitreverse64(~x);
    // bit reversal also swapped the two bits inside each group; swap back
    return ((x >> 1) & 0x5555555555555555ull) | ((x & 0x5555555555555555ull) << 1);
}

// Forward and reverse-complement keys of the k-mer at position p.
template <int W>
__device__ __forceinline__ void extract_kmer(const uint64_t* __restrict__ P, int64_t p, uint32_t k,
                                             uint64_t (&fw)[W], uint64_t (&rc)[W]) {
    const uint32_t r = k - 32u * (W - 1);  // bases in the last word, 1..32
    const uint32_t sh = 2u * (32u - r);
#pragma unroll
    for (int i = 0; i < W - 1; i++) {
        fw[i] = window32(P, p + 32 * i);
        rc[i] = revcomp32(window32(P, p + (int64_t)k - 32 * (i + 1)));
    }
    uint64_t tail = window32(P, p + 32 * (W - 1));
    fw[W - 1] = sh ? (tail >> sh) : tail;
    uint64_t rtail = revcomp32(window32(P, p - 32 + (int64_t)r));
    rc[W - 1] = sh ? (rtail >> sh) : rtail;
}

// XOR applied to a key's first word in the tables (GERBIL_DIRECT_XOR). Below
// k = 32 the one key word holds 2k bits under zero top bits, so it never
// equals the marker, and it is kept as is: the LDS path stores a key's last
// word in only as many bytes as its bases need.
__device__ __forceinline__ uint64_t stored_xor(uint32_t canonical, uint32_t k) {
    return canonical || k < 32 ? 0ull : GERBIL_DIRECT_XOR;
}

// canonical = lexicographically smaller of fw and rc (compare from word 0);
// with canon false (the `-d` mode of App. A) the key is fw itself.
template <int W>
__device__ __forceinline__ void canonical_of(const uint64_t (&fw)[W], const uint64_t (&rc)[W], uint64_t (&key)[W],
                                             bool canon) {
    bool take_rc = false, decided = !canon;
#pragma unroll
    for (int i = 0; i < W; i++) {
        if (!decided && fw[i] != rc[i]) {
            take_rc = rc[i] < fw[i];
            decided = true;
        }
    }
#pragma unroll
    for (int i = 0; i < W; i++) key[i] = take_rc ? rc[i] : fw[i];
}

// Avalanche step of MurmurHash3 (fmix64).
__device__ __forceinline__ uint64_t fmix64(uint64_t z) {
    z ^= z >> 33;
    z *= 0xff51afd7ed558ccdull;
    z ^= z >> 33;
    z *= 0xc4ceb9fe1a85ec53ull;
    z ^= z >> 33;
    return z;
}

// Hash of a key: the words folded by XOR at distinct rotations, then one
// avalanche (two 64-bit multiplies in all; a 64-bit multiply costs four
// quarter-rate 32-bit multiplies on this GPU, and every k-mer is hashed
// twice). Only slot positions depend on it, never results.
template <int W>
__device__ __forceinline__ uint64_t key_hash(const uint64_t (&key)[W], uint64_t seed) {
    uint64_t h = seed ^ key[0];
#pragma unroll
    for (int i = 1; i < W; i++) {
        const int r = (23 * i) & 63;
        h ^= (key[i] << r) | (key[i] >> ((64 - r) & 63));
    }
    return fmix64(h);
}

// Map a 32-bit value uniformly onto [0, n) (multiply-shift range reduction).
__device__ __forceinline__ uint32_t fastrange32(uint32_t x, uint32_t n) {
    return (uint32_t)(((uint64_t)x * (uint64_t)n) >> 32);
}

// Agent-scope (device-coherent) accessors for memory shared between
// workgroups. They compile to loads/stores/atomics with the sc1 bit on gfx950,
// which bypass the non-coherent per-CU cache.
template <typename T>
__device__ __forceinline__ T ld_dev(const T* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T, typename U>
__device__ __forceinline__ void st_dev(T* p, U v) {
    __hip_atomic_store(p, static_cast<T>(v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T, typename U>
__device__ __forceinline__ T add_dev(T* p, U v) {
    return __hip_atomic_fetch_add(p, static_cast<T>(v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T, typename U, typename V>
__device__ __forceinline__ T cas_dev(T* p, U expected_in, V desired) {
    T expected = static_cast<T>(expected_in);
    __hip_atomic_compare_exchange_strong(p, &expected, static_cast<T>(desired), __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
    return expected;  // the value found (== old expected on success)
}
// Wait until every memory operation this wave issued has been performed
// (loads returned, stores and atomics acknowledged). Also a compiler barrier.
__device__ __forceinline__ void drain_memory() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Item hand-off between workgroups: every thread drains its device-coherent
// writes, the block meets, then one thread raises the done counter.
__device__ __forceinline__ void signal_done(uint32_t* ctr) {
    drain_memory();
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait (one thread) until *ctr >= target; bounded by `limit` polls (sets
// `bit` in *status on give-up). Data guarded by the counter is read with
// device-coherent loads afterwards.
__device__ __forceinline__ void wait_done(const uint32_t* ctr, uint32_t target, uint32_t limit, uint32_t* status,
                                          uint32_t bit) {
    uint32_t spins = 0;
    while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        if (++spins > limit) {
            __hip_atomic_fetch_or(status, bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
        }
        __builtin_amdgcn_s_sleep(2);
    }
    asm volatile("" ::: "memory");
}

// Segment of a work item: last j with start[j] <= item, searched forward from
// `hint` (items are popped in increasing order, so a workgroup's segments
// never decrease) by galloping, then bisection.
__device__ __forceinline__ uint32_t find_segment(const uint64_t* start, uint32_t ns, uint64_t item, uint32_t hint) {
    uint32_t lo = hint, step = 1, hi = lo + 1;
    while (hi < ns && start[hi] <= item) {
        lo = hi;
        hi = lo + step;
        step <<= 1;
    }
    if (hi > ns) hi = ns;
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (start[mid] <= item) lo = mid; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ void set_status(uint32_t* status, uint32_t bits) {
    __hip_atomic_fetch_or(status, bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wave-aggregated reservation of `want` (0 or 1 per lane) slots on a global
// cursor: one atomic per wave; returns this lane's index.
__device__ __forceinline__ uint64_t wave_reserve(uint64_t* cursor, bool want) {
    uint64_t mask = __ballot(want);
    if (mask == 0) return 0;
    uint32_t lane = __lane_id();
    uint32_t leader = __ffsll((unsigned long long)mask) - 1;
    uint32_t rank = __popcll(mask & ((1ull << lane) - 1ull));
    uint64_t base = 0;
    if (lane == leader) base = add_dev(cursor, (uint64_t)__popcll(mask));
    base = __shfl(base, leader);
    return base + rank;
}

}  // namespace gerbil

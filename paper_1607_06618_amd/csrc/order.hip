// Minimizer orders of Sec. 3.1 as rank tables (table[c] = rank of canonical
// m-mer code c; 0xFFFFFFFF for codes that are not canonical).
//
// CGAT, Roberts et al., KMC2 and plain lexicographic ranks are closed forms
// of the code, one thread per code. Random and dfp(p) sort the canonical
// codes by a 64-bit key -- (generator value or sampled frequency) << 30 |
// code -- with a bitonic sort over the 4^m keys (codes that are not
// canonical carry all-ones keys and sort last); the rank is then the sorted
// position (Random) or a closed form of it (dfp: the order of positions by
// distance from the pivot, lower position first on ties).
#include "../../include/gerbil.h"
#include "common.h"
#include "internal.h"

namespace gerbil {
namespace {

constexpr uint32_t kOB = 256;
constexpr uint32_t kMaxSortM = 12;               // 4^12 keys = 128 MB of workspace
constexpr uint32_t kDefaultStride = 16;
constexpr uint64_t kCodeMask30 = (1ull << 30) - 1;

__device__ __forceinline__ uint64_t rc_code(uint64_t c, uint32_t m) {
    const uint64_t mask = m == 32 ? ~0ull : ((1ull << (2 * m)) - 1ull);
    return revcomp32(c << (64 - 2 * m)) & mask;
}

// Lexicographic rank of the m bases of c under an alphabet order given as
// the rank of A, C, G, T in four 2-bit fields (A in bits 1:0); bases at odd
// positions counted from 0 are complemented first when flip_odd is set.
__device__ __forceinline__ uint32_t remap_rank(uint64_t c, uint32_t m, uint32_t alpha, bool flip_odd) {
    uint32_t r = 0;
    for (uint32_t i = 0; i < m; i++) {
        uint32_t b = (uint32_t)(c >> (2 * (m - 1 - i))) & 3u;
        if (flip_odd && (i & 1)) b = 3u - b;
        r = (r << 2) | ((alpha >> (2 * b)) & 3u);
    }
    return r;
}

// Alphabet orders: rank of A, C, G, T packed A-first.
constexpr uint32_t kAlphaCGAT = (2u << 0) | (0u << 2) | (1u << 4) | (3u << 6);      // C<G<A<T
constexpr uint32_t kAlphaRoberts = (1u << 0) | (0u << 2) | (3u << 4) | (2u << 6);   // C<A<T<G

__global__ void __launch_bounds__(kOB) k_ranks_closed(uint32_t kind, uint32_t m, uint32_t* __restrict__ table) {
    const uint64_t n = 1ull << (2 * m);
    for (uint64_t c = (uint64_t)blockIdx.x * kOB + threadIdx.x; c < n; c += (uint64_t)gridDim.x * kOB) {
        uint32_t r = 0xFFFFFFFFu;
        if (c <= rc_code(c, m)) {
            switch (kind) {
                case GERBIL_RANKS_LEX: r = (uint32_t)c; break;
                case GERBIL_RANKS_KMC2: {
                    const uint64_t head = m >= 3 ? c >> (2 * m - 6) : 1ull;
                    r = (uint32_t)(c + ((head == 0 || head == 4) ? n : 0ull));   // AAA, ACA behind all others
                    break;
                }
                case GERBIL_RANKS_CGAT: r = remap_rank(c, m, kAlphaCGAT, false); break;
                default: r = remap_rank(c, m, kAlphaRoberts, true); break;
            }
        }
        table[c] = r;
    }
}

// SplitMix64 (Steele, Lea and Flood, 2014): output i of a generator seeded
// with `seed`, from its counter-based form.
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Sampled frequencies: the canonical m-mer starting each valid k-mer window
// at a multiple of stride.
__global__ void __launch_bounds__(kOB) k_mmer_sample(const uint64_t* __restrict__ packed,
                                                     const uint64_t* __restrict__ kmer_ok, uint64_t n_pos,
                                                     uint32_t m, uint32_t stride, uint32_t* __restrict__ hist) {
    const uint64_t n_samples = (n_pos + stride - 1) / stride;
    for (uint64_t s = (uint64_t)blockIdx.x * kOB + threadIdx.x; s < n_samples; s += (uint64_t)gridDim.x * kOB) {
        const uint64_t p = s * stride;
        if (!((kmer_ok[p >> 6] >> (p & 63)) & 1ull)) continue;
        const uint64_t fw = window32(packed, (int64_t)p) >> (64 - 2 * m);
        const uint64_t rc = rc_code(fw, m);
        atomicAdd(&hist[fw < rc ? fw : rc], 1u);
    }
}

__global__ void __launch_bounds__(kOB) k_rank_keys(uint32_t kind, uint32_t m, uint64_t seed,
                                                   const uint32_t* __restrict__ hist, uint64_t* __restrict__ keys) {
    const uint64_t n = 1ull << (2 * m);
    for (uint64_t c = (uint64_t)blockIdx.x * kOB + threadIdx.x; c < n; c += (uint64_t)gridDim.x * kOB) {
        uint64_t key = ~0ull;
        if (c <= rc_code(c, m)) {
            uint64_t v;
            if (kind == GERBIL_RANKS_RANDOM) {
                v = splitmix64(seed, c) >> 34;
            } else {
                v = hist[c];
            }
            key = (v << 30) | c;
        }
        keys[c] = key;
    }
}

// One compare-exchange pass of a bitonic sort (ascending) over n = 2^s keys.
__global__ void __launch_bounds__(kOB) k_bitonic_pass(uint64_t* __restrict__ keys, uint64_t n, uint64_t j,
                                                      uint64_t size) {
    for (uint64_t i = (uint64_t)blockIdx.x * kOB + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kOB) {
        const uint64_t l = i ^ j;
        if (l <= i) continue;
        const uint64_t x = keys[i], y = keys[l];
        const bool up = (i & size) == 0;
        if (up ? (x > y) : (x < y)) {
            keys[i] = y;
            keys[l] = x;
        }
    }
}

// dfp: rank of sorted position pos among M positions ordered by distance
// from P (0 <= P <= M), the lower position first on ties.
__device__ __forceinline__ uint64_t dfp_rank(uint64_t pos, uint64_t P, uint64_t M) {
    const int64_t d = pos > P ? (int64_t)(pos - P) : (int64_t)(P - pos);
    if (d == 0) return 0;
    const int64_t lo = (int64_t)P - d + 1 > 0 ? (int64_t)P - d + 1 : 0;
    const int64_t hi = (int64_t)P + d - 1 < (int64_t)M - 1 ? (int64_t)P + d - 1 : (int64_t)M - 1;
    const uint64_t closer = hi >= lo ? (uint64_t)(hi - lo + 1) : 0ull;
    return closer + ((pos > P && (int64_t)P - d >= 0) ? 1ull : 0ull);
}

__global__ void __launch_bounds__(kOB) k_rank_assign(uint32_t kind, uint32_t m, uint64_t P, uint64_t M,
                                                     const uint64_t* __restrict__ keys, uint32_t* __restrict__ table) {
    const uint64_t n = 1ull << (2 * m);
    for (uint64_t pos = (uint64_t)blockIdx.x * kOB + threadIdx.x; pos < n; pos += (uint64_t)gridDim.x * kOB) {
        const uint64_t key = keys[pos];
        if (key == ~0ull) continue;   // the tail of codes that are not canonical
        const uint64_t c = key & kCodeMask30;
        table[c] = (uint32_t)(kind == GERBIL_RANKS_RANDOM ? pos : dfp_rank(pos, P, M));
    }
}

uint32_t grid_for_codes(uint64_t n) {
    const uint64_t g = (n + kOB - 1) / kOB;
    return (uint32_t)(g < 1 ? 1 : g < 16384 ? g : 16384);
}

uint64_t canonical_count(uint32_t m) {
    const uint64_t all = 1ull << (2 * m);
    return (m & 1) ? all / 2 : (all + (1ull << m)) / 2;   // even m: 4^(m/2) palindromes
}

bool sorted_kind(uint32_t kind) { return kind == GERBIL_RANKS_RANDOM || kind == GERBIL_RANKS_DFP; }

}  // namespace
}  // namespace gerbil

using namespace gerbil;

extern "C" {

int32_t gerbil_order_table_workspace(uint32_t kind, uint32_t m, uint64_t* bytes) {
    if (!bytes || kind > GERBIL_RANKS_DFP || m < 1 || m > 15) return GERBIL_EINVAL;
    if (!sorted_kind(kind)) {
        *bytes = 0;
        return GERBIL_OK;
    }
    if (m > kMaxSortM) return GERBIL_EINVAL;
    const uint64_t n = 1ull << (2 * m);
    *bytes = align256(8 * n) + (kind == GERBIL_RANKS_DFP ? align256(4 * n) : 0);
    return GERBIL_OK;
}

int32_t gerbil_order_table(uint32_t kind, uint32_t m, uint64_t seed, float pivot, uint32_t stride,
                           const gerbil_encoded* enc, void* ws, uint64_t ws_bytes, uint32_t* table,
                           hipStream_t stream) {
    uint64_t need = 0;
    if (!table || gerbil_order_table_workspace(kind, m, &need) != GERBIL_OK) return GERBIL_EINVAL;
    const uint64_t n = 1ull << (2 * m);
    if (!sorted_kind(kind)) {
        hipLaunchKernelGGL(k_ranks_closed, dim3(grid_for_codes(n)), dim3(kOB), 0, stream, kind, m, table);
        return hipGetLastError() == hipSuccess ? GERBIL_OK : GERBIL_EDEVICE;
    }
    if (!ws || ws_bytes < need || (((uintptr_t)ws) & 255)) return GERBIL_EINVAL;
    if (kind == GERBIL_RANKS_DFP) {
        if (!enc || !(pivot >= 0.0f && pivot <= 1.0f) || m >= enc->k) return GERBIL_EINVAL;
        if (enc->n_bytes && (!enc->packed || !enc->kmer_ok)) return GERBIL_EINVAL;
    }
    uint64_t* keys = (uint64_t*)ws;
    uint32_t* hist = (uint32_t*)((uint8_t*)ws + align256(8 * n));
    if (kind == GERBIL_RANKS_DFP) {
        if (launch_fill_u32(hist, n, 0u, stream) != hipSuccess) return GERBIL_EDEVICE;
        const uint64_t n_pos = enc->n_bytes >= enc->k ? enc->n_bytes - enc->k + 1 : 0;
        const uint32_t st = stride ? stride : kDefaultStride;
        if (n_pos)
            hipLaunchKernelGGL(k_mmer_sample, dim3(grid_for_codes((n_pos + st - 1) / st)), dim3(kOB), 0, stream,
                               enc->packed, enc->kmer_ok, n_pos, m, st, hist);
    }
    hipLaunchKernelGGL(k_rank_keys, dim3(grid_for_codes(n)), dim3(kOB), 0, stream, kind, m, seed, hist, keys);
    for (uint64_t size = 2; size <= n; size <<= 1)
        for (uint64_t j = size >> 1; j > 0; j >>= 1)
            hipLaunchKernelGGL(k_bitonic_pass, dim3(grid_for_codes(n)), dim3(kOB), 0, stream, keys, n, j, size);
    if (launch_fill_u32(table, n, 0xFFFFFFFFu, stream) != hipSuccess) return GERBIL_EDEVICE;
    const uint64_t M = canonical_count(m);
    const uint64_t P = (uint64_t)((double)pivot * (double)M);   // floor: both factors are non-negative
    hipLaunchKernelGGL(k_rank_assign, dim3(grid_for_codes(n)), dim3(kOB), 0, stream, kind, m, P, M, keys, table);
    return hipGetLastError() == hipSuccess ? GERBIL_OK : GERBIL_EDEVICE;
}

}  // extern "C"

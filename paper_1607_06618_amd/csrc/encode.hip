// Encoding of the reads (the parser step of phase one, Sec. 2.3.1):
// ASCII -> 2-bit codes of App. C, plus the bitmaps that say which k-mer
// windows are valid (Sec. 2.4.1: a window with an undetermined base is
// ignored; windows never span two reads).
//
// Three streaming passes, all coalesced:
//   read_starts  scatter one bit per read start into a bitmap;
//   pack         16 ASCII bytes per lane -> 32 bits of packed codes and 16
//                validity bits (SWAR over 4 bytes per 32-bit word);
//   kmer_ok      bit p = window [p, p+k) is valid, from the "position i and
//                i+1 belong to one read and are both valid" bitmap: each
//                (rare) zero of that bitmap clears the windows that span it.
#include "common.h"
#include "internal.h"

namespace gerbil {

__global__ void k_fill_u64(uint64_t* __restrict__ p, uint64_t n, uint64_t v) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill_u32(uint32_t* __restrict__ p, uint64_t n, uint32_t v) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

static uint32_t grid_for(uint64_t n, uint32_t block, uint32_t max_grid = 65536) {
    uint64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > max_grid) g = max_grid;
    return (uint32_t)g;
}

hipError_t launch_fill_u64(uint64_t* p, uint64_t n, uint64_t value, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, p, n, value);
    return hipGetLastError();
}
hipError_t launch_fill_u32(uint32_t* p, uint64_t n, uint32_t value, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, p, n, value);
    return hipGetLastError();
}

// One thread per read: set the bit of its first byte; check the offsets.
__global__ void k_read_starts(const uint64_t* __restrict__ offsets, uint64_t n_reads, uint64_t n_bytes,
                              uint64_t* __restrict__ rs, uint32_t* status) {
    uint64_t r = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (r > n_reads) return;
    uint64_t pos = offsets[r];
    if (r == n_reads) {
        if (pos != n_bytes) set_status(status, ST_OFFSETS);
        return;
    }
    uint64_t nxt = offsets[r + 1];
    if (nxt < pos || (r == 0 && pos != 0)) set_status(status, ST_OFFSETS);
    if (pos < n_bytes)
        __hip_atomic_fetch_or(rs + (pos >> 6), 1ull << (pos & 63), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

hipError_t launch_read_starts(const uint64_t* offsets, uint64_t n_reads, uint64_t n_bytes, uint64_t* read_start,
                              uint32_t* status, hipStream_t s) {
    uint64_t n = n_reads + 1;
    uint64_t g = (n + 255) / 256;
    hipLaunchKernelGGL(k_read_starts, dim3((uint32_t)g), dim3(256), 0, s, offsets, n_reads, n_bytes, read_start,
                       status);
    return hipGetLastError();
}

// Four ASCII bytes -> 4 codes (2 bits each, first byte most significant in
// the returned 8 bits) and 4 validity bits (bit j = byte j is A/C/G/T/a/c/g/t).
__device__ __forceinline__ void encode4(uint32_t x, uint32_t& codes8, uint32_t& valid4) {
    // For A/C/G/T in either case, bits 2 and 1 of the byte XOR-ed give
    // A=00, C=01, G=10, T=11.
    uint32_t c = ((x >> 2) ^ (x >> 1)) & 0x03030303u;
    // The byte must equal the lower-case letter of that code after
    // folding case: bytes of 0x74676361 are 'a','c','g','t'.
    uint32_t y = x | 0x20202020u;
    uint32_t expect = __builtin_amdgcn_perm(0u, 0x74676361u, c);
    uint32_t z = y ^ expect;
    uint32_t nz = ((z & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | z;   // bit 7 of a byte set iff byte != 0
    uint32_t ok = ~nz & 0x80808080u;                        // bit 7 set iff byte matches
    c &= (ok >> 7) * 3u;                                    // invalid bytes -> code 0
    codes8 = ((c & 3u) << 6) | (((c >> 8) & 3u) << 4) | (((c >> 16) & 3u) << 2) | ((c >> 24) & 3u);
    valid4 = ((ok >> 7) & 1u) | ((ok >> 14) & 2u) | ((ok >> 21) & 4u) | ((ok >> 28) & 8u);
}

// Lane h encodes bytes [16h, 16h+16): 32 bits of packed codes (half of a
// 64-bit word; the first 16 bases of a word are its high half, hence dword
// index h^1 on a little-endian device) and 16 validity bits.
__global__ void k_pack(const uint8_t* __restrict__ ascii, uint64_t n_bytes, uint32_t* __restrict__ packed32,
                       uint16_t* __restrict__ valid16, int aligned) {
    uint64_t n16 = (n_bytes + 15) >> 4;
    for (uint64_t h = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; h < n16; h += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t b0 = h << 4;
        uint32_t x[4];
        if (aligned && b0 + 16 <= n_bytes) {
            uint4 v = *reinterpret_cast<const uint4*>(ascii + b0);
            x[0] = v.x; x[1] = v.y; x[2] = v.z; x[3] = v.w;
        } else {
#pragma unroll
            for (int j = 0; j < 4; j++) {
                uint32_t w = 0;
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    uint64_t i = b0 + 4 * j + q;
                    uint32_t byte = i < n_bytes ? ascii[i] : 0u;   // past the end: invalid
                    w |= byte << (8 * q);
                }
                x[j] = w;
            }
        }
        uint32_t out = 0, vbits = 0;
#pragma unroll
        for (int j = 0; j < 4; j++) {
            uint32_t c8, v4;
            encode4(x[j], c8, v4);
            out |= c8 << (24 - 8 * j);
            vbits |= v4 << (4 * j);
        }
        packed32[h ^ 1] = out;
        valid16[h] = (uint16_t)vbits;
    }
}

hipError_t launch_pack(const uint8_t* ascii, uint64_t n_bytes, uint64_t* packed, uint64_t* valid, hipStream_t s) {
    uint64_t n16 = (n_bytes + 15) >> 4;
    int aligned = (((uintptr_t)ascii) & 15) == 0;
    hipLaunchKernelGGL(k_pack, dim3(grid_for(n16, 256, 1 << 20)), dim3(256), 0, s, ascii, n_bytes,
                       reinterpret_cast<uint32_t*>(packed), reinterpret_cast<uint16_t*>(valid), aligned);
    return hipGetLastError();
}

// Words of the bitmaps at or beyond the end read as zero: both bitmaps have a
// zero word at index n, so the index is clamped instead of branching (all
// loads of a thread can then be in flight together).
__device__ __forceinline__ uint64_t ld_or_zero(const uint64_t* __restrict__ a, uint64_t i, uint64_t n) {
    return a[i < n ? i : n];
}

// Words of G a thread reads: 64 output bits + k - 2 following bits. Five
// words serve k <= 257, nine the longest keys (k <= 32 * GERBIL_MAX_W).
constexpr int kOkWordsShort = 5;
constexpr int kOkWordsLong = 9;
static_assert((63 + 32 * GERBIL_MAX_W - 2) / 64 + 1 <= kOkWordsLong, "windows of the longest k");

// Thread q computes bitmap word q: bit p = AND of G[p .. p+k-2], where
// G[i] = valid[i] & valid[i+1] & !read_start[i+1] (i and i+1 are consecutive
// bases of one read). For k = 1 the bitmap is just `valid`. Zeros of G are
// rare (read ends and undetermined bases), so instead of ANDing shifted
// copies the thread walks the zeros of G in [64q, 64q + 63 + k - 2] and
// clears, for each zero z, the windows p in [z - k + 2, z] of its word.
template <int kOkWords>
__global__ void __launch_bounds__(256) k_kmer_ok(const uint64_t* __restrict__ valid, const uint64_t* __restrict__ rs,
                                                 uint64_t n_mask, uint32_t k, uint64_t* __restrict__ ok,
                                                 uint64_t* n_valid) {
    __shared__ uint32_t wsum[4];
    uint64_t cnt = 0;
    for (uint64_t q = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; q < n_mask;
         q += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t res;
        if (k == 1) {
            res = valid[q];
        } else {
            const uint32_t span = k - 2;                    // window p needs G[p .. p+span]
            const uint32_t nw = (63 + span) / 64 + 1;       // words of G that can hold such zeros (<= kOkWords)
            uint64_t V[kOkWords + 1], R[kOkWords + 1];
#pragma unroll
            for (int i = 0; i <= kOkWords; i++) {
                V[i] = ld_or_zero(valid, q + i, n_mask);
                R[i] = ld_or_zero(rs, q + i, n_mask);
            }
            res = ~0ull;
#pragma unroll
            for (int i = 0; i < kOkWords; i++) {
                if ((uint32_t)i >= nw) break;
                const uint64_t vnext = (V[i] >> 1) | (V[i + 1] << 63);
                const uint64_t rnext = (R[i] >> 1) | (R[i + 1] << 63);
                uint64_t zeros = ~(V[i] & vnext & ~rnext);
                while (zeros) {
                    const uint32_t z = 64u * (uint32_t)i + (uint32_t)__builtin_ctzll(zeros);   // relative to 64q
                    zeros &= zeros - 1;
                    if (z > 63u + span) break;                      // beyond the last window of this word
                    const uint32_t lo = z > span ? z - span : 0u;   // windows [lo, hi] contain z
                    const uint32_t hi = z < 63u ? z : 63u;
                    if (lo <= hi) res &= ~((~0ull >> (63u - hi)) & (~0ull << lo));
                }
            }
        }
        ok[q] = res;
        cnt += __popcll(res);
    }
    // one atomic per workgroup (a single counter takes every add in turn)
    uint32_t tot = (uint32_t)cnt;
    for (int off = 32; off > 0; off >>= 1) tot += __shfl_xor(tot, off);
    if (__lane_id() == 0) wsum[threadIdx.x >> 6] = tot;
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint64_t t = (uint64_t)wsum[0] + wsum[1] + wsum[2] + wsum[3];
        if (t) add_dev(n_valid, t);
    }
}

hipError_t launch_kmer_ok(const uint64_t* valid, const uint64_t* read_start, uint64_t n_mask, uint32_t k,
                          uint64_t* kmer_ok, uint64_t* n_valid, hipStream_t s) {
    if (n_mask == 0) return hipSuccess;
    if ((63 + k - 2) / 64 + 1 <= (uint32_t)kOkWordsShort || k < 2)
        hipLaunchKernelGGL(k_kmer_ok<kOkWordsShort>, dim3(grid_for(n_mask, 256, 4096)), dim3(256), 0, s, valid,
                           read_start, n_mask, k, kmer_ok, n_valid);
    else
        hipLaunchKernelGGL(k_kmer_ok<kOkWordsLong>, dim3(grid_for(n_mask, 256, 4096)), dim3(256), 0, s, valid,
                           read_start, n_mask, k, kmer_ok, n_valid);
    return hipGetLastError();
}

}  // namespace gerbil

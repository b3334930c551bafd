// Binary output records of the emitted pairs (App. C): the counter -- one
// byte when it is below 255, else the byte 0xFF and the count as a
// big-endian 32-bit word -- then the k-mer, four bases per byte with the first
// base in the top bits and the last byte padded with zero bits.
//
// Record sizes take two values (1 + kb or 5 + kb bytes, kb = ceil(k/4)), so
// the offset of record i is i (1 + kb) + 4 x (large counters before i): an
// exclusive scan of one flag per pair. Three launches: flags per tile, a
// scan of the tile totals, then per tile and round the records are built in
// LDS and the round's byte range is copied out with consecutive lanes on
// consecutive bytes.
#include <mutex>

#include "../../include/gerbil.h"
#include "table.h"

namespace gerbil {
namespace {

constexpr uint32_t kRecBlock = 1024;
constexpr uint32_t kRecRounds = 8;                       // rounds of kRecBlock pairs per tile
constexpr uint64_t kRecTile = (uint64_t)kRecBlock * kRecRounds;

__device__ __forceinline__ uint32_t block_sum(uint32_t v, uint32_t* wsum) {
    uint32_t total;
    (void)block_excl_scan(v, wsum, total);
    return total;
}

// Large counters (>= 255) per tile.
__global__ void __launch_bounds__(kRecBlock) k_rec_flags(const uint32_t* __restrict__ counts, uint64_t n,
                                                         uint32_t* __restrict__ tile_big) {
    __shared__ uint32_t wsum[32];
    const uint64_t n_tiles = (n + kRecTile - 1) / kRecTile;
    for (uint64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        uint32_t big = 0;
        for (uint32_t r = 0; r < kRecRounds; r++) {
            const uint64_t i = t * kRecTile + (uint64_t)r * kRecBlock + threadIdx.x;
            big += (i < n && counts[i] >= 255u) ? 1u : 0u;
        }
        const uint32_t tot = block_sum(big, wsum);
        if (threadIdx.x == 0) tile_big[t] = tot;
        __syncthreads();
    }
}

// Exclusive prefix of the tile totals (one workgroup); writes the stream size.
__global__ void __launch_bounds__(kRecBlock) k_rec_scan(const uint32_t* __restrict__ tile_big, uint64_t n_tiles,
                                                        uint64_t* __restrict__ tile_base, uint64_t n, uint32_t kb,
                                                        uint64_t* out_bytes) {
    __shared__ uint64_t part[kRecBlock];
    const uint32_t tid = threadIdx.x;
    const uint64_t per = (n_tiles + kRecBlock - 1) / kRecBlock;
    uint64_t sum = 0;
    for (uint64_t e = 0; e < per; e++) {
        const uint64_t j = tid * per + e;
        if (j < n_tiles) sum += tile_big[j];
    }
    part[tid] = sum;
    __syncthreads();
    for (uint32_t off = 1; off < kRecBlock; off <<= 1) {
        const uint64_t y = tid >= off ? part[tid - off] : 0ull;
        __syncthreads();
        part[tid] += y;
        __syncthreads();
    }
    uint64_t run = tid ? part[tid - 1] : 0ull;
    for (uint64_t e = 0; e < per; e++) {
        const uint64_t j = tid * per + e;
        if (j < n_tiles) {
            tile_base[j] = run;
            run += tile_big[j];
        }
    }
    if (tid == kRecBlock - 1) *out_bytes = n * (1ull + kb) + 4ull * part[kRecBlock - 1];
}

// The k-mer bytes of a key: byte j holds bases 4j..4j+3.
__device__ __forceinline__ uint32_t kmer_byte(const uint64_t* key, uint32_t W, uint32_t k, uint32_t j) {
    const uint32_t w = j / 8, b = j % 8;
    uint64_t x = key[w];
    if (w == W - 1) {
        const uint32_t r = k - 32 * (W - 1);   // bases in the last word, right-aligned
        if (r < 32) x <<= 2 * (32 - r);        // left-align: the padding bits become zero
    }
    return (uint32_t)(x >> (56 - 8 * b)) & 0xFFu;
}

__global__ void __launch_bounds__(kRecBlock) k_rec_write(const uint64_t* __restrict__ keys,
                                                         const uint32_t* __restrict__ counts, uint64_t n, uint32_t k,
                                                         uint32_t W, const uint64_t* __restrict__ tile_base,
                                                         uint8_t* __restrict__ out, uint64_t out_cap) {
    extern __shared__ __align__(16) uint8_t stage[];   // one round of records
    __shared__ uint32_t wsum[32];
    const uint32_t tid = threadIdx.x;
    const uint32_t kb = (k + 3) / 4;
    const uint64_t n_tiles = (n + kRecTile - 1) / kRecTile;
    for (uint64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        uint64_t big_before = tile_base[t];   // large counters before this round
        for (uint32_t r = 0; r < kRecRounds; r++) {
            const uint64_t i0 = t * kRecTile + (uint64_t)r * kRecBlock;
            if (i0 >= n) break;
            const uint64_t i = i0 + tid;
            const bool have = i < n;
            const uint32_t c = have ? counts[i] : 0u;
            const uint32_t big = (have && c >= 255u) ? 1u : 0u;
            uint32_t big_round;
            const uint32_t big_pre = block_excl_scan(big, wsum, big_round);
            // the round's bytes start at the record offset of pair i0
            const uint64_t base = i0 * (1ull + kb) + 4ull * big_before;
            const uint32_t loc = tid * (1u + kb) + 4u * big_pre;   // this record inside the round
            const uint32_t n_here = (uint32_t)((n - i0) < kRecBlock ? (n - i0) : kRecBlock);
            const uint32_t round_bytes = n_here * (1u + kb) + 4u * big_round;
            if (have) {
                uint32_t o = loc;
                if (c < 255u) {
                    stage[o++] = (uint8_t)c;
                } else {
                    stage[o++] = 0xFF;
                    stage[o++] = (uint8_t)(c >> 24);
                    stage[o++] = (uint8_t)(c >> 16);
                    stage[o++] = (uint8_t)(c >> 8);
                    stage[o++] = (uint8_t)c;
                }
                const uint64_t* key = keys + i * W;
                for (uint32_t j = 0; j < kb; j++) stage[o++] = (uint8_t)kmer_byte(key, W, k, j);
            }
            __syncthreads();
            for (uint32_t b = tid; b < round_bytes; b += kRecBlock) {
                const uint64_t g = base + b;
                if (g < out_cap) out[g] = stage[b];
            }
            big_before += big_round;
            __syncthreads();   // the stage is reused by the next round
        }
    }
}

// Workspace bytes for n_tiles tiles: the large-counter count per tile, then
// the large counters before each tile.
constexpr uint64_t rec_ws_bytes(uint64_t n_tiles) { return 256 + ((4 * n_tiles + 255) & ~255ull) + 8 * n_tiles; }

hipError_t enqueue_records(const uint64_t* keys, const uint32_t* counts, uint64_t n, uint32_t k, uint8_t* ws,
                           uint8_t* out, uint64_t out_cap, uint64_t* out_bytes, hipStream_t stream) {
    const uint32_t W = (k + 31) / 32, kb = (k + 3) / 4;
    if (n == 0) return launch_fill_u64(out_bytes, 1, 0ull, stream);
    const uint64_t n_tiles = (n + kRecTile - 1) / kRecTile;
    uint32_t* tile_big = (uint32_t*)(ws + 256);
    uint64_t* tile_base = (uint64_t*)(ws + 256 + ((4 * n_tiles + 255) & ~255ull));
    const uint32_t grid = (uint32_t)(n_tiles < 4096 ? n_tiles : 4096);
    hipLaunchKernelGGL(k_rec_flags, dim3(grid), dim3(kRecBlock), 0, stream, counts, n, tile_big);
    hipLaunchKernelGGL(k_rec_scan, dim3(1), dim3(kRecBlock), 0, stream, tile_big, n_tiles, tile_base, n, kb, out_bytes);
    const uint32_t lds = kRecBlock * (5 + kb);   // up to 69 KB: above the default dynamic LDS limit
    // set on every call: the attribute belongs to the current device's module
    hipError_t e = hipFuncSetAttribute((const void*)k_rec_write, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rec_write, dim3(grid), dim3(kRecBlock), lds, stream, keys, counts, n, k, W, tile_base, out,
                       out_cap);
    return hipGetLastError();
}

// The allocation-free variant keeps the workspace in a static device array
// of the library: one copy per GPU, at that GPU's own address, which the host
// learns once per device with hipGetSymbolAddress. The array's name in host
// code is only a host-side stand-in and is never passed to a kernel.
constexpr uint64_t kNoAllocTiles = GERBIL_RECORDS_NOALLOC_MAX / kRecTile;
static_assert(GERBIL_RECORDS_NOALLOC_MAX % kRecTile == 0, "the pair limit is whole tiles");
constexpr uint64_t kScratchBytes = rec_ws_bytes(kNoAllocTiles);
constexpr int kMaxDevices = 64;

}  // namespace

static __device__ __align__(256) uint8_t scratch[kScratchBytes];

namespace {

std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once per device).
hipError_t scratch_address(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

}  // namespace
}  // namespace gerbil

using namespace gerbil;

extern "C" {

int32_t gerbil_records_workspace(uint64_t n, uint64_t* bytes) {
    if (!bytes) return GERBIL_EINVAL;
    *bytes = rec_ws_bytes((n + kRecTile - 1) / kRecTile);
    return GERBIL_OK;
}

int32_t gerbil_records(const uint64_t* keys, const uint32_t* counts, uint64_t n, uint32_t k, void* ws,
                       uint64_t ws_bytes, uint8_t* out, uint64_t out_cap, uint64_t* out_bytes, hipStream_t stream) {
    if (!out_bytes || k < 1 || k > 32 * GERBIL_MAX_W) return GERBIL_EINVAL;
    if (n && (!keys || !counts || !ws || (out_cap && !out))) return GERBIL_EINVAL;
    if (n && (ws_bytes < rec_ws_bytes((n + kRecTile - 1) / kRecTile) || (((uintptr_t)ws) & 255))) return GERBIL_EINVAL;
    return enqueue_records(keys, counts, n, k, (uint8_t*)ws, out, out_cap, out_bytes, stream) == hipSuccess
               ? GERBIL_OK
               : GERBIL_EDEVICE;
}

int32_t gerbil_records_noalloc(const uint64_t* keys, const uint32_t* counts, uint64_t n, uint32_t k, uint8_t* out,
                               uint64_t out_cap, uint64_t* out_bytes, hipStream_t stream) {
    if (!out_bytes || k < 1 || k > 32 * GERBIL_MAX_W || n > GERBIL_RECORDS_NOALLOC_MAX) return GERBIL_EINVAL;
    if (n && (!keys || !counts || (out_cap && !out))) return GERBIL_EINVAL;
    void* ws = nullptr;
    if (scratch_address(&ws) != hipSuccess) return GERBIL_EDEVICE;
    return enqueue_records(keys, counts, n, k, (uint8_t*)ws, out, out_cap, out_bytes, stream) == hipSuccess
               ? GERBIL_OK
               : GERBIL_EDEVICE;
}

}  // extern "C"

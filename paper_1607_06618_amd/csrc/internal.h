// Internal launch interface between the C-ABI layer and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gerbil {

constexpr uint32_t kBucket = 8;         // slots per bucket: one 64-byte line of probe words
constexpr uint32_t kHistInternal = 65536;  // internal count-of-counts buckets (last saturates)
constexpr uint32_t kLdsHist = 256;      // histogram buckets privatised in LDS during compaction
constexpr uint32_t kTile = 2048;        // k-mer positions per minimizer-scan tile
constexpr uint32_t kMaxBins = 4096;

// ------------------------------------------------------------ encode
hipError_t launch_fill_u64(uint64_t* p, uint64_t n, uint64_t value, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint64_t n, uint32_t value, hipStream_t s);
hipError_t launch_read_starts(const uint64_t* offsets, uint64_t n_reads, uint64_t n_bytes, uint64_t* read_start,
                              uint32_t* status, hipStream_t s);
hipError_t launch_pack(const uint8_t* ascii, uint64_t n_bytes, uint64_t* packed, uint64_t* valid, hipStream_t s);
hipError_t launch_kmer_ok(const uint64_t* valid, const uint64_t* read_start, uint64_t n_mask, uint32_t k,
                          uint64_t* kmer_ok, uint64_t* n_valid, hipStream_t s);

// ------------------------------------------------------------ bins
struct BinArgs {
    const uint64_t* packed;
    const uint64_t* kmer_ok;
    uint64_t n_bytes;
    uint32_t k, m, n_bins, order;
    const uint32_t* bin_map;
    uint64_t cap;
    uint64_t* list_desc;    // [cap] tile order
    uint32_t* list_bin;     // [cap]
    uint64_t* n_superm;     // scalar
    uint32_t* bin_count;    // [n_bins] super-mers per bin
    uint32_t* bin_fill;     // [n_bins] scatter cursors
    uint64_t* bin_off;      // [n_bins+1]
    uint64_t* bin_kmers;    // [n_bins]
    uint64_t* desc;         // [cap] bin order
    uint32_t* status;
};
hipError_t launch_bin(const BinArgs& a, uint32_t grid, hipStream_t s);

// ------------------------------------------------------------ count
struct Table {
    uint64_t* w0;     // [stride] probe words (word 0 of the key)
    uint64_t* rest;   // [(W-1) * stride] words 1..W-1, word-major
    uint32_t* cnt;    // [stride]
    uint64_t stride;  // slots allocated per table
};

struct CountArgs {
    const uint64_t* packed;
    uint64_t n_bytes;     // k-mer windows must lie inside [0, n_bytes)
    const uint64_t* desc;
    uint32_t k, W, threshold, theta;
    uint64_t seed;
    // emergency area
    uint64_t* ovf_keys;   // [ovf_cap * W]
    uint64_t ovf_cap;
    uint64_t* n_ovf;
    // output
    uint64_t* out_keys;   // [cap * W]
    uint32_t* out_counts;
    uint64_t cap;
    uint64_t* n_out;
    uint64_t* hist;       // [kHistInternal]
    uint64_t* max_count;
    uint32_t* status;
};

// Table j of a pool: [w0: slots][rest: (W-1) * slots][cnt: slots], each part 256-byte aligned.
__host__ __device__ inline uint64_t align256(uint64_t x) { return (x + 255) & ~255ull; }
__host__ __device__ inline uint64_t pool_table_bytes(uint64_t slots, uint32_t W) {
    return align256(slots * 8) + align256(slots * 8 * (W - 1)) + align256(slots * 4);
}
__host__ __device__ inline Table pool_table(uint8_t* pool, uint64_t slots, uint32_t W, uint32_t j) {
    uint8_t* p = pool + (uint64_t)j * pool_table_bytes(slots, W);
    Table t;
    t.stride = slots;
    t.w0 = (uint64_t*)p;
    p += align256(slots * 8);
    t.rest = (uint64_t*)p;
    p += align256(slots * 8 * (W - 1));
    t.cnt = (uint32_t*)p;
    return t;
}

// BATCHED schedule: every bin in one persistent launch.
struct PersistArgs {
    uint8_t* pool;            // Q tables of `slots` slots each
    uint64_t slots;
    uint32_t Q;               // tables resident at once
    uint32_t lag;             // dump of rank i is queued after the inserts of rank i+lag (lag < Q)
    uint32_t n_bins;
    uint32_t ins_chunk;       // descriptors per insert item (= block size)
    uint32_t cmp_chunk;       // slots per dump item
    float load;
    const uint64_t* bin_off;  // [n_bins+1]
    const uint64_t* bin_kmers;
    uint32_t* order;          // [n_bins] rank -> bin, largest bin first
    uint32_t* nb;             // [n_bins] buckets used by rank
    uint32_t* n_ins;          // [n_bins] insert items of rank
    uint32_t* n_cmp;          // [n_bins] dump items of rank
    uint32_t* ins_done;       // [n_bins]
    uint32_t* cmp_done;       // [n_bins]
    uint32_t* seg_code;       // [2 n_bins] (kind << 31) | rank
    uint64_t* seg_start;      // [2 n_bins + 1] first item of each queue segment
    uint64_t* cursor;         // work-stealing cursor
    const uint64_t* n_superm; // descriptors found by the binning
    uint64_t superm_cap;      // descriptors stored; nothing is scheduled if exceeded
    uint32_t* status;
};
hipError_t launch_plan(const PersistArgs& q, hipStream_t s);
hipError_t launch_count_persistent(const CountArgs& a, const PersistArgs& q, uint32_t grid, uint32_t block,
                                   hipStream_t s);
uint32_t persistent_blocks_per_cu(uint32_t W, uint32_t block);

// PLAIN: insert the k-mers of descriptors [d0, d1) into a table of nb buckets.
hipError_t launch_count_bin(const CountArgs& a, const Table& t, uint32_t nb, uint64_t d0, uint64_t d1,
                            uint32_t block, hipStream_t s);
// PLAIN: compact nb buckets of a table (emit, histogram, reset).
hipError_t launch_compact(const CountArgs& a, const Table& t, uint32_t nb, hipStream_t s);
// Emergency area: sort-and-count every key that did not fit in a table.
hipError_t launch_overflow(const CountArgs& a, hipStream_t s);

}  // namespace gerbil

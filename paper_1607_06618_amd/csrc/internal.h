// Internal launch interface between the C-ABI layer and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
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
    const uint32_t* rank_table;   // order TABLE: rank of each canonical m-mer code
    uint64_t cap;           // descriptors (super-mer pieces) that fit in desc
    uint64_t list_cap;      // cap + kListSlack: slots of the tile-order list, holes included
    uint64_t* list_desc;    // [list_cap] tile order
    uint32_t* list_bin;     // [list_cap] bin, or kHole for a slot left unused
    uint64_t* list_used;    // scalar: list slots handed out
    uint64_t* n_superm;     // scalar
    uint32_t* bin_count;    // [n_bins] super-mers per bin
    uint32_t* bin_fill;     // [n_bins] scatter cursors
    uint64_t* bin_off;      // [n_bins+1]
    uint64_t* bin_kmers;    // [n_bins]
    uint64_t* desc;         // [cap] bin order
    uint32_t* status;
};
hipError_t launch_bin(const BinArgs& a, uint32_t max_grid, uint32_t cus, hipStream_t s);
// bins[i] = the bin gerbil_bin gives key i (uses a.k, a.m, a.order, a.rank_table, a.bin_map, a.n_bins)
hipError_t launch_key_bins(const uint64_t* keys, uint64_t n, const BinArgs& a, uint32_t* bins, hipStream_t s);
// HyperLogLog registers [n_bins << p] of every bin's canonical (or, canonical = 0, as read) k-mers
hipError_t launch_hll(const uint64_t* packed, uint64_t n_bytes, const uint64_t* desc, const uint64_t* bin_off,
                      uint32_t n_bins, uint32_t k, uint32_t canonical, uint32_t p, uint32_t* regs, hipStream_t s);
// The tile kernel hands out list slots to each workgroup in chunks of at
// least kListChunk and fills them without gaps; only the unused end of each
// workgroup's last chunk (under kListChunk slots) is a hole. At most
// kMaxTileGrid workgroups, hence the slack.
constexpr uint32_t kListChunk = 2048;
constexpr uint32_t kMaxTileGrid = 2048;
constexpr uint64_t kListSlack = (uint64_t)kListChunk * kMaxTileGrid;
constexpr uint32_t kHole = 0xFFFFFFFFu;

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
    uint32_t canonical;   // 1: key = smaller of the k-mer and its reverse complement; 0: the k-mer (`-d`)
    uint64_t seed;
    // emergency area
    uint64_t* ovf_keys;   // [ovf_cap * W]
    uint64_t ovf_cap;
    uint64_t* n_ovf;
    // its counting table: ovf_slots = 2 ovf_cap (a power of two) slots
    uint32_t* ovf_state;  // [ovf_slots] 0 free, 1 being claimed, 2 published
    uint64_t* ovf_tkeys;  // [ovf_slots * W]
    uint32_t* ovf_tcnt;   // [ovf_slots]
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

// LDS sub-table path. A rank is one hash slice of a bin (bins too large for
// max_sub sub-tables are cut into slices by the high hash bits); a rank has P
// sub-tables, each counted by one workgroup in LDS.
//
// Two workgroup shapes share the CU's 160 KB of LDS: one workgroup of 1024
// threads per CU with all of it, or two of 512 threads with half each (their
// stages then overlap on the CU; tables hold half as many keys). The per-bin
// schedule always uses the first.
constexpr uint32_t kLdsBlock = 1024;   // threads of the 1024-thread shape (and of the per-bin schedule)
template <uint32_t B>
struct LdsShape {
    static_assert(B == 1024 || B == 512, "LDS workgroups have 512 or 1024 threads");
    static constexpr uint32_t bytes = (160u * 1024u) / (1024u / B);   // dynamic LDS per workgroup
    // sub-tables per rank: bounded by the three per-sub-table arrays of the scatter stage
    static constexpr uint32_t max_sub = B == 1024 ? 4096u : 1536u;
};
inline uint32_t lds_bytes_for(uint32_t B) { return B == 512 ? LdsShape<512>::bytes : LdsShape<1024>::bytes; }
inline uint32_t lds_max_sub_for(uint32_t B) { return B == 512 ? LdsShape<512>::max_sub : LdsShape<1024>::max_sub; }
// Bytes that hold the last word of a key: 2 bits per base of its k - 32(W-1) bases.
inline uint32_t tail_bytes_for(uint32_t k) {
    const uint32_t W = (k + 31) / 32, r = k - 32 * (W - 1);
    return r <= 4 ? 1u : r <= 8 ? 2u : r <= 16 ? 4u : 8u;
}
// Run sizing from a sample: every S-th segment of L = kSegMax / S k-mers is
// counted. A sampled segment adds at most L keys to any run, so the estimate
// S c of a run holding n keys has variance at most S L n, whatever the input
// (clumps of one key included). A run gets S c plus four standard deviations
// of that bound plus a floor; with S = 1 the count is exact.
constexpr uint32_t kSegMax = 32;
__host__ __device__ inline uint32_t sample_seg_len(uint32_t S) { return S >= kSegMax ? 1u : kSegMax / S; }
__host__ __device__ inline uint64_t run_capacity(uint64_t c, uint32_t S) {
    if (S <= 1) return c;
    const double L = sample_seg_len(S), est = (double)S * (double)c;
    return (uint64_t)est + (uint64_t)(4.0 * sqrt((double)S * L * (est + L))) + 32ull;
}
inline uint64_t slot_words_for(uint64_t slot_keys, uint32_t k) {
    const uint32_t W = (k + 31) / 32;
    return slot_keys * (W - 1) + (slot_keys * tail_bytes_for(k) + 7) / 8;
}
constexpr uint32_t kLdsReserved = 2048;         // LDS kept for the histogram and scalars
constexpr uint32_t kProbeHist = 32;             // probe-count buckets (GERBIL_PROBE_HIST)
constexpr uint32_t kProbeHistAt = 1536;         // their LDS copy inside the reserved region
// Slots of an LDS table: the largest prime that fits, so that double hashing
// has a full period.
constexpr uint32_t kLdsTableScratch = 256;      // scan scratch of the table stage after its slots
// Keys an LDS-table thread loads per batch (registers bound it); a sub-table
// gets at most 0.95 of a batch, so it is loaded in one.
__host__ __device__ constexpr int lds_table_batch(int W) {
    return W == 1 ? 12 : W == 2 ? 7 : W == 3 ? 5 : W == 4 ? 4 : W <= 7 ? 3 : 2;
}
// Packed slots hold a key's last word (at most 16 bases, 32 bits) in the high
// half of the counter's 64-bit word: 8W bytes a slot instead of 8W + 4.
inline bool lds_packed(uint32_t k) {
    const uint32_t W = (k + 31) / 32;
    return W >= 2 && k - 32 * (W - 1) <= 16;
}
inline uint32_t lds_table_slots(uint32_t W, uint32_t B, bool packed) {
    uint32_t c = (lds_bytes_for(B) - kLdsReserved - kLdsTableScratch) / (packed ? 8 * W : 8 * W + 4);
    for (;; c--) {
        bool prime = c > 2;
        for (uint32_t d = 2; prime && d * d <= c; d++) prime = c % d != 0;
        if (prime) return c;
    }
}

// Work queues of the batched LDS schedule: one per XCD (MI355X has 8, each
// with its own L2). Rank r belongs to queue r mod n_queues, and workgroup i
// starts on queue i mod n_queues: workgroups are dispatched to the XCDs in
// turn, so the scatter items of a rank run on one XCD and the partly filled
// lines of its sub-table runs merge in one L2. Cursors sit 256 bytes apart.
constexpr uint32_t kLdsQueues = 8;
constexpr uint32_t kCursorStride = 32;

struct LdsArgs {
    uint32_t block;           // threads per workgroup: 1024 or 512 (LdsShape)
    uint32_t n_queues;        // work queues (1 .. kLdsQueues, at most the grid)
    uint32_t max_sub;         // LdsShape<block>::max_sub
    uint32_t n_bins, ranks_cap;
    uint32_t* n_ranks;        // scalar (plan output)
    uint32_t* rank_bin;       // [ranks_cap]
    uint32_t* rank_slice;
    uint32_t* rank_nslice;
    uint32_t* rank_nsub;      // P (0 for an empty bin)
    uint32_t* rank_nchunk;    // descriptor chunks of `block` descriptors
    uint64_t* rank_spbase;    // first sub-table of the rank
    uint64_t* rank_keys;      // keys of the rank (scan output)
    uint64_t sp_cap;
    uint32_t* sp_cnt;         // [sp_cap] keys per sub-table
    uint64_t* sp_off;         // [sp_cap] first key of a sub-table inside its key slot
    uint32_t* sp_cur;         // [sp_cap] scatter cursors
    // Q key slots of slot_keys keys each, word-major: word w < W-1 of key i at
    // w * slot_keys + i (uint64), then the last word of every key in
    // tail_bytes bytes (1, 2, 4 or 8: it holds only k - 32(W-1) bases).
    uint64_t* keys;
    uint64_t slot_keys;
    uint64_t slot_words;      // uint64 words per slot
    uint32_t tail_bytes;
    uint32_t Q, lag;
    uint32_t target;          // keys per sub-table
    uint32_t sample;          // sub-table runs sized from every sample-th super-mer (1 = all)
    uint32_t table_slots;     // LDS slots per sub-table
    uint32_t packed;          // 1: packed slots (the last key word shares a 64-bit word with the counter)
    uint32_t theta;           // probes per key before the emergency area
    uint64_t* stage_clocks;   // optional [8]: busy wall-clock ticks per stage, then items per stage
    uint64_t* probe_hist;     // optional [kProbeHist]: inserts by the probe that settled them
    const uint64_t* bin_off;
    const uint64_t* bin_kmers;
    uint32_t* done;           // [4 * ranks_cap] finished items per (rank, stage)
    uint64_t* seg_start;      // [kLdsQueues][4 * (ranks_cap + 3 + lag) + 1]: queue q at q * (n_seg + 1)
    uint32_t* n_seg;          // scalar
    uint64_t* cursor;         // [kLdsQueues * kCursorStride]: queue q at q * kCursorStride
    const uint64_t* n_superm;
    uint64_t superm_cap;
    uint32_t* status;
};
hipError_t launch_lds_plan(const LdsArgs& l, hipStream_t s);
hipError_t launch_lds_persistent(const CountArgs& a, const LdsArgs& l, uint32_t grid, hipStream_t s);
// PLAIN: one stage of one rank (stage 0 count, 1 scan, 2 scatter, 3 LDS count + dump), `items` blocks.
hipError_t launch_lds_stage(const CountArgs& a, const LdsArgs& l, uint32_t stage, uint32_t rank, uint32_t items,
                            hipStream_t s);

// PLAIN: insert the k-mers of descriptors [d0, d1) into a table of nb buckets.
hipError_t launch_count_bin(const CountArgs& a, const Table& t, uint32_t nb, uint64_t d0, uint64_t d1,
                            uint32_t block, hipStream_t s);
// PLAIN: compact nb buckets of a table (emit, histogram, reset).
hipError_t launch_compact(const CountArgs& a, const Table& t, uint32_t nb, hipStream_t s);
// Emergency area: count every key that did not fit in a table (clear, insert and
// dump its counting table; many workgroups, no host synchronisation).
hipError_t launch_overflow(const CountArgs& a, hipStream_t s);
inline uint64_t ovf_table_slots(uint64_t ovf_cap) { return 2 * ovf_cap; }

}  // namespace gerbil

// C-ABI of the counting library: argument checks, workspace layout and the
// launch sequences of gerbil_encode / gerbil_bin / gerbil_count /
// gerbil_histogram. No device memory is allocated here; every buffer is
// carved out of a caller-owned workspace.
#include <string.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <vector>

#include "../../include/gerbil.h"
#include "common.h"
#include "internal.h"

using namespace gerbil;

namespace {

constexpr uint64_t kAlign = 256;
constexpr uint64_t kHashSeed = 0x243F6A8885A308D3ull;   // digits of pi; only slot positions depend on it
constexpr uint64_t kDefaultOverflow = 1ull << 20;
constexpr uint32_t kDefaultTheta = 8;
constexpr float kDefaultLoad = 0.5f;
constexpr uint32_t kDefaultBlock = 256;

uint64_t align_up(uint64_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// Bump allocator over a workspace (or a dry run that only measures).
struct Carve {
    uint8_t* base;
    uint64_t used = 0;
    explicit Carve(void* b) : base((uint8_t*)b) {}
    template <typename T>
    T* take(uint64_t count) {
        uint64_t off = used;
        used = align_up(used + count * sizeof(T));
        return base ? (T*)(base + off) : nullptr;
    }
};

uint32_t words_for(uint32_t k) { return (k + 31) / 32; }

// Compute units of the current device (looked up per device, once).
int device_cus() {
    constexpr int kMaxDev = 64;
    static std::atomic<int> cus[kMaxDev];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDev) return 256;
    int c = cus[dev].load(std::memory_order_relaxed);
    if (!c) {
        hipDeviceProp_t prop;
        c = hipGetDeviceProperties(&prop, dev) == hipSuccess ? prop.multiProcessorCount : 0;
        if (c <= 0) c = 256;
        cus[dev].store(c, std::memory_order_relaxed);
    }
    return c;
}

uint64_t next_pow2(uint64_t x) {
    uint64_t n = 1;
    while (n < x) n <<= 1;
    return n;
}

// ---------------------------------------------------------------- encode
struct EncLayout {
    uint64_t* packed_alloc;
    uint64_t* valid;
    uint64_t* read_start;
    uint64_t* kmer_ok;
    uint64_t* scalars;   // [0] n_valid, [1] status (as uint32 in the low half)
};

uint64_t enc_layout(uint64_t n_bytes, void* ws, EncLayout* L) {
    uint64_t n_words = (n_bytes + 31) / 32, n_mask = (n_bytes + 63) / 64;
    Carve c(ws);
    EncLayout l;
    l.packed_alloc = c.take<uint64_t>(n_words + 3);
    l.valid = c.take<uint64_t>(n_mask + 1);
    l.read_start = c.take<uint64_t>(n_mask + 1);
    l.kmer_ok = c.take<uint64_t>(n_mask + 1);
    l.scalars = c.take<uint64_t>(4);   // [0] n_superm [1] list slots handed out
    if (L) *L = l;
    return c.used;
}

// ------------------------------------------------------------------ bins
uint64_t default_superm_cap(uint64_t n_bytes, uint32_t k, uint32_t m) {
    uint64_t w = k - m + 1;
    // random minimizers give about 2/(w+1) super-mers per k-mer; allow twice
    // that, plus one cut per tile
    uint64_t est = n_bytes * 4 / (w + 1) + n_bytes / kTile + 4096;
    return std::min<uint64_t>(est, n_bytes + 4096);
}

struct BinLayout {
    uint64_t* list_desc;
    uint32_t* list_bin;
    uint64_t* desc;
    uint32_t* bin_count;
    uint32_t* bin_fill;
    uint64_t* bin_off;
    uint64_t* bin_kmers;
    uint64_t* scalars;   // [0] n_superm
};

uint64_t bin_layout(uint64_t cap, uint32_t n_bins, void* ws, BinLayout* L) {
    Carve c(ws);
    BinLayout l;
    l.list_desc = c.take<uint64_t>(cap + kListSlack);
    l.list_bin = c.take<uint32_t>(cap + kListSlack);
    l.desc = c.take<uint64_t>(cap);
    l.bin_count = c.take<uint32_t>(n_bins);
    l.bin_fill = c.take<uint32_t>(n_bins);
    l.bin_off = c.take<uint64_t>(n_bins + 1);
    l.bin_kmers = c.take<uint64_t>(n_bins);
    l.scalars = c.take<uint64_t>(4);   // [0] n_superm [1] list slots handed out
    if (L) *L = l;
    return c.used;
}

int32_t check_params(const gerbil_params* p) {
    if (!p) return GERBIL_EINVAL;
    if (p->k < 2 || p->m < 1 || p->m > 15 || p->m >= p->k) return GERBIL_EINVAL;
    if (p->n_bins < 1 || p->n_bins > kMaxBins) return GERBIL_EINVAL;
    if (p->threshold < 1) return GERBIL_EINVAL;
    if (p->order > GERBIL_ORDER_TABLE || p->mode > 1 || p->table > 2) return GERBIL_EINVAL;
    if (p->order == GERBIL_ORDER_TABLE && (!p->rank_table || p->bin_map)) return GERBIL_EINVAL;
    // HBM tables hold every distinct key of a bin: at most 0.95 per slot. LDS
    // sub-tables are sized in k-mer occurrences, which repeat, so more than
    // one per slot can still fit (distinct keys beyond the slots go to the
    // emergency area, exactly).
    const float max_load = p->table == GERBIL_TABLE_HBM ? 0.95f : 4.0f;
    if (p->load_factor < 0.0f || p->load_factor > max_load) return GERBIL_EINVAL;
    if (p->block && (p->block < 64 || p->block > 1024 || (p->block & 63))) return GERBIL_EINVAL;
    if (p->k > 32 * GERBIL_MAX_W) return GERBIL_EUNSUPPORTED;
    if (p->table == GERBIL_TABLE_LDS && (p->k + 31) / 32 > GERBIL_MAX_LDS_W) return GERBIL_EUNSUPPORTED;
    if (p->canonical > 1) return GERBIL_EINVAL;
    // the emergency area's counting table refers to keys by a 32-bit index
    if (p->overflow_cap > (1ull << 31)) return GERBIL_EINVAL;
    return GERBIL_OK;
}

// ----------------------------------------------------------------- count
constexpr uint32_t kDefaultPool = 4;
constexpr uint32_t kCmpChunk = 4096;   // slots per dump item of the batched schedule

struct CountLayout {
    uint64_t* scalars;   // [0] n_out [1] n_ovf [2] max_count [3] status
    uint64_t* hist;
    uint64_t* ovf_keys;
    uint32_t* ovf_state;
    uint64_t* ovf_tkeys;
    uint32_t* ovf_tcnt;
    // batched plan
    uint32_t *order, *nb, *n_ins, *n_cmp, *ins_done, *cmp_done, *seg_code;
    uint64_t *seg_start, *cursor;
    uint8_t* pool;
};

uint64_t slots_for(uint64_t kmers, float load) {
    // The distinct count of a bin is at most its k-mer count; size for that,
    // in a power-of-two number of buckets (full-period double hashing).
    double want = (double)kmers / (double)load;
    uint64_t nb = next_pow2((uint64_t)(want / kBucket) + 1);
    if (nb > (1ull << 31)) nb = 1ull << 31;
    return nb * kBucket;
}
uint64_t prev_pow2(uint64_t x) {
    uint64_t n = 1;
    while (n * 2 <= x) n *= 2;
    return n;
}

// Everything but the table pool.
uint64_t count_fixed(uint32_t W, uint64_t ovf_cap, uint32_t n_bins, bool batched, void* ws, CountLayout* L) {
    Carve c(ws);
    CountLayout l;
    memset(&l, 0, sizeof(l));
    l.scalars = c.take<uint64_t>(8);
    l.hist = c.take<uint64_t>(kHistInternal);
    l.ovf_keys = c.take<uint64_t>(ovf_cap * W);
    l.ovf_state = c.take<uint32_t>(ovf_table_slots(ovf_cap));
    l.ovf_tkeys = c.take<uint64_t>(ovf_table_slots(ovf_cap) * W);
    l.ovf_tcnt = c.take<uint32_t>(ovf_table_slots(ovf_cap));
    if (batched) {
        l.order = c.take<uint32_t>(n_bins);
        l.nb = c.take<uint32_t>(n_bins);
        l.n_ins = c.take<uint32_t>(n_bins);
        l.n_cmp = c.take<uint32_t>(n_bins);
        l.ins_done = c.take<uint32_t>(n_bins);
        l.cmp_done = c.take<uint32_t>(n_bins);
        l.seg_code = c.take<uint32_t>(2 * n_bins);
        l.seg_start = c.take<uint64_t>(2 * n_bins + 1);
        l.cursor = c.take<uint64_t>(4);
    }
    l.pool = ws ? (uint8_t*)ws + c.used : nullptr;
    if (L) *L = l;
    return c.used;
}

uint64_t ovf_capacity(const gerbil_params* p) { return next_pow2(p->overflow_cap ? p->overflow_cap : kDefaultOverflow); }
uint32_t pool_size(const gerbil_params* p) {
    if (p->mode != GERBIL_BATCHED) return 1;
    uint32_t q = p->pool ? p->pool : kDefaultPool;
    return std::min(q, p->n_bins);
}
float load_of(const gerbil_params* p) { return p->load_factor > 0 ? p->load_factor : kDefaultLoad; }
// AUTO takes LDS tables for keys of up to GERBIL_MAX_LDS_W words, HBM tables beyond
bool use_lds(const gerbil_params* p) {
    return p->table == GERBIL_TABLE_LDS || (p->table == GERBIL_TABLE_AUTO && (p->k + 31) / 32 <= GERBIL_MAX_LDS_W);
}

// Two key slots per XCD queue: with slots a multiple of the queues, a rank and
// the earlier rank whose slot it reuses sit in the same queue, and each XCD
// scatters one rank while it counts the tables of the one before.
constexpr uint32_t kDefaultKeySlots = 2 * kLdsQueues;
constexpr uint32_t kDefaultLdsTheta = 64;   // single-slot probes are cheap in LDS
constexpr double kDefaultLdsFill = 0.8;     // k-mers per LDS slot (distinct keys are fewer)

struct LdsSizing {
    uint32_t block, max_sub;   // workgroup shape (LdsShape)
    bool packed;               // packed table slots (lds_packed)
    uint32_t C, target, ranks_cap, Q, lag, sample;
    uint64_t sp_cap;
};

// Threads per LDS-path workgroup: two 512-thread workgroups per CU when the
// batched schedule asks for blocks of 512, else one of 1024.
uint32_t lds_block(const gerbil_params* p) {
    return p->mode == GERBIL_BATCHED && p->block == 512 ? 512u : kLdsBlock;
}

constexpr uint32_t kDefaultSizeSample = 8;

LdsSizing lds_sizing(const gerbil_params* p, uint64_t n_bytes) {
    LdsSizing z;
    const uint32_t W = words_for(p->k);
    z.block = lds_block(p);
    z.max_sub = lds_max_sub_for(z.block);
    z.packed = lds_packed(p->k);
    z.C = lds_table_slots(W, z.block, z.packed);
    const double fill = p->load_factor > 0 ? p->load_factor : kDefaultLdsFill;
    z.target = std::max<uint32_t>(64, (uint32_t)((double)z.C * fill));
    // packed tables have more slots than one batch of keys fills: keep a sub-table to one batch
    if (z.packed && !(p->load_factor > 0))
        z.target = std::min<uint32_t>(z.target, (uint32_t)(0.95 * lds_table_batch((int)W) * z.block));
    const uint64_t per_slice = (uint64_t)z.max_sub * z.target;
    z.ranks_cap = (uint32_t)std::min<uint64_t>(p->n_bins + n_bytes / per_slice + 1, 1u << 20);
    z.sp_cap = n_bytes / z.target + 2ull * z.ranks_cap + 1;
    if (p->mode == GERBIL_BATCHED) {
        uint32_t q = p->pool ? p->pool : kDefaultKeySlots;
        z.Q = std::max<uint32_t>(1, std::min(q, z.ranks_cap));
    } else {
        z.Q = 1;
    }
    z.lag = z.Q / 2;
    z.sample = p->size_sample ? p->size_sample : kDefaultSizeSample;
    return z;
}

// Keys a slot must hold: the k-mers of the largest bin, plus the margins of
// its sampled run capacities: with S the sampling step and L its segment
// length, N keys in P runs, the capacities add up to at most N + 4 sqrt(S L N)
// (error of the sampled total) + 4 sqrt(S L) sqrt(P (N + P L)) (sum of the
// per-run margins, by Cauchy-Schwarz) + 32 P. A hash slice of a large bin is
// bounded by the whole bin only: slices split distinct keys evenly, but a
// key's occurrences all go to one slice, so repeats can load one slice with
// most of the bin.
uint64_t lds_slot_keys(uint64_t max_kmers, const LdsSizing& z) {
    const double N = (double)std::max<uint64_t>(max_kmers, 1);
    if (z.sample <= 1) return (uint64_t)N;
    const double S = z.sample;
    double P = std::ceil(N / z.target);
    if (P < 1) P = 1;
    if (P > z.max_sub) P = z.max_sub;
    const double L = sample_seg_len(z.sample);
    const double bound = N + 4.0 * std::sqrt(S * L * N) + 4.0 * std::sqrt(S * L) * std::sqrt(P * (N + P * L)) + 33.0 * P;
    return (uint64_t)std::ceil(bound);
}

struct LdsLayout {
    uint32_t *n_ranks, *rank_bin, *rank_slice, *rank_nslice, *rank_nsub, *rank_nchunk;
    uint64_t *rank_spbase, *rank_keys;
    uint32_t *sp_cnt, *sp_cur;
    uint64_t* sp_off;
    uint32_t* done;
    uint64_t* seg_start;
    uint32_t* n_seg;
    uint64_t* cursor;
    uint64_t* keys;
};

uint64_t lds_fixed(const LdsSizing& z, void* ws, uint64_t start, LdsLayout* L) {
    Carve c(ws ? (uint8_t*)ws + start : nullptr);
    LdsLayout l;
    l.n_ranks = c.take<uint32_t>(4);
    l.rank_bin = c.take<uint32_t>(z.ranks_cap);
    l.rank_slice = c.take<uint32_t>(z.ranks_cap);
    l.rank_nslice = c.take<uint32_t>(z.ranks_cap);
    l.rank_nsub = c.take<uint32_t>(z.ranks_cap);
    l.rank_nchunk = c.take<uint32_t>(z.ranks_cap);
    l.rank_spbase = c.take<uint64_t>(z.ranks_cap);
    l.rank_keys = c.take<uint64_t>(z.ranks_cap);
    l.sp_cnt = c.take<uint32_t>(z.sp_cap);
    l.sp_cur = c.take<uint32_t>(z.sp_cap);
    l.sp_off = c.take<uint64_t>(z.sp_cap);
    l.done = c.take<uint32_t>(4ull * z.ranks_cap);
    l.seg_start = c.take<uint64_t>(kLdsQueues * (4ull * ((uint64_t)z.ranks_cap + 3 + z.lag) + 1));
    l.n_seg = c.take<uint32_t>(4);
    l.cursor = c.take<uint64_t>(kLdsQueues * kCursorStride);
    l.keys = ws ? (uint64_t*)((uint8_t*)ws + start + c.used) : nullptr;
    if (L) *L = l;
    return c.used;
}

int32_t hip_status(hipError_t e) { return e == hipSuccess ? GERBIL_OK : GERBIL_EDEVICE; }

__global__ void k_fold_hist(const uint64_t* __restrict__ hist, uint32_t len, uint64_t* __restrict__ out) {
    __shared__ uint64_t part[256];
    const uint32_t tid = threadIdx.x;
    for (uint32_t c = tid; c + 1 < len; c += blockDim.x) out[c] = c == 0 ? 0ull : hist[c];
    uint64_t s = 0;
    for (uint32_t c = len - 1 + tid; c < kHistInternal; c += blockDim.x) s += hist[c];
    part[tid] = s;
    __syncthreads();
    for (uint32_t off = 128; off > 0; off >>= 1) {
        if (tid < off) part[tid] += part[tid + off];
        __syncthreads();
    }
    if (tid == 0) out[len - 1] = part[0];
}

void fill_state(gerbil_counted* state, const gerbil_params* p, const gerbil_bins* bins, uint64_t cap, uint64_t ovf_cap,
                const CountLayout& L) {
    memset(state, 0, sizeof(*state));
    state->k = p->k;
    state->W = words_for(p->k);
    state->threshold = p->threshold;
    state->hist_len = kHistInternal;
    state->cap = cap;
    state->overflow_cap = ovf_cap;
    state->n_out = L.scalars;
    state->n_overflow = L.scalars + 1;
    state->max_count = L.scalars + 2;
    state->status = (uint32_t*)(L.scalars + 3);
    state->hist = L.hist;
    state->n_superm = bins->n_superm;
    state->bin_status = bins->status;
}

CountArgs count_args(const gerbil_params* p, const gerbil_bins* bins, const gerbil_counted* state, uint64_t* keys,
                     uint32_t* counts, uint64_t cap, const CountLayout& L) {
    CountArgs a;
    a.packed = bins->packed;
    a.n_bytes = bins->n_bytes;
    a.desc = bins->desc;
    a.k = p->k;
    a.W = words_for(p->k);
    a.threshold = p->threshold;
    a.theta = p->max_probes ? p->max_probes : kDefaultTheta;
    a.canonical = p->canonical;
    a.seed = kHashSeed;
    a.ovf_keys = L.ovf_keys;
    a.ovf_state = L.ovf_state;
    a.ovf_tkeys = L.ovf_tkeys;
    a.ovf_tcnt = L.ovf_tcnt;
    a.ovf_cap = state->overflow_cap;
    a.n_ovf = state->n_overflow;
    a.out_keys = keys;
    a.out_counts = counts;
    a.cap = cap;
    a.n_out = state->n_out;
    a.hist = L.hist;
    a.max_count = state->max_count;
    a.status = state->status;
    return a;
}

// LDS sub-table path: plan on the device, then one persistent launch
// (BATCHED) or four launches per rank (PLAIN).
int32_t count_lds(const gerbil_bins* bins, const gerbil_params* p, void* ws, uint64_t ws_bytes, uint64_t* keys,
                  uint32_t* counts, uint64_t cap, gerbil_counted* state, hipStream_t stream) {
    const uint32_t W = words_for(p->k);
    const bool batched = p->mode == GERBIL_BATCHED;
    const uint64_t ovf_cap = ovf_capacity(p);
    const LdsSizing z = lds_sizing(p, bins->n_bytes);
    CountLayout L;
    const uint64_t fixed0 = count_fixed(W, ovf_cap, p->n_bins, false, ws, &L);
    LdsLayout LL;
    const uint64_t fixed = fixed0 + lds_fixed(z, ws, fixed0, &LL);
    if (fixed + kAlign > ws_bytes) return GERBIL_EINVAL;
    const uint64_t key_bytes = 8ull * (W - 1) + tail_bytes_for(p->k);
    uint64_t slot_keys = (ws_bytes - fixed - kAlign) / ((uint64_t)z.Q * key_bytes);
    while (slot_keys && (uint64_t)z.Q * slot_words_for(slot_keys, p->k) * 8ull > ws_bytes - fixed - kAlign) slot_keys--;
    if (slot_keys < 1) return GERBIL_EINVAL;
    if (slot_keys > 0xFFFFFFFFull) slot_keys = 0xFFFFFFFFull;   // run offsets are 32-bit inside a slot
    fill_state(state, p, bins, cap, ovf_cap, L);
    CountArgs a = count_args(p, bins, state, keys, counts, cap, L);

    // one 1024-thread workgroup per CU, or two of 512
    const uint32_t grid = batched ? (uint32_t)device_cus() * (kLdsBlock / z.block) : 1u;
    LdsArgs l;
    l.block = z.block;
    l.n_queues = std::max<uint32_t>(1, std::min(kLdsQueues, grid));
    l.max_sub = z.max_sub;
    l.n_bins = p->n_bins;
    l.ranks_cap = z.ranks_cap;
    l.n_ranks = LL.n_ranks;
    l.rank_bin = LL.rank_bin;
    l.rank_slice = LL.rank_slice;
    l.rank_nslice = LL.rank_nslice;
    l.rank_nsub = LL.rank_nsub;
    l.rank_nchunk = LL.rank_nchunk;
    l.rank_spbase = LL.rank_spbase;
    l.rank_keys = LL.rank_keys;
    l.sp_cap = z.sp_cap;
    l.sp_cnt = LL.sp_cnt;
    l.sp_off = LL.sp_off;
    l.sp_cur = LL.sp_cur;
    l.keys = LL.keys;
    l.slot_keys = slot_keys;
    l.slot_words = slot_words_for(slot_keys, p->k);
    l.tail_bytes = tail_bytes_for(p->k);
    l.Q = z.Q;
    l.lag = z.lag;
    l.target = z.target;
    l.sample = z.sample;
    l.table_slots = z.C;
    l.packed = z.packed ? 1u : 0u;
    l.theta = p->max_probes ? p->max_probes : kDefaultLdsTheta;
    l.stage_clocks = p->stage_clocks;
    l.probe_hist = batched ? p->probe_hist : nullptr;
    l.bin_off = bins->bin_off;
    l.bin_kmers = bins->bin_kmers;
    l.done = LL.done;
    l.seg_start = LL.seg_start;
    l.n_seg = LL.n_seg;
    l.cursor = LL.cursor;
    l.n_superm = bins->n_superm;
    l.superm_cap = bins->cap_superm;
    l.status = state->status;

    hipError_t e = launch_fill_u64(L.scalars, 8, 0, stream);
    if (e == hipSuccess) e = launch_fill_u64(L.hist, kHistInternal, 0, stream);
    if (e == hipSuccess) e = launch_lds_plan(l, stream);
    if (e != hipSuccess) return GERBIL_EDEVICE;
    if (batched) {
        if (p->timing_events) e = hipEventRecord(p->timing_events[0], stream);
        if (e == hipSuccess) e = launch_lds_persistent(a, l, grid, stream);
        if (e == hipSuccess && p->timing_events) e = hipEventRecord(p->timing_events[1], stream);
    } else {
        uint32_t n_ranks = 0;
        e = hipMemcpyAsync(&n_ranks, LL.n_ranks, 4, hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        std::vector<uint32_t> nchunk(n_ranks), nsub(n_ranks);
        if (e == hipSuccess && n_ranks) {
            e = hipMemcpyAsync(nchunk.data(), LL.rank_nchunk, 4ull * n_ranks, hipMemcpyDeviceToHost, stream);
            if (e == hipSuccess) e = hipMemcpyAsync(nsub.data(), LL.rank_nsub, 4ull * n_ranks, hipMemcpyDeviceToHost, stream);
            if (e == hipSuccess) e = hipStreamSynchronize(stream);
        }
        if (e == hipSuccess && p->timing_events) e = hipEventRecord(p->timing_events[0], stream);
        for (uint32_t r = 0; r < n_ranks && e == hipSuccess; r++) {
            if (!nchunk[r]) continue;
            e = launch_lds_stage(a, l, 0, r, nchunk[r], stream);
            if (e == hipSuccess) e = launch_lds_stage(a, l, 1, r, 1, stream);
            if (e == hipSuccess) e = launch_lds_stage(a, l, 2, r, nchunk[r], stream);
            if (e == hipSuccess) e = launch_lds_stage(a, l, 3, r, nsub[r], stream);
        }
        if (e == hipSuccess && p->timing_events) e = hipEventRecord(p->timing_events[1], stream);
    }
    if (e == hipSuccess) e = launch_overflow(a, stream);
    return hip_status(e);
}

}  // namespace

extern "C" {

uint32_t gerbil_version(void) { return 0x000100; }

const char* gerbil_status_string(int32_t s) {
    switch (s) {
        case GERBIL_OK: return "ok";
        case GERBIL_EINVAL: return "invalid argument";
        case GERBIL_EUNSUPPORTED: return "unsupported parameter";
        case GERBIL_ECAPACITY: return "device capacity exceeded";
        case GERBIL_EDEVICE: return "device error";
    }
    return "unknown status";
}

int32_t gerbil_encode_workspace(uint64_t n_reads, uint64_t n_bytes, uint32_t k, uint64_t* bytes) {
    (void)n_reads;
    if (!bytes || k < 2 || k > 32 * GERBIL_MAX_W || n_bytes >= (1ull << 40)) return GERBIL_EINVAL;
    *bytes = enc_layout(n_bytes, nullptr, nullptr);
    return GERBIL_OK;
}

int32_t gerbil_encode(const uint8_t* ascii, const uint64_t* offsets, uint64_t n_reads, uint64_t n_bytes, uint32_t k,
                      void* ws, uint64_t ws_bytes, gerbil_encoded* out, hipStream_t stream) {
    if (!out || !ws || !offsets || (n_bytes && !ascii)) return GERBIL_EINVAL;
    if (k < 2 || k > 32 * GERBIL_MAX_W || n_bytes >= (1ull << 40)) return GERBIL_EINVAL;
    if (((uintptr_t)ws) & (kAlign - 1)) return GERBIL_EINVAL;
    EncLayout L;
    if (enc_layout(n_bytes, ws, &L) > ws_bytes) return GERBIL_EINVAL;
    const uint64_t n_words = (n_bytes + 31) / 32, n_mask = (n_bytes + 63) / 64;
    memset(out, 0, sizeof(*out));
    out->n_reads = n_reads;
    out->n_bytes = n_bytes;
    out->k = k;
    out->n_words = n_words;
    out->n_mask = n_mask;
    out->packed = L.packed_alloc + 1;
    out->valid = L.valid;
    out->read_start = L.read_start;
    out->kmer_ok = L.kmer_ok;
    out->n_valid = L.scalars;
    out->status = (uint32_t*)(L.scalars + 1);
    hipError_t e = launch_fill_u64(L.scalars, 4, 0, stream);
    // zero words that no lane of the packing kernel writes: the pads, the last word
    if (e == hipSuccess) e = launch_fill_u64(L.packed_alloc, 1, 0, stream);
    if (e == hipSuccess) e = launch_fill_u64(L.packed_alloc + 1 + (n_words ? n_words - 1 : 0), n_words ? 3 : 2, 0, stream);
    if (e == hipSuccess) e = launch_fill_u64(L.valid + (n_mask ? n_mask - 1 : 0), n_mask ? 2 : 1, 0, stream);
    if (e == hipSuccess) e = launch_fill_u64(L.read_start, n_mask + 1, 0, stream);
    if (e == hipSuccess) e = launch_fill_u64(L.kmer_ok + n_mask, 1, 0, stream);
    if (e == hipSuccess) e = launch_read_starts(offsets, n_reads, n_bytes, L.read_start, out->status, stream);
    if (n_bytes) {
        if (e == hipSuccess) e = launch_pack(ascii, n_bytes, out->packed, L.valid, stream);
        if (e == hipSuccess) e = launch_kmer_ok(L.valid, L.read_start, n_mask, k, L.kmer_ok, out->n_valid, stream);
    }
    return hip_status(e);
}

int32_t gerbil_bin_workspace(const gerbil_encoded* enc, const gerbil_params* p, uint64_t* bytes) {
    int32_t st = check_params(p);
    if (st) return st;
    if (!enc || !bytes || enc->k != p->k) return GERBIL_EINVAL;
    uint64_t cap = p->superm_cap ? p->superm_cap : default_superm_cap(enc->n_bytes, p->k, p->m);
    *bytes = bin_layout(cap, p->n_bins, nullptr, nullptr);
    return GERBIL_OK;
}

int32_t gerbil_bin(const gerbil_encoded* enc, const gerbil_params* p, void* ws, uint64_t ws_bytes, gerbil_bins* out,
                   hipStream_t stream) {
    int32_t st = check_params(p);
    if (st) return st;
    if (!enc || !out || !ws || enc->k != p->k) return GERBIL_EINVAL;
    if (((uintptr_t)ws) & (kAlign - 1)) return GERBIL_EINVAL;
    uint64_t cap = p->superm_cap ? p->superm_cap : default_superm_cap(enc->n_bytes, p->k, p->m);
    BinLayout L;
    if (bin_layout(cap, p->n_bins, ws, &L) > ws_bytes) return GERBIL_EINVAL;
    memset(out, 0, sizeof(*out));
    out->k = p->k;
    out->m = p->m;
    out->n_bins = p->n_bins;
    out->tile = kTile;
    out->cap_superm = cap;
    out->n_bytes = enc->n_bytes;
    out->packed = enc->packed;
    out->desc = L.desc;
    out->bin_off = L.bin_off;
    out->bin_kmers = L.bin_kmers;
    out->n_superm = L.scalars;
    out->status = enc->status;

    BinArgs a;
    a.packed = enc->packed;
    a.kmer_ok = enc->kmer_ok;
    a.n_bytes = enc->n_bytes;
    a.k = p->k;
    a.m = p->m;
    a.n_bins = p->n_bins;
    a.order = p->order;
    a.bin_map = p->bin_map;
    a.rank_table = p->order == GERBIL_ORDER_TABLE ? p->rank_table : nullptr;
    a.cap = cap;
    a.list_cap = cap + kListSlack;
    a.list_desc = L.list_desc;
    a.list_bin = L.list_bin;
    a.list_used = L.scalars + 1;
    a.n_superm = L.scalars;
    a.bin_count = L.bin_count;
    a.bin_fill = L.bin_fill;
    a.bin_off = L.bin_off;
    a.bin_kmers = L.bin_kmers;
    a.desc = L.desc;
    a.status = enc->status;
    hipError_t e = launch_fill_u64(L.scalars, 4, 0, stream);
    if (e == hipSuccess) e = launch_fill_u32(L.bin_count, p->n_bins, 0, stream);
    uint64_t n_tiles = (enc->n_bytes + kTile - 1) / kTile;
    uint64_t g = std::max<uint64_t>(n_tiles, 1);
    if (g > kMaxTileGrid) g = kMaxTileGrid;   // bounds the list's slack (one partial chunk per workgroup)
    if (e == hipSuccess) e = launch_bin(a, (uint32_t)g, (uint32_t)device_cus(), stream);
    return hip_status(e);
}

int32_t gerbil_count_workspace(const gerbil_bins* bins, const gerbil_params* p, uint64_t* bytes,
                               hipStream_t stream) {
    int32_t st = check_params(p);
    if (st) return st;
    if (!bytes || !bins || p->k != bins->k || p->n_bins != bins->n_bins) return GERBIL_EINVAL;
    std::vector<uint64_t> kmers(bins->n_bins);
    if (hipMemcpyAsync(kmers.data(), bins->bin_kmers, 8 * (size_t)bins->n_bins, hipMemcpyDeviceToHost, stream) !=
            hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
        return GERBIL_EDEVICE;
    uint64_t mx = 1;
    for (uint64_t v : kmers) mx = std::max(mx, v);
    const uint32_t W = words_for(p->k);
    if (use_lds(p)) {
        LdsSizing z = lds_sizing(p, bins->n_bytes);
        uint64_t fixed = count_fixed(W, ovf_capacity(p), p->n_bins, false, nullptr, nullptr);
        fixed += lds_fixed(z, nullptr, 0, nullptr);
        *bytes = fixed + (uint64_t)z.Q * slot_words_for(lds_slot_keys(mx, z), p->k) * 8ull + kAlign;
        return GERBIL_OK;
    }
    const uint64_t slots = slots_for(mx, load_of(p));
    *bytes = count_fixed(W, ovf_capacity(p), p->n_bins, p->mode == GERBIL_BATCHED, nullptr, nullptr) +
             (uint64_t)pool_size(p) * pool_table_bytes(slots, W);
    return GERBIL_OK;
}

int32_t gerbil_count(const gerbil_bins* bins, const gerbil_params* p, void* ws, uint64_t ws_bytes, uint64_t* keys,
                     uint32_t* counts, uint64_t cap, gerbil_counted* state, hipStream_t stream) {
    int32_t st = check_params(p);
    if (st) return st;
    if (!bins || !ws || !state || (cap && (!keys || !counts))) return GERBIL_EINVAL;
    if (p->k != bins->k || p->n_bins != bins->n_bins) return GERBIL_EINVAL;
    if (((uintptr_t)ws) & (kAlign - 1)) return GERBIL_EINVAL;
    const uint32_t W = words_for(p->k);
    const uint32_t n_bins = bins->n_bins;
    const bool batched = p->mode == GERBIL_BATCHED;
    const float load = load_of(p);
    const uint64_t ovf_cap = ovf_capacity(p);
    if (use_lds(p)) return count_lds(bins, p, ws, ws_bytes, keys, counts, cap, state, stream);
    const uint32_t Q = pool_size(p);
    CountLayout L;
    const uint64_t fixed = count_fixed(W, ovf_cap, n_bins, batched, ws, &L);
    if (fixed > ws_bytes) return GERBIL_EINVAL;
    // The pool takes the rest of the workspace: Q tables of `slots` slots.
    uint64_t slots = 0;
    {
        uint64_t per_table = (ws_bytes - fixed) / Q;
        uint64_t s_guess = per_table / (8ull * W + 4);
        while (s_guess >= kBucket && pool_table_bytes(s_guess, W) > per_table) s_guess -= s_guess / 64 + 1;
        slots = s_guess - s_guess % kBucket;
    }
    if (slots < kBucket || slots / kBucket > 0xFFFFFFFFull) return GERBIL_EINVAL;

    std::vector<uint64_t> off, kmers;
    uint64_t n_superm = 0;
    hipError_t e = hipSuccess;
    if (!batched) {
        // The plain schedule reads the bin sizes once.
        off.resize(n_bins + 1);
        kmers.resize(n_bins);
        e = hipMemcpyAsync(off.data(), bins->bin_off, 8 * (size_t)(n_bins + 1), hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(kmers.data(), bins->bin_kmers, 8 * (size_t)n_bins, hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipMemcpyAsync(&n_superm, bins->n_superm, 8, hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return GERBIL_EDEVICE;
    }

    memset(state, 0, sizeof(*state));
    state->k = p->k;
    state->W = W;
    state->threshold = p->threshold;
    state->hist_len = kHistInternal;
    state->cap = cap;
    state->overflow_cap = ovf_cap;
    state->n_out = L.scalars;
    state->n_overflow = L.scalars + 1;
    state->max_count = L.scalars + 2;
    state->status = (uint32_t*)(L.scalars + 3);
    state->hist = L.hist;
    state->n_superm = bins->n_superm;
    state->bin_status = bins->status;

    CountArgs a;
    a.packed = bins->packed;
    a.n_bytes = bins->n_bytes;
    a.desc = bins->desc;
    a.k = p->k;
    a.W = W;
    a.threshold = p->threshold;
    a.theta = p->max_probes ? p->max_probes : kDefaultTheta;
    a.canonical = p->canonical;
    a.seed = kHashSeed;
    a.ovf_keys = L.ovf_keys;
    a.ovf_state = L.ovf_state;
    a.ovf_tkeys = L.ovf_tkeys;
    a.ovf_tcnt = L.ovf_tcnt;
    a.ovf_cap = ovf_cap;
    a.n_ovf = state->n_overflow;
    a.out_keys = keys;
    a.out_counts = counts;
    a.cap = cap;
    a.n_out = state->n_out;
    a.hist = L.hist;
    a.max_count = state->max_count;
    a.status = state->status;

    e = launch_fill_u64(L.scalars, 8, 0, stream);
    if (e == hipSuccess) e = launch_fill_u64(L.hist, kHistInternal, 0, stream);
    for (uint32_t j = 0; j < Q && e == hipSuccess; j++) {
        Table t = pool_table(L.pool, slots, W, j);
        e = launch_fill_u64(t.w0, slots, GERBIL_EMPTY, stream);
        if (e == hipSuccess) e = launch_fill_u32(t.cnt, slots, 0, stream);
    }
    if (e != hipSuccess) return GERBIL_EDEVICE;

    if (batched) {
        PersistArgs q;
        q.pool = L.pool;
        q.slots = slots;
        q.Q = Q;
        q.lag = Q / 2;
        q.n_bins = n_bins;
        // threads per workgroup: 256, 512 or 1024 (other values take 256)
        const uint32_t hb = p->block == 512 || p->block == 1024 ? p->block : 256u;
        q.ins_chunk = hb;
        q.cmp_chunk = kCmpChunk;
        q.load = load;
        q.bin_off = bins->bin_off;
        q.bin_kmers = bins->bin_kmers;
        q.order = L.order;
        q.nb = L.nb;
        q.n_ins = L.n_ins;
        q.n_cmp = L.n_cmp;
        q.ins_done = L.ins_done;
        q.cmp_done = L.cmp_done;
        q.seg_code = L.seg_code;
        q.seg_start = L.seg_start;
        q.cursor = L.cursor;
        q.n_superm = bins->n_superm;
        q.superm_cap = bins->cap_superm;
        q.status = state->status;
        e = launch_plan(q, stream);
        uint32_t grid = (uint32_t)device_cus() * persistent_blocks_per_cu(W, hb);
        if (e == hipSuccess && p->timing_events) e = hipEventRecord(p->timing_events[0], stream);
        if (e == hipSuccess) e = launch_count_persistent(a, q, grid, hb, stream);
        if (e == hipSuccess && p->timing_events) e = hipEventRecord(p->timing_events[1], stream);
    } else {
        if (n_superm > bins->cap_superm) return GERBIL_OK;   // reported by gerbil_result as ECAPACITY
        Table t = pool_table(L.pool, slots, W, 0);
        const uint32_t block = p->block ? p->block : kDefaultBlock;
        if (p->timing_events) e = hipEventRecord(p->timing_events[0], stream);
        for (uint32_t b = 0; b < n_bins && e == hipSuccess; b++) {
            uint64_t d0 = off[b], d1 = off[b + 1];
            if (d1 <= d0) continue;
            uint32_t nb = (uint32_t)std::min<uint64_t>(slots_for(kmers[b], load) / kBucket, prev_pow2(slots / kBucket));
            e = launch_count_bin(a, t, nb, d0, d1, block, stream);
            if (e == hipSuccess) e = launch_compact(a, t, nb, stream);
        }
        if (e == hipSuccess && p->timing_events) e = hipEventRecord(p->timing_events[1], stream);
    }
    if (e == hipSuccess) e = launch_overflow(a, stream);
    return hip_status(e);
}

int32_t gerbil_histogram(const gerbil_counted* state, uint64_t* hist, uint32_t len, hipStream_t stream) {
    if (!state || !hist || len < 2 || len > kHistInternal || !state->hist) return GERBIL_EINVAL;
    hipLaunchKernelGGL(k_fold_hist, dim3(1), dim3(256), 0, stream, state->hist, len, hist);
    return hip_status(hipGetLastError());
}

int32_t gerbil_result(const gerbil_encoded* enc, const gerbil_bins* bins, const gerbil_counted* state,
                      gerbil_report* report, hipStream_t stream) {
    if (!report) return GERBIL_EINVAL;
    memset(report, 0, sizeof(*report));
    if (hipStreamSynchronize(stream) != hipSuccess) return GERBIL_EDEVICE;
    uint32_t status = 0, s32 = 0;
    if (enc) {
        if (hipMemcpy(&report->n_valid, enc->n_valid, 8, hipMemcpyDeviceToHost) != hipSuccess) return GERBIL_EDEVICE;
        if (hipMemcpy(&s32, enc->status, 4, hipMemcpyDeviceToHost) != hipSuccess) return GERBIL_EDEVICE;
        status |= s32;
    }
    if (bins) {
        if (hipMemcpy(&report->n_superm, bins->n_superm, 8, hipMemcpyDeviceToHost) != hipSuccess) return GERBIL_EDEVICE;
        if (hipMemcpy(&s32, bins->status, 4, hipMemcpyDeviceToHost) != hipSuccess) return GERBIL_EDEVICE;
        status |= s32;
        if (report->n_superm > bins->cap_superm) status |= ST_SUPERM_CAP;
    }
    if (state) {
        if (hipMemcpy(&report->n_out, state->n_out, 8, hipMemcpyDeviceToHost) != hipSuccess) return GERBIL_EDEVICE;
        if (hipMemcpy(&report->n_overflow, state->n_overflow, 8, hipMemcpyDeviceToHost) != hipSuccess)
            return GERBIL_EDEVICE;
        if (hipMemcpy(&report->max_count, state->max_count, 8, hipMemcpyDeviceToHost) != hipSuccess)
            return GERBIL_EDEVICE;
        if (hipMemcpy(&s32, state->status, 4, hipMemcpyDeviceToHost) != hipSuccess) return GERBIL_EDEVICE;
        status |= s32;
        if (report->n_out > state->cap) status |= ST_OUT_CAP;
        if (report->n_overflow > state->overflow_cap) status |= ST_OVF_CAP;
        if (state->bin_status) {
            if (hipMemcpy(&s32, state->bin_status, 4, hipMemcpyDeviceToHost) != hipSuccess) return GERBIL_EDEVICE;
            status |= s32;
        }
        if (state->n_superm) {
            uint64_t ns = 0;
            if (hipMemcpy(&ns, state->n_superm, 8, hipMemcpyDeviceToHost) != hipSuccess) return GERBIL_EDEVICE;
            if (bins && ns > bins->cap_superm) status |= ST_SUPERM_CAP;
        }
    }
    report->status = status;
    if (status & (ST_SPIN)) return GERBIL_EDEVICE;
    if (status & ST_OFFSETS) return GERBIL_EINVAL;
    if (status & (ST_OUT_CAP | ST_OVF_CAP | ST_SUPERM_CAP | ST_POOL | ST_COUNT_SAT)) return GERBIL_ECAPACITY;
    return GERBIL_OK;
}

}  // extern "C"

extern "C" int32_t gerbil_key_bins(const uint64_t* keys, uint64_t n, const gerbil_params* p, uint32_t* bins,
                                   hipStream_t stream) {
    if (check_params(p) != GERBIL_OK) return check_params(p);
    if (n && (!keys || !bins)) return GERBIL_EINVAL;
    BinArgs a{};
    a.k = p->k;
    a.m = p->m;
    a.n_bins = p->n_bins;
    a.order = p->order;
    a.bin_map = p->bin_map;
    a.rank_table = p->order == GERBIL_ORDER_TABLE ? p->rank_table : nullptr;
    return launch_key_bins(keys, n, a, bins, stream) == hipSuccess ? GERBIL_OK : GERBIL_EDEVICE;
}

extern "C" int32_t gerbil_hll_bins(const gerbil_bins* bins, const gerbil_params* p, uint32_t log2_regs,
                                   uint32_t* regs, hipStream_t stream) {
    const int32_t st = check_params(p);
    if (st) return st;
    if (!bins || !regs || p->k != bins->k || p->n_bins != bins->n_bins) return GERBIL_EINVAL;
    if (log2_regs < 4 || log2_regs > 15) return GERBIL_EINVAL;
    if (!bins->desc || !bins->bin_off || !bins->packed) return GERBIL_EINVAL;
    return launch_hll(bins->packed, bins->n_bytes, bins->desc, bins->bin_off, bins->n_bins, p->k, p->canonical,
                      log2_regs, regs, stream) == hipSuccess
               ? GERBIL_OK
               : GERBIL_EDEVICE;
}

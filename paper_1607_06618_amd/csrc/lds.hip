// LDS sub-table counting (the default table placement).
//
// Phase two of the paper splits the k-mers of a temporary file over several
// hasher threads by a hash of the k-mer, each with its own table
// (Sec. 2.3.2, step 2). Here a hasher is a workgroup and its table lives in
// the 160 KB of LDS of one CU. For every rank (a bin, or a hash slice of a
// very large bin) four stages run:
//   A  count:   every k-mer of the bin is extracted, canonicalised and hashed;
//               the keys of this slice are counted per sub-table (LDS
//               histogram, one global add per sub-table and chunk);
//   S  scan:    prefix of the sub-table sizes -> contiguous key runs;
//   C  scatter: the keys are extracted again and written to their sub-table
//               run (LDS ranks, one global reservation per sub-table and
//               round), so every run is contiguous in HBM;
//   D  count:   one workgroup streams a run through an open-addressing LDS
//               table (Alg. 1: CAS on word 0, publish the other words, add to
//               the counter; theta probes, then the emergency area), then
//               dumps it (threshold, histogram).
// HBM traffic is streaming (keys written once and read once), and all table
// atomics stay inside one CU.
#include "table.h"

namespace gerbil {

constexpr uint32_t kLdsSpin = 1u << 20;     // bounded wait for an unpublished LDS slot
constexpr uint32_t kLdsWait = 1u << 25;     // bounded wait between work items
constexpr uint32_t kNone = 0xFFFFFFFFu;


__device__ __forceinline__ uint32_t slice_of(uint64_t h, uint32_t V) { return fastrange32((uint32_t)(h >> 32), V); }
__device__ __forceinline__ uint32_t sub_of(uint64_t h, uint32_t P) { return fastrange32((uint32_t)h, P); }

// ----------------------------------------------------------------- plan
// One workgroup. Ranks follow the bins in LPT order (largest first); a bin
// with more k-mers than max_sub sub-tables of `target` keys is cut into
// V slices. Queue segment 4*tick + stage holds stage `stage` of rank
// tick - lag[stage], lag = {0, 1, 2, 2 + L}: every dependency of an item is
// in an earlier segment.
__global__ void __launch_bounds__(1024) k_lds_plan(LdsArgs l) {
    __shared__ uint64_t skey[kMaxBins];
    __shared__ uint32_t sval[kMaxBins];
    __shared__ uint64_t part[1024];
    __shared__ uint32_t s_total;
    const uint32_t tid = threadIdx.x, n = l.n_bins;
    uint32_t N = 1;
    while (N < n) N <<= 1;
    for (uint32_t i = tid; i < N; i += 1024) {
        skey[i] = i < n ? l.bin_kmers[i] : 0ull;
        sval[i] = i;
    }
    __syncthreads();
    for (uint32_t size = 2; size <= N; size <<= 1) {
        for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
            for (uint32_t i = tid; i < N / 2; i += 1024) {
                uint32_t lo = 2 * stride * (i / stride) + (i % stride), hi = lo + stride;
                bool desc = (lo & size) == 0;
                bool lo_first = skey[lo] > skey[hi] || (skey[lo] == skey[hi] && sval[lo] < sval[hi]);
                if (desc != lo_first) {
                    uint64_t tk = skey[lo]; skey[lo] = skey[hi]; skey[hi] = tk;
                    uint32_t tv = sval[lo]; sval[lo] = sval[hi]; sval[hi] = tv;
                }
            }
            __syncthreads();
        }
    }
    const bool overfull = *l.n_superm > l.superm_cap;
    const uint64_t per_slice = (uint64_t)l.max_sub * l.target;
    // 1. slices per bin (in LPT order) and their prefix -> first rank of each bin
    auto slices = [&](uint32_t i) -> uint64_t {
        uint64_t km = skey[i];
        uint64_t v = (km + per_slice - 1) / per_slice;
        return v ? v : 1;
    };
    const uint32_t per = (n + 1023) / 1024;
    uint64_t sum = 0;
    for (uint32_t e = 0; e < per; e++) {
        uint32_t i = tid * per + e;
        if (i < n) sum += slices(i);
    }
    part[tid] = sum;
    __syncthreads();
    for (uint32_t off = 1; off < 1024; off <<= 1) {
        uint64_t y = tid >= off ? part[tid - off] : 0ull;
        __syncthreads();
        part[tid] += y;
        __syncthreads();
    }
    const uint64_t n_ranks = part[1023];
    const bool too_many = n_ranks > l.ranks_cap;
    if (tid == 0 && (too_many || overfull)) set_status(l.status, too_many ? ST_POOL : ST_SUPERM_CAP);
    if (!too_many) {
        uint64_t r = tid ? part[tid - 1] : 0ull;
        for (uint32_t e = 0; e < per; e++) {
            uint32_t i = tid * per + e;
            if (i >= n) break;
            uint32_t b = sval[i];
            uint64_t V = slices(i);
            uint64_t nd = l.bin_off[b + 1] - l.bin_off[b];
            uint64_t kest = (skey[i] + V - 1) / V;
            uint64_t P = (kest + l.target - 1) / l.target;
            if (P < 1) P = 1;
            if (P > l.max_sub) P = l.max_sub;
            bool empty = nd == 0 || overfull;
            for (uint64_t v = 0; v < V; v++, r++) {
                l.rank_bin[r] = b;
                l.rank_slice[r] = (uint32_t)v;
                l.rank_nslice[r] = (uint32_t)V;
                l.rank_nsub[r] = empty ? 0u : (uint32_t)P;
                l.rank_nchunk[r] = empty ? 0u : (uint32_t)((nd + l.block - 1) / l.block);
            }
        }
    }
    if (tid == 0) {
        *l.n_ranks = too_many ? 0u : (uint32_t)n_ranks;
        s_total = too_many ? 0u : (uint32_t)n_ranks;
    }
    __threadfence();
    __syncthreads();
    const uint32_t R = s_total;
    // 2. first sub-table of every rank; zero the per-rank state
    const uint32_t rper = (R + 1023) / 1024;
    sum = 0;
    for (uint32_t e = 0; e < rper; e++) {
        uint32_t r = tid * rper + e;
        if (r < R) sum += l.rank_nsub[r];
    }
    part[tid] = sum;
    __syncthreads();
    for (uint32_t off = 1; off < 1024; off <<= 1) {
        uint64_t y = tid >= off ? part[tid - off] : 0ull;
        __syncthreads();
        part[tid] += y;
        __syncthreads();
    }
    const bool sp_over = part[1023] > l.sp_cap;
    if (tid == 0 && sp_over) set_status(l.status, ST_POOL);
    uint64_t base = tid ? part[tid - 1] : 0ull;
    for (uint32_t e = 0; e < rper; e++) {
        uint32_t r = tid * rper + e;
        if (r >= R) break;
        if (sp_over) l.rank_nsub[r] = 0, l.rank_nchunk[r] = 0;
        l.rank_spbase[r] = base;
        l.rank_keys[r] = 0;
        base += l.rank_nsub[r];
        for (int s = 0; s < 4; s++) l.done[4 * r + s] = 0;
    }
    __threadfence();
    __syncthreads();
    const uint64_t n_sp = sp_over ? 0 : part[1023];
    for (uint64_t j = tid; j < n_sp; j += 1024) {
        l.sp_cnt[j] = 0;
        l.sp_cur[j] = 0;
    }
    // 3. queue segments: items per segment, then their prefix, for every
    // queue (a queue holds the items of its ranks, in the same segment order)
    const uint32_t L = l.lag;
    const uint32_t ticks = R + 3 + L;
    const uint32_t ns = 4 * ticks;
    const uint32_t NQ = l.n_queues;
    const uint32_t lag[4] = {0u, 1u, 2u, 2u + L};
    const uint32_t sper = (ns + 1023) / 1024;
    auto items = [&](uint32_t seg, uint32_t q) -> uint64_t {
        uint32_t st = seg & 3, tick = seg >> 2;
        if (tick < lag[st]) return 0;
        uint32_t r = tick - lag[st];
        if (r >= R || r % NQ != q) return 0;
        uint32_t nc = l.rank_nchunk[r];
        if (nc == 0) return 0;
        switch (st) {
            case 0: return nc;
            case 1: return 1;
            case 2: return nc;
            default: return l.rank_nsub[r];
        }
    };
    for (uint32_t q = 0; q < NQ; q++) {
        uint64_t* start = l.seg_start + (uint64_t)q * (ns + 1);
        sum = 0;
        for (uint32_t e = 0; e < sper; e++) {
            uint32_t j = tid * sper + e;
            if (j < ns) sum += items(j, q);
        }
        part[tid] = sum;
        __syncthreads();
        for (uint32_t off = 1; off < 1024; off <<= 1) {
            uint64_t y = tid >= off ? part[tid - off] : 0ull;
            __syncthreads();
            part[tid] += y;
            __syncthreads();
        }
        uint64_t run = tid ? part[tid - 1] : 0ull;
        for (uint32_t e = 0; e < sper; e++) {
            uint32_t j = tid * sper + e;
            if (j < ns) {
                start[j] = run;
                run += items(j, q);
            }
        }
        if (tid == 1023) {
            start[ns] = part[1023];
            l.cursor[q * kCursorStride] = 0;
        }
        __syncthreads();   // part[] is read above before the next queue's sums overwrite it
    }
    if (tid == 0) *l.n_seg = ns;
}

hipError_t launch_lds_plan(const LdsArgs& l, hipStream_t s) {
    hipLaunchKernelGGL(k_lds_plan, dim3(1), dim3(1024), 0, s, l);
    return hipGetLastError();
}

// ---------------------------------------------------------- LDS layout
struct Lds {
    uint32_t* hist;     // [kLdsHist] count-of-counts, flushed at the end of the kernel
    uint32_t* probes;   // [kProbeHist] inserts by settling probe (only with LdsArgs::probe_hist)
    uint32_t* flag;     // one word for block-wide votes (last word of the reserved region)
    uint8_t* u;         // union region, carved per stage
};
__device__ __forceinline__ Lds lds_carve(uint8_t* base) {
    Lds x;
    x.hist = (uint32_t*)base;
    x.probes = (uint32_t*)(base + kProbeHistAt);
    x.flag = (uint32_t*)(base + kLdsReserved - 4);
    x.u = base + kLdsReserved;
    return x;
}

// Descriptor chunk `chunk` of bin b, one descriptor per thread, with every
// super-mer cut into segments of at most L k-mers: sdesc[d] is descriptor d,
// sgpre[d] the first segment of d (sgpre[B] = number of segments).
template <uint32_t B>
__device__ __forceinline__ uint32_t load_chunk_seg(const CountArgs& a, const LdsArgs& l, uint32_t b, uint32_t chunk,
                                                   uint32_t L, uint64_t* sdesc, uint32_t* sgpre, uint32_t* wsum) {
    const uint32_t tid = threadIdx.x;
    const uint64_t d_end = l.bin_off[b + 1];
    const uint64_t i = l.bin_off[b] + (uint64_t)chunk * B + tid;
    const uint64_t d = i < d_end ? a.desc[i] : 0ull;
    const uint32_t n = (uint32_t)(d & 0xFFFFFFu);
    uint32_t total;
    const uint32_t pre = block_excl_scan((n + L - 1) / L, wsum, total);
    sdesc[tid] = d;
    sgpre[tid] = pre;
    if (tid == 0) sgpre[B] = total;
    __syncthreads();
    return total;
}

// A segment of consecutive k-mers of one super-mer, rolled one base at a time
// (Sec. 2.3.2 splitter step): the first k-mer is read from the packed reads,
// every following one shifts one base into the forward key and its
// complement into the reverse-complement key. A segment adds at most 32 new
// bases, all inside the two packed words read at its start, so rolling never
// waits for memory.

template <int W>
struct Segment {
    uint64_t fw[W], rc[W];
    int64_t p;         // position of the current k-mer
    uint32_t len;      // k-mers in the segment
    int64_t q;         // packed word holding the next base to shift in
    uint64_t cur, nxt;
    bool ok;
};

// The packed words a segment needs, fetched without being used: the bases of
// its first k-mer and the bases it rolls in lie in the W + 2 words from the
// one holding its first base. Kept apart from seg_build so that the fetch
// of the next segment can be issued while the current one is still in use.
template <int W>
struct SegRaw {
    uint64_t w[W + 2];
    int64_t p;      // position of the first k-mer
    uint32_t len;   // k-mers in the segment
    bool ok;
};

template <int W, uint32_t B>
__device__ __forceinline__ void seg_fetch(const CountArgs& a, const uint64_t* sdesc, const uint32_t* sgpre, uint32_t sg,
                                          uint32_t L, SegRaw<W>& r) {
    uint32_t lo = 0, hi = B;   // last descriptor whose first segment is <= sg
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (sgpre[mid] <= sg) lo = mid; else hi = mid;
    }
    const uint64_t d = sdesc[lo];
    const int64_t start = (int64_t)(d >> 24);
    const uint32_t n = (uint32_t)(d & 0xFFFFFFu);
    const uint32_t off = (sg - sgpre[lo]) * L;
    r.p = start + off;
    r.len = n - off < L ? n - off : L;
    r.ok = start >= 0 && (uint64_t)(r.p + r.len - 1) + a.k <= a.n_bytes;
    if (!r.ok) {
        set_status(a.status, ST_SPIN);   // a corrupt descriptor must not read out of range
        return;
    }
    // the packed stream has two zero words past word (n_bytes-1)/32: indexes are clamped to the last
    const int64_t q0 = r.p >> 5, last = (int64_t)((a.n_bytes + 31) >> 5) + 1;
#pragma unroll
    for (int j = 0; j < W + 2; j++) r.w[j] = a.packed[q0 + j < last ? q0 + j : last];
}

// Forward key, reverse-complement key and rolling words of a fetched segment,
// from registers only. Word i < W-1 of the reverse complement is the
// reverse complement of the 32 forward bases ending 32i bases before the end
// (the last 32 - r bases of forward word W-2-i followed by the first r of
// word W-1-i, r = k - 32(W-1)); its last word is that of the first r bases.
template <int W>
__device__ __forceinline__ void seg_build(const SegRaw<W>& r, uint32_t k, Segment<W>& g) {
    g.p = r.p;
    g.len = r.len;
    g.ok = r.ok;
    const uint32_t o = (uint32_t)(r.p & 31);
    const uint32_t rb = k - 32u * (W - 1), sh = 2u * (32u - rb);
    const uint64_t tmask = rb == 32 ? ~0ull : ((1ull << (2 * rb)) - 1ull);
#pragma unroll
    for (int i = 0; i < W; i++) {
        const uint64_t x = o ? ((r.w[i] << (2 * o)) | (r.w[i + 1] >> (64 - 2 * o))) : r.w[i];
        g.fw[i] = (i == W - 1 && sh) ? (x >> sh) : x;
    }
    if (W == 1) {
        g.rc[0] = revcomp32(sh ? (g.fw[0] << sh) : g.fw[0]) & tmask;
    } else {
#pragma unroll
        for (int i = 0; i + 1 < W; i++) {
            uint64_t x;
            if (rb == 32) x = g.fw[W - 1 - i];
            else if (i == 0) x = (g.fw[W - 2] << (2 * rb)) | g.fw[W - 1];
            else x = (g.fw[W - 2 - i] << (2 * rb)) | (g.fw[W - 1 - i] >> (64 - 2 * rb));
            g.rc[i] = revcomp32(x);
        }
        g.rc[W - 1] = revcomp32(g.fw[0]) & tmask;
    }
    g.q = (r.p + (int64_t)k) >> 5;   // word of the next base to roll in: word W-1 or W of the fetch
    const bool hiw = ((o + k) >> 5) == (uint32_t)W;
    g.cur = hiw ? r.w[W] : r.w[W - 1];
    g.nxt = hiw ? r.w[W + 1] : r.w[W];
}

// Open a segment at once. Short keys go through seg_fetch/seg_build (W + 2
// loads); longer keys read each 32-base window directly, which keeps fewer
// words live at a time.
template <int W, uint32_t B>
__device__ __forceinline__ void seg_open(const CountArgs& a, const uint64_t* sdesc, const uint32_t* sgpre, uint32_t sg,
                                         uint32_t L, Segment<W>& g) {
    if (W <= 3) {
        SegRaw<W> r;
        seg_fetch<W, B>(a, sdesc, sgpre, sg, L, r);
        if (r.ok) seg_build<W>(r, a.k, g);
        else g.ok = false;
        return;
    }
    uint32_t lo = 0, hi = B;   // last descriptor whose first segment is <= sg
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (sgpre[mid] <= sg) lo = mid; else hi = mid;
    }
    const uint64_t d = sdesc[lo];
    const int64_t start = (int64_t)(d >> 24);
    const uint32_t n = (uint32_t)(d & 0xFFFFFFu);
    const uint32_t off = (sg - sgpre[lo]) * L;
    g.p = start + off;
    g.len = n - off < L ? n - off : L;
    g.ok = start >= 0 && (uint64_t)(g.p + g.len - 1) + a.k <= a.n_bytes;
    if (!g.ok) {
        set_status(a.status, ST_SPIN);   // a corrupt descriptor must not read out of range
        return;
    }
    extract_kmer<W>(a.packed, g.p, a.k, g.fw, g.rc);
    g.q = (g.p + (int64_t)a.k) >> 5;   // p + k <= n_bytes, so q + 1 is at most a padded word
    g.cur = a.packed[g.q];
    g.nxt = a.packed[g.q + 1];
}

// Shift in base b (code 0..3) at the end of the forward key and its
// complement at the front of the reverse-complement key.
template <int W>
__device__ __forceinline__ void roll_base(uint64_t (&fw)[W], uint64_t (&rc)[W], uint32_t b, uint32_t k) {
    const uint32_t rb = k - 32u * (W - 1);   // bases in the last word
    const uint64_t tail_mask = rb == 32 ? ~0ull : ((1ull << (2 * rb)) - 1ull);
#pragma unroll
    for (int i = 0; i + 1 < W; i++) {
        uint64_t top_next = (i + 2 < W) ? (fw[i + 1] >> 62) : (fw[W - 1] >> (2 * rb - 2));
        fw[i] = (fw[i] << 2) | top_next;
    }
    fw[W - 1] = ((fw[W - 1] << 2) | b) & tail_mask;
    if (W == 1) {
        rc[0] = (rc[0] >> 2) | ((uint64_t)(3u - b) << (2 * rb - 2));
    } else {
        rc[W - 1] = (rc[W - 1] >> 2) | ((rc[W - 2] & 3ull) << (2 * rb - 2));
#pragma unroll
        for (int i = W - 2; i >= 1; i--) rc[i] = (rc[i] >> 2) | ((rc[i - 1] & 3ull) << 62);
        rc[0] = (rc[0] >> 2) | ((uint64_t)(3u - b) << 62);
    }
}

// Advance to the next k-mer of the segment.
template <int W>
__device__ __forceinline__ void seg_step(uint32_t k, Segment<W>& g) {
    g.p += 1;
    const int64_t x = g.p + (int64_t)k - 1;   // the base that enters the window
    if ((x >> 5) != g.q) {
        g.q += 1;
        g.cur = g.nxt;
    }
    const uint32_t b = (uint32_t)((g.cur >> (62 - 2 * (x & 31))) & 3ull);
    roll_base<W>(g.fw, g.rc, b, k);
}

// The last word of key i of a slot, stored in `tb` bytes (plain store).
__device__ __forceinline__ void store_tail(uint8_t* tail, uint64_t i, uint64_t v, uint32_t tb) {
    switch (tb) {
        case 1: tail[i] = (uint8_t)v; break;
        case 2: ((uint16_t*)tail)[i] = (uint16_t)v; break;
        case 4: ((uint32_t*)tail)[i] = (uint32_t)v; break;
        default: ((uint64_t*)tail)[i] = v; break;
    }
}

// Last words of K keys (run positions off + ix[e]); one uniform branch on the width.
template <int K, int W>
__device__ __forceinline__ void load_tails(const uint8_t* tail, uint64_t off, const uint64_t (&ix)[K], uint32_t tb,
                                           uint64_t (&key)[K][W]) {
    switch (tb) {
        case 1:
#pragma unroll
            for (int e = 0; e < K; e++) key[e][W - 1] = ld_dev(tail + off + ix[e]);
            break;
        case 2:
#pragma unroll
            for (int e = 0; e < K; e++) key[e][W - 1] = ld_dev((const uint16_t*)tail + off + ix[e]);
            break;
        case 4:
#pragma unroll
            for (int e = 0; e < K; e++) key[e][W - 1] = ld_dev((const uint32_t*)tail + off + ix[e]);
            break;
        default:
#pragma unroll
            for (int e = 0; e < K; e++) key[e][W - 1] = ld_dev((const uint64_t*)tail + off + ix[e]);
            break;
    }
}

// True on every thread if v is true on any thread (an LDS word, not static
// shared memory: the kernels already take all 160 KB of dynamic LDS).
__device__ __forceinline__ bool block_any(bool v, uint32_t* flag) {
    if (threadIdx.x == 0) *flag = 0u;
    __syncthreads();
    if (v) *flag = 1u;
    __syncthreads();
    return *flag != 0u;
}

// Exclusive prefix of cnt[0..n) into pre[0..n) by the whole block; returns the total.
template <uint32_t B>
__device__ __forceinline__ uint32_t block_scan_array(const uint32_t* cnt, uint32_t* pre, uint32_t n, uint32_t* wsum) {
    const uint32_t per = (n + B - 1) / B;
    const uint32_t j0 = threadIdx.x * per;
    uint32_t sum = 0;
    for (uint32_t e = 0; e < per; e++)
        if (j0 + e < n) sum += cnt[j0 + e];
    uint32_t total;
    uint32_t run = block_excl_scan(sum, wsum, total);
    for (uint32_t e = 0; e < per; e++)
        if (j0 + e < n) {
            pre[j0 + e] = run;
            run += cnt[j0 + e];
        }
    return total;
}

// Round size of the scatter stage: R keys per thread (one segment of at most
// R k-mers), staged in 96 KB of LDS at most.
template <int W>
struct ScatterRound { static constexpr int R = W == 1 ? 8 : W == 2 ? 5 : W == 3 ? 4 : W == 4 ? 3 : W == 5 ? 2 : 1; };

// LDS of the chunk stages: descriptors, segment prefixes and scan scratch.
template <uint32_t B>
constexpr uint32_t chunk_header() { return 8 * B + 4 * (B + 4) + 4 * 32; }

struct ChunkLds {
    uint64_t* sdesc;
    uint32_t* sgpre;
    uint32_t* wsum;
    uint8_t* rest;
};
template <uint32_t B>
__device__ __forceinline__ ChunkLds chunk_lds(const Lds& s) {
    ChunkLds c;
    c.sdesc = (uint64_t*)s.u;
    c.sgpre = (uint32_t*)(s.u + 8 * B);
    c.wsum = c.sgpre + B + 4;
    c.rest = (uint8_t*)(c.wsum + 32);
    return c;
}

// Stage A: keys of this slice per sub-table. One segment of up to 32 k-mers
// per thread and round, so all lanes read their first k-mer together.
template <int W, uint32_t B>
__device__ void stage_count(const CountArgs& a, const LdsArgs& l, const Lds& s, uint32_t r, uint32_t chunk) {
    const uint32_t tid = threadIdx.x;
    const uint64_t kx = stored_xor(a.canonical, a.k);
    const uint32_t b = l.rank_bin[r], v = l.rank_slice[r], V = l.rank_nslice[r], P = l.rank_nsub[r];
    const ChunkLds c = chunk_lds<B>(s);
    static_assert(chunk_header<B>() + 4 * LdsShape<B>::max_sub <= LdsShape<B>::bytes - kLdsReserved,
                  "count stage exceeds the LDS budget");
    uint32_t* hist = (uint32_t*)c.rest;
    for (uint32_t j = tid; j < P; j += B) hist[j] = 0;
    // with sampling, segments are short and only every l.sample-th one is walked
    const uint32_t smp = l.sample > 1 ? l.sample : 1u, L = smp > 1 ? sample_seg_len(smp) : kSegMax;
    const uint32_t S = load_chunk_seg<B>(a, l, b, chunk, L, c.sdesc, c.sgpre, c.wsum);
    for (uint32_t sg = tid * smp; sg < S; sg += B * smp) {
        Segment<W> g;
        seg_open<W, B>(a, c.sdesc, c.sgpre, sg, L, g);
        if (!g.ok) continue;
        for (uint32_t j = 0; j < g.len; j++) {
            if (j) seg_step<W>(a.k, g);
            uint64_t key[W];
            canonical_of<W>(g.fw, g.rc, key, a.canonical);
            key[0] ^= kx;
            const uint64_t h = key_hash<W>(key, a.seed);
            if (V > 1 && slice_of(h, V) != v) continue;
            atomicAdd(&hist[sub_of(h, P)], 1u);
        }
    }
    __syncthreads();
    const uint64_t sb = l.rank_spbase[r];
    for (uint32_t j = tid; j < P; j += B)
        if (hist[j]) add_dev(&l.sp_cnt[sb + j], hist[j]);
}

// Stage S: sub-table runs of the rank (one workgroup).
template <uint32_t B>
__device__ void stage_scan(const CountArgs& a, const LdsArgs& l, const Lds& s, uint32_t r) {
    const uint32_t tid = threadIdx.x, P = l.rank_nsub[r];
    const uint64_t sb = l.rank_spbase[r];
    uint64_t* part = (uint64_t*)s.u;
    const uint32_t per = (P + B - 1) / B;
    uint64_t sum = 0;
    // sampled counts -> run capacities (sp_cnt then holds the capacity)
    for (uint32_t e = 0; e < per; e++) {
        uint32_t j = tid * per + e;
        if (j < P) {
            uint64_t cap = run_capacity(ld_dev(&l.sp_cnt[sb + j]), l.sample);
            if (cap > 0xFFFFFFFFull) cap = 0xFFFFFFFFull;
            st_dev(&l.sp_cnt[sb + j], (uint32_t)cap);
            sum += cap;
        }
    }
    part[tid] = sum;
    __syncthreads();
    for (uint32_t off = 1; off < B; off <<= 1) {
        uint64_t y = tid >= off ? part[tid - off] : 0ull;
        __syncthreads();
        part[tid] += y;
        __syncthreads();
    }
    uint64_t run = tid ? part[tid - 1] : 0ull;
    for (uint32_t e = 0; e < per; e++) {
        uint32_t j = tid * per + e;
        if (j < P) {
            st_dev(&l.sp_off[sb + j], run);
            run += ld_dev(&l.sp_cnt[sb + j]);
            st_dev(&l.sp_cur[sb + j], 0u);
        }
    }
    if (tid == 0) {
        st_dev(&l.rank_keys[r], part[B - 1]);
        if (part[B - 1] > l.slot_keys) set_status(a.status, ST_POOL);
    }
}

// Stage C: write the keys of this slice into their sub-table runs. Per round
// every thread takes one segment of up to R k-mers (keys held in registers);
// the round's keys are grouped by sub-table in LDS, one global reservation is
// made per sub-table, and each run is written as consecutive words.
template <int W, uint32_t B>
__device__ void stage_scatter(const CountArgs& a, const LdsArgs& l, const Lds& s, uint32_t r, uint32_t chunk) {
    constexpr int R = ScatterRound<W>::R;
    const uint32_t tid = threadIdx.x;
    const uint64_t kx = stored_xor(a.canonical, a.k);
    const uint32_t b = l.rank_bin[r], v = l.rank_slice[r], V = l.rank_nslice[r], P = l.rank_nsub[r];
    const uint64_t sb = l.rank_spbase[r];
    uint64_t* slot = l.keys + (uint64_t)(r % l.Q) * l.slot_words;
    uint8_t* tail = (uint8_t*)(slot + (uint64_t)(W - 1) * l.slot_keys);
    const ChunkLds c = chunk_lds<B>(s);
    static_assert(chunk_header<B>() + 3 * 4 * LdsShape<B>::max_sub + (uint64_t)R * 8 * W * B <= LdsShape<B>::bytes - kLdsReserved,
                  "scatter stage exceeds the LDS budget");
    uint32_t* cnt = (uint32_t*)c.rest;
    uint32_t* lp = cnt + LdsShape<B>::max_sub;
    uint32_t* dst = lp + LdsShape<B>::max_sub;   // run start of this round, relative to the key slot
    uint64_t* buf = (uint64_t*)(dst + LdsShape<B>::max_sub);
    for (uint32_t j = tid; j < P; j += B) cnt[j] = 0;
    const uint32_t S = load_chunk_seg<B>(a, l, b, chunk, R, c.sdesc, c.sgpre, c.wsum);
    const uint32_t rounds = (S + B - 1) / B;
    // For short keys the next round's words are fetched while this round is
    // written out; longer keys (more registers per key) open at round start.
    constexpr bool kAhead = W <= 3;
    // A last key word of at most 16 bases (2r <= 32 bits) carries the key's
    // sub-table in its top 16 bits while it is staged in LDS, so the store
    // loop reads the sub-table of a sorted position instead of searching lp[].
    const bool tagged = a.k - 32u * (W - 1) <= 16u;
    constexpr uint64_t kTagMask = (1ull << 48) - 1;
    SegRaw<W> raw;
    raw.ok = false;
    if (kAhead && tid < S) seg_fetch<W, B>(a, c.sdesc, c.sgpre, tid, R, raw);
    for (uint32_t round = 0; round < rounds; round++) {
        uint64_t key[R][W];
        uint32_t sp[R], rk[R];
#pragma unroll
        for (int e = 0; e < R; e++) sp[e] = kNone;
        const uint32_t sg = round * B + tid;
        if (sg < S) {
            Segment<W> g;
            g.ok = false;
            if (kAhead) {
                if (raw.ok) seg_build<W>(raw, a.k, g);
            } else {
                seg_open<W, B>(a, c.sdesc, c.sgpre, sg, R, g);
            }
            if (g.ok) {
#pragma unroll
                for (int e = 0; e < R; e++) {
                    if ((uint32_t)e < g.len) {
                        if (e) seg_step<W>(a.k, g);
                        canonical_of<W>(g.fw, g.rc, key[e], a.canonical);
                        key[e][0] ^= kx;
                        const uint64_t h = key_hash<W>(key[e], a.seed);
                        if (V == 1 || slice_of(h, V) == v) {
                            sp[e] = sub_of(h, P);
                            rk[e] = atomicAdd(&cnt[sp[e]], 1u);
                        }
                    }
                }
            }
        }
        __syncthreads();
        const uint32_t T = block_scan_array<B>(cnt, lp, P, c.wsum);
        __syncthreads();   // every lp[] written (and every cnt[] read) before keys are placed or counts reset
        for (uint32_t j = tid; j < P; j += B) {
            const uint32_t n = cnt[j];
            if (n) {
                const uint32_t gsub = add_dev(&l.sp_cur[sb + j], n);
                const uint32_t cap = ld_dev(&l.sp_cnt[sb + j]);
                dst[j] = (uint32_t)(ld_dev(&l.sp_off[sb + j]) + gsub);
                cnt[j] = gsub >= cap ? 0u : (cap - gsub < n ? cap - gsub : n);   // keys that fit the run
            }
        }
#pragma unroll
        for (int e = 0; e < R; e++) {
            if (sp[e] == kNone) continue;
            const uint32_t pos = lp[sp[e]] + rk[e];
#pragma unroll
            for (int w = 0; w + 1 < W; w++) buf[(uint64_t)pos * W + w] = key[e][w];
            buf[(uint64_t)pos * W + W - 1] = tagged ? key[e][W - 1] | ((uint64_t)sp[e] << 48) : key[e][W - 1];
        }
        if (kAhead) {
            raw.ok = false;
            if (sg + B < S) seg_fetch<W, B>(a, c.sdesc, c.sgpre, sg + B, R, raw);
        }
        __syncthreads();
        // stores only: nothing in this loop waits for memory (a returning
        // atomic here would make every iteration wait for all earlier stores)
        uint32_t spilled = 0;
        for (uint32_t i = tid; i < T; i += B) {
            const uint64_t lw = buf[(uint64_t)i * W + W - 1];
            uint32_t lo = 0;   // sub-table of sorted position i
            if (tagged) {
                lo = (uint32_t)(lw >> 48);
            } else {
                uint32_t hi = P;   // last sub-table whose run starts at or before i
                while (hi - lo > 1) {
                    uint32_t mid = (lo + hi) >> 1;
                    if (lp[mid] <= i) lo = mid; else hi = mid;
                }
            }
            const uint32_t q = i - lp[lo];
            if (q < cnt[lo]) {
                const uint64_t gpos = (uint64_t)dst[lo] + q;
                if (gpos < l.slot_keys) {
                    // plain stores: merged in L2 and written back once, by the
                    // release fence that ends the item (see the persistent loop)
#pragma unroll
                    for (int w = 0; w + 1 < W; w++)
                        slot[(uint64_t)w * l.slot_keys + gpos] = buf[(uint64_t)i * W + w];
                    store_tail(tail, gpos, tagged ? lw & kTagMask : lw, l.tail_bytes);
                } else {
                    set_status(a.status, ST_POOL);
                }
            } else {
                spilled = 1;
            }
        }
        // keys past the end of their run (runs are sized from a sample): emergency area
        if (block_any(spilled != 0, s.flag)) {
            for (uint32_t i = tid; i < T; i += B) {
                const uint64_t lw = buf[(uint64_t)i * W + W - 1];
                uint32_t lo = 0;
                if (tagged) {
                    lo = (uint32_t)(lw >> 48);
                } else {
                    uint32_t hi = P;
                    while (hi - lo > 1) {
                        uint32_t mid = (lo + hi) >> 1;
                        if (lp[mid] <= i) lo = mid; else hi = mid;
                    }
                }
                if (i - lp[lo] < cnt[lo]) continue;
                uint64_t key[W];
#pragma unroll
                for (int w = 0; w + 1 < W; w++) key[w] = buf[(uint64_t)i * W + w];
                key[W - 1] = tagged ? lw & kTagMask : lw;
                overflow_push<W>(a, key);
                if (l.probe_hist) atomicAdd(&s.probes[0], 1u);
            }
        }
        __syncthreads();
        for (uint32_t j = tid; j < P; j += B) cnt[j] = 0;
        __syncthreads();   // counts cleared before the next round adds to them
    }
}

// Alg. 1 in an LDS table of C slots (structure of arrays) for the K keys a
// lane holds, of which the first n are valid. One probe per loop iteration,
// and a lane that settles a key starts its next key in the same iteration:
// a wave then runs about as many iterations as its busiest lane has probes
// in all, instead of, key after key, as many as its slowest lane needs for
// that key. A probe reads the slot's probe word, counter and other words in
// one batch: the wave's LDS accesses are performed in order, and a claimer
// writes the other words before it raises the counter from zero, so a
// counter found non-zero guarantees that the words read after it are the
// slot's key. A slot found claimed but not yet published, or lost to
// another claimer, is probed again in the next iteration. Keys whose theta
// probes fail, and keys whose stored first word is the empty-slot marker
// (never stored), go to the emergency area.
//
// Slot layouts (PK): unpacked, probe words w0[C], the other words rest[(W-1) C]
// and 32-bit counters cnt[C]; packed (W >= 2 and a last word of at most 16
// bases), w0[C], the middle words rest[(W-2) C] and one 64-bit word per slot
// holding the last key word in its high half and the counter in its low half
// (tc[C]): 8W bytes a slot instead of 8W + 4, and one read fewer per probe.
template <int K, int W, bool PK>
__device__ __forceinline__ void lds_insert_all(const CountArgs& a, uint64_t* w0, uint64_t* rest, uint32_t* cnt,
                                               uint64_t* tc, uint32_t C, uint32_t theta, uint64_t (&key)[K][W],
                                               uint32_t n, uint32_t* probes) {
    // C is prime and 1 <= step < C: double hashing visits theta distinct slots.
    // The sub-table is chosen by the top bits of h's low half and the slice by
    // the top bits of its high half, so the slot and the step take bits 0-19
    // and 32-51, which neither choice depends on.
    uint32_t sl[K], st[K];
#pragma unroll
    for (int e = 0; e < K; e++) {
        const uint64_t h = key_hash<W>(key[e], a.seed);
        st[e] = 1u + fastrange32((uint32_t)((h >> 32) << 12), C - 1);
        sl[e] = fastrange32((uint32_t)(h << 12), C);
    }
    constexpr int RW = PK ? (W > 2 ? W - 2 : 1) : (W > 1 ? W - 1 : 1);   // words read after the counter
    constexpr int NR = PK ? W - 2 : W - 1;                                 // of which in use
    uint32_t t = 0, spins = 0;
    while (__ballot(n > 0) != 0ull) {
        if (n > 0) {
            bool settled = false;
            uint32_t pb = 0;   // probe bucket of the key when it settles (probe statistic)
            if (key[0][0] == GERBIL_EMPTY) {
                overflow_push<W>(a, key[0]);
                settled = true;
            } else {
                pb = t + 1 < kProbeHist - 1 ? t + 1 : kProbeHist - 1;
                const uint32_t s = sl[0];
                const uint64_t cur = __hip_atomic_load(w0 + s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                bool published = true;
                uint64_t ctc = 0;
                uint64_t rw[RW];
                if (W > 1) {
                    if (PK) {
                        ctc = __hip_atomic_load(tc + s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                        published = ctc != 0;
                    } else {
                        published = __hip_atomic_load(cnt + s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) != 0;
                    }
                    asm volatile("" ::: "memory");   // the other words are read after the counter
#pragma unroll
                    for (int i = 0; i < NR; i++)
                        rw[i] = __hip_atomic_load(rest + (uint32_t)i * C + s, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_WORKGROUP);
                }
                bool again = false;   // same slot next iteration
                if (cur == GERBIL_EMPTY) {
                    uint64_t exp = GERBIL_EMPTY;
                    __hip_atomic_compare_exchange_strong(w0 + s, &exp, key[0][0], __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_WORKGROUP);
                    if (exp == GERBIL_EMPTY) {
#pragma unroll
                        for (int i = 0; i < NR; i++) rest[(uint32_t)i * C + s] = key[0][i + 1];
                        if (PK) {
                            // the last word and a count of one, published together
                            if (NR > 0) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                            __hip_atomic_store(tc + s, (key[0][W - 1] << 32) | 1ull, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_WORKGROUP);
                        } else {
                            if (W > 1) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                            __hip_atomic_fetch_add(cnt + s, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                        }
                        settled = true;
                    } else {
                        again = true;
                    }
                } else if (cur == key[0][0]) {
                    bool eq = published;
#pragma unroll
                    for (int i = 0; i < NR; i++) eq &= rw[i] == key[0][i + 1];
                    if (PK) eq &= (ctc >> 32) == key[0][W - 1];
                    if (eq) {
                        // a run holds fewer than 2^32 keys, so a count cannot wrap; a packed
                        // slot's counter is the low 32-bit half of its word (a 32-bit add
                        // costs half of a 64-bit one in LDS)
                        if (PK)
                            __hip_atomic_fetch_add((uint32_t*)(tc + s), 1u, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_WORKGROUP);
                        else
                            __hip_atomic_fetch_add(cnt + s, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                        settled = true;
                    } else if (!published) {
                        again = true;
                        if (++spins > kLdsSpin) {
                            set_status(a.status, ST_SPIN);
                            settled = true;
                        }
                    }
                }
                if (!settled && !again) {
                    if (++t >= theta) {
                        overflow_push<W>(a, key[0]);
                        settled = true;
                        pb = kProbeHist - 1;
                    } else {
                        const uint32_t x = s + st[0];
                        sl[0] = x >= C ? x - C : x;
                    }
                }
            }
            if (settled) {
                if (probes) atomicAdd(&probes[pb], 1u);
                n--;
                t = 0;
                spins = 0;
#pragma unroll
                for (int e = 0; e + 1 < K; e++) {
#pragma unroll
                    for (int i = 0; i < W; i++) key[e][i] = key[e + 1][i];
                    sl[e] = sl[e + 1];
                    st[e] = st[e + 1];
                }
            }
        }
    }
}

// Keys loaded per thread before they are inserted (independent loads in
// flight): enough that a sub-table filled to its default target (0.8 of the
// slots) is loaded in one batch.
template <int W, bool PK>
struct TableBatch {
    static constexpr int K = lds_table_batch(W);
};

// Stage D: count one sub-table in LDS, then dump it.
template <int W, uint32_t B, bool PK>
__device__ void stage_table(const CountArgs& a, const LdsArgs& l, const Lds& s, uint32_t r, uint32_t j,
                            uint32_t& wmax) {
    constexpr int K = TableBatch<W, PK>::K;
    const uint32_t tid = threadIdx.x;
    const uint32_t C = l.table_slots;
    uint64_t* w0 = (uint64_t*)s.u;
    uint64_t* rest = w0 + C;
    // packed: tc[C] after the middle words; unpacked: cnt[C] after the other words
    uint64_t* tc = rest + (uint64_t)(W >= 2 ? W - 2 : 0) * C;
    uint32_t* cnt = (uint32_t*)(rest + (uint64_t)(W - 1) * C);
    uint32_t* wsum = PK ? (uint32_t*)(tc + C) + 1 : cnt + C + 1;
    uint64_t* s_base = (uint64_t*)(((uintptr_t)(wsum + 32) + 7) & ~(uintptr_t)7);
    const uint64_t sb = l.rank_spbase[r];
    const uint32_t n_put = ld_dev(&l.sp_cur[sb + j]), n_cap = ld_dev(&l.sp_cnt[sb + j]);
    const uint64_t n = n_put < n_cap ? n_put : n_cap;   // keys written to the run
    const uint64_t off = ld_dev(&l.sp_off[sb + j]);
    // the slot holds its keys word-major (word w of run position i at
    // w * slot_keys + i), so each word of a batch is one coalesced load per wave
    const uint64_t* keys = l.keys + (uint64_t)(r % l.Q) * l.slot_words + off;
    const uint8_t* tail = (const uint8_t*)(l.keys + (uint64_t)(r % l.Q) * l.slot_words + (uint64_t)(W - 1) * l.slot_keys);
    const uint64_t lim = (off + n <= l.slot_keys) ? n : 0;   // a run past the slot was never written
    // A run sized from a sample can overflow while keys are scattered; the
    // keys past its end are then already in the emergency area, so every key
    // of this sub-table goes there too and each key is counted in one place.
    const bool spill = n_put > n_cap;
    for (uint32_t i = tid; i < C; i += B) {
        w0[i] = GERBIL_EMPTY;
        if (PK) tc[i] = 0; else cnt[i] = 0;
    }
    __syncthreads();
    // count of slot sl (a packed slot keeps it in the low half of its last word)
    auto count_at = [&](uint32_t sl) -> uint32_t { return PK ? (uint32_t)tc[sl] : cnt[sl]; };
    for (uint64_t base = 0; base < lim; base += (uint64_t)B * K) {
        // every lane loads K keys (lanes past the run re-read its last key and
        // drop it), so all loads of the batch are in flight together
        uint64_t key[K][W];
        uint64_t ix[K];
#pragma unroll
        for (int e = 0; e < K; e++) {
            const uint64_t i = base + (uint64_t)e * B + tid;
            ix[e] = i < lim ? i : lim - 1;
        }
#pragma unroll
        for (int e = 0; e < K; e++)
#pragma unroll
            for (int w = 0; w + 1 < W; w++) key[e][w] = ld_dev(&keys[(uint64_t)w * l.slot_keys + ix[e]]);
        load_tails<K, W>(tail, off, ix, l.tail_bytes, key);
        uint32_t nk = 0;   // valid keys of this lane: a prefix of the batch
#pragma unroll
        for (int e = 0; e < K; e++)
            if (base + (uint64_t)e * B + tid < lim) nk = (uint32_t)e + 1;
        if (spill) {
#pragma unroll
            for (int e = 0; e < K; e++)
                if ((uint32_t)e < nk) overflow_push<W>(a, key[e]);
            if (l.probe_hist && nk) atomicAdd(&s.probes[0], nk);
        } else {
            lds_insert_all<K, W, PK>(a, w0, rest, cnt, tc, C, l.theta, key, nk, l.probe_hist ? s.probes : nullptr);
        }
    }
    __syncthreads();
    // dump: count this thread's pairs, one reservation for the block (its
    // round trip overlaps the histogram), write
    uint32_t mine = 0;
    for (uint32_t sl = tid; sl < C; sl += B) mine += count_at(sl) >= a.threshold;
    uint32_t total;
    const uint32_t pre = block_excl_scan(mine, wsum, total);
    uint64_t base = 0;
    if (tid == 0 && total) base = add_dev(a.n_out, (uint64_t)total);
    // most distinct keys occur once: count those per wave with one LDS add
    for (uint32_t b0 = 0; b0 < C; b0 += B) {
        const uint32_t sl = b0 + tid;
        const uint32_t c = sl < C ? count_at(sl) : 0u;
        const uint64_t ones = __ballot(c == 1u);
        if (ones && __lane_id() == (uint32_t)__ffsll((unsigned long long)ones) - 1u)
            atomicAdd(&s.hist[1], (uint32_t)__popcll(ones));
        if (c > 1u) {
            if (c < kLdsHist) atomicAdd(&s.hist[c], 1u);
            else add_dev(&a.hist[c < kHistInternal - 1 ? c : kHistInternal - 1], 1ull);
        }
        wmax = c > wmax ? c : wmax;
    }
    if (tid == 0) *s_base = base;
    __syncthreads();
    uint64_t pos = *s_base + pre;
    for (uint32_t sl = tid; sl < C && mine; sl += B) {
        const uint32_t c = count_at(sl);
        if (c && c >= a.threshold) {
            if (pos < a.cap) {
                a.out_keys[pos * W] = w0[sl] ^ stored_xor(a.canonical, a.k);
                if (PK) {
#pragma unroll
                    for (int i = 1; i + 1 < W; i++) a.out_keys[pos * W + i] = rest[(uint32_t)(i - 1) * C + sl];
                    a.out_keys[pos * W + W - 1] = tc[sl] >> 32;
                } else {
#pragma unroll
                    for (int i = 1; i < W; i++) a.out_keys[pos * W + i] = rest[(uint32_t)(i - 1) * C + sl];
                }
                a.out_counts[pos] = c;
            } else {
                set_status(a.status, ST_OUT_CAP);
            }
            pos++;
            mine--;
        }
    }
}

template <int W, uint32_t B, bool PK>
__device__ __forceinline__ void run_stage(const CountArgs& a, const LdsArgs& l, const Lds& s, uint32_t st,
                                          uint32_t r, uint32_t local, uint32_t& wmax) {
    switch (st) {
        case 0: stage_count<W, B>(a, l, s, r, local); break;
        case 1: stage_scan<B>(a, l, s, r); break;
        case 2: stage_scatter<W, B>(a, l, s, r, local); break;
        default: stage_table<W, B, PK>(a, l, s, r, local, wmax); break;
    }
}

template <uint32_t B>
__device__ __forceinline__ void hist_begin(const LdsArgs& l, const Lds& s) {
    for (uint32_t b = threadIdx.x; b < kLdsHist; b += B) s.hist[b] = 0;
    if (l.probe_hist && threadIdx.x < kProbeHist) s.probes[threadIdx.x] = 0;
    __syncthreads();
}
template <uint32_t B>
__device__ __forceinline__ void hist_end(const CountArgs& a, const LdsArgs& l, const Lds& s, uint32_t wmax) {
    flush_max(a.max_count, wmax);
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < kLdsHist; b += B)
        if (s.hist[b]) add_dev(&a.hist[b], (uint64_t)s.hist[b]);
    if (l.probe_hist && threadIdx.x < kProbeHist && s.probes[threadIdx.x])
        add_dev(&l.probe_hist[threadIdx.x], (uint64_t)s.probes[threadIdx.x]);
}

// Segment of queue item `item` (last j < ns with start[j] <= item) and its
// first item, searched by the 64 lanes of one wave from `hint`: one
// coalesced load of 64 segment starts per step. Items a workgroup pops
// increase, so start[hint] <= item and the answer is at most a few segments on.
__device__ __forceinline__ uint32_t locate_item(const uint64_t* start, uint32_t ns, uint64_t item, uint32_t hint,
                                                uint64_t& first) {
    const uint32_t lane = __lane_id();
    for (;;) {
        const uint32_t j = hint + lane;
        const uint64_t v = j < ns ? start[j] : ~0ull;
        const uint64_t m = __ballot(v <= item);   // a prefix of the lanes (starts never decrease)
        if (m != ~0ull) {
            const uint32_t h = m ? 63u - (uint32_t)__clzll(m) : 0u;
            first = __shfl(v, (int)h);
            return hint + h;
        }
        hint += 63;
    }
}

// Segment of queue item `item` with no hint: a 64-ary search, one coalesced
// load of 64 evenly spaced segment starts per step (starts never decrease,
// start[0] = 0 <= item < start[ns]).
__device__ __forceinline__ uint32_t locate_far(const uint64_t* start, uint32_t ns, uint64_t item, uint64_t& first) {
    const uint32_t lane = __lane_id();
    uint32_t lo = 0, hi = ns;   // start[lo] <= item, and the answer is below hi
    while (hi - lo > 64) {
        const uint32_t step = (hi - lo + 63) / 64;
        const uint32_t j = lo + lane * step;
        const uint64_t v = j < hi ? start[j] : ~0ull;
        const uint64_t m = __ballot(v <= item);   // a prefix of the lanes, lane 0 included
        const uint32_t h = 63u - (uint32_t)__clzll(m);
        const uint32_t nlo = lo + h * step;
        if (nlo + step < hi) hi = nlo + step;
        lo = nlo;
    }
    const uint32_t j = lo + lane;
    const uint64_t v = j < hi ? start[j] : ~0ull;
    const uint64_t m = __ballot(v <= item);
    const uint32_t h = 63u - (uint32_t)__clzll(m);
    first = __shfl(v, (int)h);
    return lo + h;
}

// Wave 0: place item `it`, popped from queue q, in its segment; when it lies
// past the end of q, pop the other queues in turn. Returns false once every
// queue is exhausted (cursors only grow, so an exhausted queue stays so).
// `near` says sg is the current segment of q, a valid search hint.
__device__ __forceinline__ bool settle_item(const LdsArgs& l, uint32_t ns, uint32_t& q, uint64_t& it, uint32_t& sg,
                                            uint64_t& first, bool near) {
    const uint32_t NQ = l.n_queues;
    const uint64_t* start = l.seg_start + (uint64_t)q * (ns + 1);
    if (it < start[ns]) {
        sg = near ? locate_item(start, ns, it, sg, first) : locate_far(start, ns, it, first);
        return true;
    }
    for (uint32_t d = 1; d < NQ; d++) {
        const uint32_t q2 = (q + d) % NQ;
        const uint64_t* s2 = l.seg_start + (uint64_t)q2 * (ns + 1);
        uint64_t v = 0;
        if (__lane_id() == 0) v = add_dev(&l.cursor[q2 * kCursorStride], 1ull);
        v = __shfl(v, 0);
        if (v < s2[ns]) {
            q = q2;
            it = v;
            sg = locate_far(s2, ns, v, first);
            return true;
        }
    }
    return false;
}

// BATCHED: every stage of every rank from per-XCD queues. A workgroup takes
// the items of its own queue, then helps the others. Wave 0 pops the next item
// of the current queue as soon as the current one starts, so the queue's round
// trip and the segment search overlap with the stage's work.
// No deadlock: dependencies point to items of earlier segments only. Take the
// unfinished item X of the earliest segment, in queue q. If it runs, what it
// waits for has finished. If it is held popped ahead, its holder runs an item
// of q before it, which cannot depend on it. If it is not popped, every
// workgroup of q (one at least: n_queues <= grid) runs an earlier item of q,
// finished or independent of X, and then pops on towards X.
template <int W, uint32_t B, bool PK>
__global__ void __launch_bounds__(B, 4) k_lds_persistent(CountArgs a, LdsArgs l) {
    extern __shared__ __align__(16) uint8_t lds_raw[];
    const Lds s = lds_carve(lds_raw);
    uint64_t* s_item = (uint64_t*)(lds_raw + kLdsHist * 4);
    uint64_t* s_first = s_item + 1;
    uint32_t* s_seg = (uint32_t*)(s_item + 2);
    uint32_t* s_q = s_seg + 1;   // current queue; n_queues once every queue is exhausted
    static_assert(kLdsHist * 4 + 24 <= kProbeHistAt && kProbeHistAt + 4 * kProbeHist <= kLdsReserved - 4,
                  "queue scalars and probe counts exceed the reserved LDS");
    const uint32_t tid = threadIdx.x;
    hist_begin<B>(l, s);
    uint32_t wmax = 0;
    const uint32_t ns = *l.n_seg;
    const uint32_t NQ = l.n_queues;
    const uint32_t L = l.lag;
    if (tid < 64) {
        uint32_t q = blockIdx.x % NQ, sg = 0;
        uint64_t it = 0, first = 0;
        if (tid == 0) it = add_dev(&l.cursor[q * kCursorStride], 1ull);
        it = __shfl(it, 0);
        const bool ok = settle_item(l, ns, q, it, sg, first, false);
        if (tid == 0) {
            *s_item = it;
            *s_first = first;
            *s_seg = sg;
            *s_q = ok ? q : NQ;
        }
    }
    __syncthreads();
    for (;;) {
        const uint32_t q = *s_q;
        if (q >= NQ) break;
        const uint64_t item = *s_item;
        const uint32_t seg = *s_seg;
        const uint32_t local = (uint32_t)(item - *s_first);
        uint64_t nxt = 0;
        if (tid == 0) nxt = add_dev(&l.cursor[q * kCursorStride], 1ull);   // waited for only after the stage
        const uint32_t st = seg & 3, tick = seg >> 2;
        const uint32_t lagv = st == 0 ? 0u : st == 1 ? 1u : st == 2 ? 2u : 2u + L;
        const uint32_t r = tick - lagv;
        if (tid == 0) {
            if (st == 1) wait_done(l.done + 4 * r + 0, l.rank_nchunk[r], kLdsWait, a.status, ST_SPIN);
            if (st == 2) {
                wait_done(l.done + 4 * r + 1, 1u, kLdsWait, a.status, ST_SPIN);
                if (r >= l.Q) wait_done(l.done + 4 * (r - l.Q) + 3, l.rank_nsub[r - l.Q], kLdsWait, a.status, ST_SPIN);
            }
            if (st == 3) wait_done(l.done + 4 * r + 2, l.rank_nchunk[r], kLdsWait, a.status, ST_SPIN);
        }
        __syncthreads();
        const uint64_t t0 = l.stage_clocks ? wall_clock64() : 0;
        run_stage<W, B, PK>(a, l, s, st, r, local, wmax);
        // Stages 0 and 1 publish with device-coherent stores and atomics, so a
        // drain before the signal suffices. The scatter writes its keys with
        // plain stores (merged in this XCD's L2): once every wave has drained
        // them into L2, one agent-scope release fence writes L2 back to memory
        // before the signal, and readers load the keys device-coherently. The
        // table stage only releases its key slot: its key loads have completed
        // (their values were inserted), and its output stores are read by no
        // other stage, so it signals without a drain.
        if (st == 3) {
            __syncthreads();
            if (tid == 0) __hip_atomic_fetch_add(l.done + 4 * r + st, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else if (st == 2) {
            drain_memory();
            __syncthreads();
            if (tid == 0) {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                __hip_atomic_fetch_add(l.done + 4 * r + st, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        } else {
            signal_done(l.done + 4 * r + st);
        }
        // (either way a barrier: every thread has read this item's scalars)
        if (l.stage_clocks && tid == 0) {
            add_dev(&l.stage_clocks[st], wall_clock64() - t0);
            add_dev(&l.stage_clocks[4 + st], 1ull);
        }
        if (tid < 64) {
            uint32_t q2 = q, sg = seg;
            uint64_t it = __shfl(nxt, 0), first = 0;
            const bool ok = settle_item(l, ns, q2, it, sg, first, true);
            if (tid == 0) {
                *s_item = it;
                *s_first = first;
                *s_seg = sg;
                *s_q = ok ? q2 : NQ;
            }
        }
        __syncthreads();
    }
    hist_end<B>(a, l, s, wmax);
}

// PLAIN: `items` blocks of one stage of one rank.
template <int W, bool PK>
__global__ void __launch_bounds__(kLdsBlock) k_lds_stage(CountArgs a, LdsArgs l, uint32_t st, uint32_t r) {
    constexpr uint32_t B = kLdsBlock;
    extern __shared__ __align__(16) uint8_t lds_raw[];
    const Lds s = lds_carve(lds_raw);
    hist_begin<B>(l, s);
    uint32_t wmax = 0;
    run_stage<W, B, PK>(a, l, s, st, r, blockIdx.x, wmax);
    __syncthreads();
    hist_end<B>(a, l, s, wmax);
}

// The LDS attribute is set on every launch: it belongs to the current device's
// module, and a process-wide "already set" flag would race between threads
// and miss other devices.
template <int W, uint32_t B, bool PK>
static hipError_t persistent_lds_w(const CountArgs& a, const LdsArgs& l, uint32_t grid, hipStream_t s) {
    hipError_t e = hipFuncSetAttribute((const void*)k_lds_persistent<W, B, PK>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, LdsShape<B>::bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_lds_persistent<W, B, PK>), dim3(grid), dim3(B), LdsShape<B>::bytes, s, a, l);
    return hipGetLastError();
}

template <int W, bool PK>
static hipError_t stage_lds_w(const CountArgs& a, const LdsArgs& l, uint32_t st, uint32_t r, uint32_t items,
                              hipStream_t s) {
    if (items == 0) return hipSuccess;
    hipError_t e = hipFuncSetAttribute((const void*)k_lds_stage<W, PK>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       LdsShape<kLdsBlock>::bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_lds_stage<W, PK>), dim3(items), dim3(kLdsBlock), LdsShape<kLdsBlock>::bytes, s, a, l, st, r);
    return hipGetLastError();
}

// Packed slots exist for keys of two words or more (lds_packed).
template <uint32_t B>
static hipError_t persistent_lds_b(const CountArgs& a, const LdsArgs& l, uint32_t grid, hipStream_t s) {
    const bool pk = l.packed != 0;
    switch (a.W) {
        case 1: return persistent_lds_w<1, B, false>(a, l, grid, s);
        case 2: return pk ? persistent_lds_w<2, B, true>(a, l, grid, s) : persistent_lds_w<2, B, false>(a, l, grid, s);
        case 3: return pk ? persistent_lds_w<3, B, true>(a, l, grid, s) : persistent_lds_w<3, B, false>(a, l, grid, s);
        case 4: return pk ? persistent_lds_w<4, B, true>(a, l, grid, s) : persistent_lds_w<4, B, false>(a, l, grid, s);
        case 5: return pk ? persistent_lds_w<5, B, true>(a, l, grid, s) : persistent_lds_w<5, B, false>(a, l, grid, s);
        case 6: return pk ? persistent_lds_w<6, B, true>(a, l, grid, s) : persistent_lds_w<6, B, false>(a, l, grid, s);
        case 7: return pk ? persistent_lds_w<7, B, true>(a, l, grid, s) : persistent_lds_w<7, B, false>(a, l, grid, s);
        case 8: return pk ? persistent_lds_w<8, B, true>(a, l, grid, s) : persistent_lds_w<8, B, false>(a, l, grid, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_lds_persistent(const CountArgs& a, const LdsArgs& l, uint32_t grid, hipStream_t s) {
    if (l.block == 1024) return persistent_lds_b<1024>(a, l, grid, s);
    if (l.block == 512) return persistent_lds_b<512>(a, l, grid, s);
    return hipErrorInvalidValue;
}

hipError_t launch_lds_stage(const CountArgs& a, const LdsArgs& l, uint32_t st, uint32_t r, uint32_t items,
                            hipStream_t s) {
    const bool pk = l.packed != 0;
    switch (a.W) {
        case 1: return stage_lds_w<1, false>(a, l, st, r, items, s);
        case 2: return pk ? stage_lds_w<2, true>(a, l, st, r, items, s) : stage_lds_w<2, false>(a, l, st, r, items, s);
        case 3: return pk ? stage_lds_w<3, true>(a, l, st, r, items, s) : stage_lds_w<3, false>(a, l, st, r, items, s);
        case 4: return pk ? stage_lds_w<4, true>(a, l, st, r, items, s) : stage_lds_w<4, false>(a, l, st, r, items, s);
        case 5: return pk ? stage_lds_w<5, true>(a, l, st, r, items, s) : stage_lds_w<5, false>(a, l, st, r, items, s);
        case 6: return pk ? stage_lds_w<6, true>(a, l, st, r, items, s) : stage_lds_w<6, false>(a, l, st, r, items, s);
        case 7: return pk ? stage_lds_w<7, true>(a, l, st, r, items, s) : stage_lds_w<7, false>(a, l, st, r, items, s);
        case 8: return pk ? stage_lds_w<8, true>(a, l, st, r, items, s) : stage_lds_w<8, false>(a, l, st, r, items, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace gerbil

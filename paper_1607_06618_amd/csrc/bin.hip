// Distribution into bins (phase one, Sec. 2.1 and Sec. 2.3.1 splitter step).
//
// The minimizer of a k-mer is its smallest m-mer under a total order on
// m-mers (Sec. 2.1); here the m-mers are canonical (smaller of the m-mer and
// its reverse complement) so that a k-mer and its reverse complement share a
// minimizer and therefore a bin. Orders (Sec. 3.1): KMC2-style -- canonical
// code c, moved behind all others (c + 4^m) when it starts with AAA or ACA --
// or plain lexicographic. A super-mer is a maximal run of consecutive valid
// k-mers with equal minimizers (Fig. 1); all of its k-mers go to the bin of
// that minimizer, so every occurrence of a canonical k-mer lands in one bin
// (the partition property of Sec. 2.1).
//
// GPU design: the read stream is cut into tiles of kTile k-mer start
// positions. A workgroup computes the m-mer ranks of its tile plus a halo of
// w = k-m+1 positions (each thread rolls the canonical m-mer over a run of
// positions), takes the minimum of every window of w ranks (each thread
// covers a run of windows as suffix minimum + shared middle + prefix
// minimum), finds super-mer starts with wave ballots, and writes
// one descriptor per super-mer piece (super-mers are also cut at tile
// boundaries; both pieces keep the same bin). Per-bin super-mer counts are
// privatised in LDS. A scan and an LDS-privatised scatter then group the
// descriptors by bin.
#include "../../include/gerbil.h"
#include "common.h"
#include "internal.h"

namespace gerbil {

constexpr uint32_t kBinBlock = 256;
// Longest window w = k - m + 1 a tile kernel serves: one instantiation for
// w <= 256, one for the longest keys (the halo of ranks grows with w).
constexpr uint32_t kMaxWShort = 256;
constexpr uint32_t kMaxWLong = 32 * GERBIL_MAX_W;
// ranks for positions P0-1 .. P0+kTile-1+w-1
template <uint32_t MW> constexpr uint32_t rank_len() { return kTile + MW; }
constexpr uint32_t kWordsPerTile = kTile / 64;

// The same rank for m-mers held in 32 bits (m <= 15: 30 bits; the moved codes
// c + 4^m stay below 2^31).
__device__ __forceinline__ uint32_t rank_of32(uint32_t fw, uint32_t rc, uint32_t m, uint32_t order,
                                              const uint32_t* __restrict__ table) {
    uint32_t c = fw < rc ? fw : rc;
    if (order == GERBIL_ORDER_TABLE) return table[c];
    if (order == 0 && m >= 3) {
        const uint32_t head = c >> (2 * m - 6);
        if (head == 0 /* AAA */ || head == 4 /* ACA */) c += 1u << (2 * m);
    }
    return c;
}

__device__ __forceinline__ uint32_t rank_of(uint64_t fw, uint64_t rc, uint32_t m, uint32_t order,
                                            const uint32_t* __restrict__ table) {
    uint64_t c = fw < rc ? fw : rc;
    if (order == GERBIL_ORDER_TABLE) return table[c];
    if (order == 0 && m >= 3) {
        uint64_t head = c >> (2 * m - 6);
        if (head == 0 /* AAA */ || head == 4 /* ACA */) c += 1ull << (2 * m);
    }
    return (uint32_t)c;
}

template <uint32_t MW> constexpr uint32_t rank_per() { return (rank_len<MW>() + kBinBlock - 1) / kBinBlock; }
constexpr uint32_t kMinPer = (kTile + 1 + kBinBlock - 1) / kBinBlock;      // minimizers per thread
// The bases a thread's ranks need (kRankPer m-mers, m <= 15) start at most 31
// bases into a packed word, so they lie in that word and the next.
static_assert(31 + rank_per<kMaxWLong>() - 1 + 15 <= 64, "a rank run must fit in two packed words");
static_assert(15 + rank_per<kMaxWLong>() - 1 <= 32, "a rank run must fit in the 32 bases from its start");
static_assert(kWordsPerTile <= kBinBlock, "one bitmap word per thread");

// Position of the n-th (from 0) set bit of x; x has more than n set bits.
__device__ __forceinline__ uint32_t select_bit(uint64_t x, uint32_t n) {
    uint32_t pos = 0;
#pragma unroll
    for (uint32_t s = 32; s >= 1; s >>= 1) {
        const uint32_t c = (uint32_t)__popcll(x & ((1ull << s) - 1ull));
        if (n >= c) {
            n -= c;
            x >>= s;
            pos += s;
        }
    }
    return pos;
}

// Global data one tile needs, loaded one tile ahead into registers.
struct TileFetch {
    uint64_t w0, w1;   // the two packed words of this thread's rank run
    uint64_t ok;       // threads < kWordsPerTile: one word of the valid-window bitmap
};

template <uint32_t MW>
__device__ __forceinline__ TileFetch tile_fetch(const BinArgs& a, uint64_t tile, uint64_t n_tiles, uint64_t n_mask) {
    TileFetch f{0ull, 0ull, 0ull};
    if (tile >= n_tiles) return f;
    const int64_t P0 = (int64_t)(tile * kTile);
    const int64_t j0 = P0 - 1 + (int64_t)(threadIdx.x * rank_per<MW>());
    if (j0 < (int64_t)a.n_bytes) {   // j0 >= -1: word -1 is the zero pad; q + 1 <= n_words
        const int64_t q = j0 >> 5;
        f.w0 = a.packed[q];
        f.w1 = a.packed[q + 1];
    }
    if (threadIdx.x < kWordsPerTile) {
        const uint64_t qq = (uint64_t)(P0 >> 6) + threadIdx.x;
        f.ok = qq < n_mask ? a.kmer_ok[qq] : 0ull;
    }
    return f;
}

// Base at offset o (0..63) of the 64-base pair (w0, w1).
__device__ __forceinline__ uint64_t pair_base(uint64_t w0, uint64_t w1, uint32_t o) {
    const uint64_t w = o < 32 ? w0 : w1;
    return (w >> (62 - 2 * (o & 31))) & 3ull;
}

template <uint32_t MW>
__global__ void __launch_bounds__(kBinBlock, 7) k_bin_tiles(BinArgs a) {
    constexpr uint32_t kRankPer = rank_per<MW>();
    // When a thread's run of ranks is one block of kMinPer positions, it also
    // writes the block's minimum, and a window's middle part is read as block
    // minima plus the ranks at its two ends.
    constexpr bool kBlockMin = kRankPer == kMinPer;
    constexpr uint32_t kBlocks = kBlockMin ? rank_len<MW>() / kMinPer : 1;
    __shared__ uint32_t R[rank_len<MW>()];
    __shared__ uint32_t BM[kBlocks];   // BM[j] = min R[j*kMinPer .. (j+1)*kMinPer), whole blocks below len
    __shared__ uint32_t M[kTile + 1];
    __shared__ uint64_t brk[kWordsPerTile];
    __shared__ uint64_t stw[kWordsPerTile];
    __shared__ uint64_t okS[kWordsPerTile];
    __shared__ uint32_t wpre[kWordsPerTile + 1];
    __shared__ uint64_t tile_base, tile_split, tile_base2;
    extern __shared__ uint32_t bin_cnt[];   // [n_bins]

    const uint32_t tid = threadIdx.x, lane = __lane_id(), wave = tid >> 6;
    const uint32_t w = a.k - a.m + 1;
    const uint64_t n_pos = a.n_bytes;
    const uint64_t n_tiles = (n_pos + kTile - 1) / kTile;
    const uint64_t n_mask = (n_pos + 63) >> 6;
    const uint32_t code_mask = (uint32_t)((1ull << (2 * a.m)) - 1ull);
    const uint64_t mmask = (1ull << (2 * a.m)) - 1ull;
    // list slots of this workgroup's current chunk [ch_cur, ch_end) (used by wave 0's last word lane)
    uint64_t ch_cur = 0, ch_end = 0;
    uint64_t n_mine = 0;   // pieces found by this workgroup, added to n_superm once at the end

    for (uint32_t b = tid; b < a.n_bins; b += kBinBlock) bin_cnt[b] = 0;

    TileFetch f = tile_fetch<MW>(a, blockIdx.x, n_tiles, n_mask);
    for (uint64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int64_t P0 = (int64_t)(tile * kTile);
        const uint32_t len = kTile + w;   // ranks R[i] for positions P0-1+i
        // 1. ranks: every thread rolls the canonical m-mer over its own run of
        //    positions, from the two packed words fetched for it
        {
            const uint32_t i0 = tid * kRankPer;
            const uint32_t i1 = i0 + kRankPer < len ? i0 + kRankPer : len;
            const int64_t j0 = P0 - 1 + (int64_t)i0;
            const uint32_t s0 = (uint32_t)(j0 & 31);
            // the run's first m-mer and the bases rolled in after it all lie in the
            // 32 bases from s0 (m + kRankPer - 1 <= 32); 32-bit arithmetic throughout
            uint32_t fw = 0, rc = 0;
            uint64_t nb = 0;   // the bases still to roll in, first one in the top two bits
            if (i0 < i1) {
                const uint64_t win = s0 ? ((f.w0 << (2 * s0)) | (f.w1 >> (64 - 2 * s0))) : f.w0;
                fw = (uint32_t)(win >> (64 - 2 * a.m));
                rc = (uint32_t)(revcomp32(win) & mmask);
                nb = win << (2 * a.m);
            }
            // positions of this run inside the read stream, at most kRankPer
            const int64_t n_left = (int64_t)n_pos - (P0 - 1 + (int64_t)i0);
            const uint32_t n_in = n_left <= 0 ? 0u : n_left >= (int64_t)kRankPer ? kRankPer : (uint32_t)n_left;
            uint32_t bmin = 0xFFFFFFFFu;
#pragma unroll
            for (uint32_t e = 0; e < kRankPer; e++) {
                if (i0 + e < i1) {
                    if (e > 0) {
                        const uint32_t b2 = (uint32_t)(nb >> 62);
                        nb <<= 2;
                        fw = ((fw << 2) | b2) & code_mask;
                        rc = (rc >> 2) | ((3u - b2) << (2 * a.m - 2));
                    }
                    const uint32_t rk = e < n_in ? rank_of32(fw, rc, a.m, a.order, a.rank_table) : 0xFFFFFFFFu;
                    R[i0 + e] = rk;
                    bmin = min(bmin, rk);
                }
            }
            if constexpr (kBlockMin) {
                if (i0 + kMinPer <= len) BM[tid] = bmin;   // a whole block: i0 = tid * kMinPer
            }
            if (tid < kWordsPerTile) okS[tid] = f.ok;
        }
        // the next tile's loads are in flight while this one is processed
        f = tile_fetch<MW>(a, tile + gridDim.x, n_tiles, n_mask);
        __syncthreads();
        // 2. minimizer of the k-mer at P0-1+i = min R[i .. i+w): each thread takes
        //    a run of kMinPer positions; their windows share the middle part.
        {
            const uint32_t i0 = tid * kMinPer;
            const uint32_t i1 = i0 + kMinPer < kTile + 1 ? i0 + kMinPer : kTile + 1;
            if (i0 < i1) {
                if (w <= 2 * kMinPer) {
                    for (uint32_t i = i0; i < i1; i++) {
                        uint32_t mn = 0xFFFFFFFFu;
                        for (uint32_t t = 0; t < w; t++) mn = min(mn, R[i + t]);
                        M[i] = mn;
                    }
                } else {
                    // window [i, i+w) = [i, i1-1) + [i1-1, i0+w) + [i0+w, i+w)
                    uint32_t mid = 0xFFFFFFFFu;
                    const uint32_t lo = i1 - 1, hi = i0 + w;   // hi <= kTile + w = len
                    const uint32_t jb = (lo + kMinPer - 1) / kMinPer, je = hi / kMinPer;
                    if (kBlockMin && jb < je) {
                        // whole blocks jb .. je-1 lie in [lo, hi) and below len
                        for (uint32_t t = lo; t < jb * kMinPer; t++) mid = min(mid, R[t]);
                        for (uint32_t j = jb; j < je; j++) mid = min(mid, BM[j]);
                        for (uint32_t t = je * kMinPer; t < hi; t++) mid = min(mid, R[t]);
                    } else {
#pragma unroll 8
                        for (uint32_t t = lo; t < hi; t++) mid = min(mid, R[t]);
                    }
                    uint32_t suf[kMinPer], pre[kMinPer];
                    uint32_t run = 0xFFFFFFFFu;
#pragma unroll
                    for (int e = kMinPer - 1; e >= 0; e--) {   // suffix minima of [i, i1-1)
                        const uint32_t i = i0 + e;
                        if (i + 1 < i1) run = min(run, R[i]);
                        suf[e] = run;
                    }
                    run = 0xFFFFFFFFu;
#pragma unroll
                    for (int e = 0; e < (int)kMinPer; e++) {   // prefix minima of [i0+w, i+w)
                        pre[e] = run;
                        const uint32_t t = i0 + w + e;
                        if (i0 + e + 1 < i1) run = min(run, R[t]);
                    }
#pragma unroll
                    for (int e = 0; e < (int)kMinPer; e++) {
                        const uint32_t i = i0 + e;
                        if (i < i1) M[i] = min(min(suf[e], mid), pre[e]);
                    }
                }
            }
        }
        __syncthreads();
        // 3. super-mer starts and ends (ballot per 64 positions); the first
        //    position of a tile always starts a piece (the tile cut)
        for (uint32_t c = wave; c < kWordsPerTile; c += kBinBlock / 64) {
            const uint64_t okw = okS[c];
            const uint64_t okprev = c ? okS[c - 1] : 0ull;
            bool ok = (okw >> lane) & 1ull;
            bool ok_before = lane ? ((okw >> (lane - 1)) & 1ull) : ((okprev >> 63) & 1ull);
            uint32_t t = c * 64 + lane;   // position P0 + t, minimizer M[t+1]
            bool start = ok && (t == 0 || !ok_before || M[t + 1] != M[t]);
            uint64_t sb = __ballot(start);
            uint64_t bb = __ballot(!ok || start);
            if (lane == 0) { stw[c] = sb; brk[c] = bb; }
        }
        __syncthreads();
        // list slots for this tile's pieces: the rest of the workgroup's
        // chunk first, then a new chunk (reserved only when the current one
        // runs out), so only the unused end of a workgroup's last chunk is
        // left as a hole
        if (wave == 0) {
            uint32_t n = lane < kWordsPerTile ? (uint32_t)__popcll(stw[lane]) : 0u;
            uint32_t incl = n;
            for (int off = 1; off < 64; off <<= 1) {
                uint32_t y = __shfl_up(incl, off);
                if (lane >= (uint32_t)off) incl += y;
            }
            if (lane < kWordsPerTile) wpre[lane] = incl - n;
            if (lane == kWordsPerTile - 1) {
                wpre[kWordsPerTile] = incl;
                const uint64_t rem = ch_end - ch_cur;
                uint64_t b1 = ch_cur, sp = incl, b2 = 0;
                if (incl > rem) {
                    const uint64_t need = incl - rem;
                    const uint64_t take = need > kListChunk ? need : kListChunk;
                    b2 = add_dev(a.list_used, take);
                    sp = rem;
                    ch_cur = b2 + need;
                    ch_end = b2 + take;
                } else {
                    ch_cur += incl;
                }
                n_mine += incl;
                tile_base = b1;
                tile_split = sp;
                tile_base2 = b2;
            }
        }
        __syncthreads();
        // 4. one descriptor per start: thread i takes starts i, i + kBinBlock, ...
        //    of the tile, so the lanes stay busy however sparse the starts are
        const uint32_t n_st = wpre[kWordsPerTile];
        for (uint32_t q = tid; q < n_st; q += kBinBlock) {
            uint32_t lo = 0, hi = kWordsPerTile;   // word of start q: last c with wpre[c] <= q
            while (hi - lo > 1) {
                const uint32_t mid = (lo + hi) >> 1;
                if (wpre[mid] <= q) lo = mid; else hi = mid;
            }
            const uint32_t c = lo;
            const uint32_t bit = select_bit(stw[c], q - wpre[c]);
            const uint32_t t = c * 64 + bit;
            const uint64_t above = (bit == 63) ? 0ull : (brk[c] & ~((2ull << bit) - 1ull));
            uint32_t end = kTile;
            if (above) {
                end = c * 64 + (uint32_t)__builtin_ctzll(above);
            } else {
                for (uint32_t d = c + 1; d < kWordsPerTile; d++) {
                    if (brk[d]) { end = d * 64 + (uint32_t)__builtin_ctzll(brk[d]); break; }
                }
            }
            const uint32_t nk = end - t;
            const uint32_t mr = M[t + 1];
            const uint32_t code = mr & code_mask;
            uint32_t bin = a.bin_map ? a.bin_map[code] : (mr % a.n_bins);
            if (bin >= a.n_bins) bin = a.n_bins - 1;   // defensive: a bad map must not index out of range
            const uint64_t idx = q < tile_split ? tile_base + q : tile_base2 + (q - tile_split);
            if (idx < a.list_cap) {
                a.list_desc[idx] = ((uint64_t)(P0 + t) << 24) | nk;
                a.list_bin[idx] = bin;
                atomicAdd(&bin_cnt[bin], 1u);
            } else {
                set_status(a.status, ST_SUPERM_CAP);
            }
        }
        __syncthreads();
    }
    // the unused end of the last chunk is a hole
    if (wave == 0) {
        const uint64_t lo = __shfl(ch_cur, (int)kWordsPerTile - 1), hi = __shfl(ch_end, (int)kWordsPerTile - 1);
        for (uint64_t i = lo + lane; i < hi; i += 64)
            if (i < a.list_cap) a.list_bin[i] = kHole;
        if (lane == kWordsPerTile - 1 && n_mine) add_dev(a.n_superm, n_mine);
    }
    __syncthreads();
    for (uint32_t b = tid; b < a.n_bins; b += kBinBlock)
        if (bin_cnt[b]) atomicAdd(&a.bin_count[b], bin_cnt[b]);
}

// Exclusive prefix of the per-bin super-mer counts (single workgroup).
__global__ void __launch_bounds__(1024) k_bin_scan(BinArgs a) {
    __shared__ uint64_t part[1024];
    const uint32_t tid = threadIdx.x;
    const uint32_t per = (a.n_bins + 1023) / 1024;
    uint64_t local[4];
    uint64_t s = 0;
    for (uint32_t e = 0; e < per; e++) {
        uint32_t b = tid * per + e;
        uint64_t v = b < a.n_bins ? (uint64_t)a.bin_count[b] : 0ull;
        local[e] = s;
        s += v;
    }
    part[tid] = s;
    __syncthreads();
    for (uint32_t off = 1; off < 1024; off <<= 1) {
        uint64_t y = tid >= off ? part[tid - off] : 0ull;
        __syncthreads();
        part[tid] += y;
        __syncthreads();
    }
    uint64_t base = tid ? part[tid - 1] : 0ull;
    for (uint32_t e = 0; e < per; e++) {
        uint32_t b = tid * per + e;
        if (b < a.n_bins) {
            a.bin_off[b] = base + local[e];
            a.bin_fill[b] = 0;
            a.bin_kmers[b] = 0;
        }
    }
    if (tid == 1023) a.bin_off[a.n_bins] = part[1023];
}

constexpr uint32_t kScatterPer = 16;   // descriptors per thread per chunk

__global__ void __launch_bounds__(kBinBlock) k_bin_scatter(BinArgs a) {
    extern __shared__ uint32_t sh[];
    uint32_t* lh = sh;                  // [n_bins] counts in this chunk
    uint32_t* lk = sh + a.n_bins;       // [n_bins] k-mers in this chunk
    uint32_t* gb = sh + 2 * a.n_bins;   // [n_bins] global base of this chunk in the bin
    // [n_bins] k-mers of this workgroup's chunks, added to the bins' totals once at the end
    uint64_t* tk = (uint64_t*)(sh + 3 * a.n_bins + (a.n_bins & 1u));
    const uint32_t tid = threadIdx.x;
    uint64_t n = ld_dev(a.list_used);   // list slots handed out, holes included
    if (n > a.list_cap) n = a.list_cap;
    const uint64_t chunk = (uint64_t)kBinBlock * kScatterPer;
    for (uint32_t b = tid; b < a.n_bins; b += kBinBlock) tk[b] = 0;   // read back only by thread b % kBinBlock
    for (uint64_t c0 = blockIdx.x * chunk; c0 < n; c0 += (uint64_t)gridDim.x * chunk) {
        for (uint32_t b = tid; b < a.n_bins; b += kBinBlock) { lh[b] = 0; lk[b] = 0; }
        __syncthreads();
        uint64_t d[kScatterPer];
        uint32_t bn[kScatterPer], lr[kScatterPer];
#pragma unroll
        for (uint32_t e = 0; e < kScatterPer; e++) {
            uint64_t i = c0 + tid + (uint64_t)e * kBinBlock;
            bn[e] = 0xFFFFFFFFu;
            if (i < n) {
                bn[e] = a.list_bin[i];
                if (bn[e] < a.n_bins) {
                    d[e] = a.list_desc[i];
                    lr[e] = atomicAdd(&lh[bn[e]], 1u);
                    atomicAdd(&lk[bn[e]], (uint32_t)(d[e] & 0xFFFFFFu));
                } else {
                    bn[e] = 0xFFFFFFFFu;   // a hole
                }
            }
        }
        __syncthreads();
        for (uint32_t b = tid; b < a.n_bins; b += kBinBlock) {
            if (lh[b]) {
                gb[b] = atomicAdd(&a.bin_fill[b], lh[b]);
                tk[b] += lk[b];
            }
        }
        __syncthreads();
#pragma unroll
        for (uint32_t e = 0; e < kScatterPer; e++) {
            if (bn[e] == 0xFFFFFFFFu) continue;
            uint64_t pos = a.bin_off[bn[e]] + gb[bn[e]] + lr[e];
            if (pos < a.bin_off[bn[e] + 1] && pos < a.cap) a.desc[pos] = d[e];
        }
        __syncthreads();
    }
    for (uint32_t b = tid; b < a.n_bins; b += kBinBlock)
        if (tk[b]) add_dev(&a.bin_kmers[b], tk[b]);
}

// Bin of each key, as the tile kernel assigns it: the smallest rank over the
// k-m+1 canonical m-mers of the k-mer the key encodes, then bin_map or
// rank mod n_bins. (A key's m-mers are those of every window that holds it,
// on either strand, so the bin is the one its occurrences went to.)
__global__ void __launch_bounds__(256) k_key_bins(const uint64_t* __restrict__ keys, uint64_t n, uint32_t k,
                                                  uint32_t W, uint32_t m, uint32_t order,
                                                  const uint32_t* __restrict__ rank_table,
                                                  const uint32_t* __restrict__ bin_map, uint32_t n_bins,
                                                  uint32_t* __restrict__ bins) {
    const uint64_t mmask = (1ull << (2 * m)) - 1ull;
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256) {
        const uint64_t* key = keys + i * W;
        uint64_t fw = 0, rc = 0;
        uint32_t best = 0xFFFFFFFFu, p = 0;
        for (uint32_t w = 0; w < W; w++) {
            const uint64_t x = key[w];
            const uint32_t r = w + 1 < W ? 32u : k - 32u * (W - 1);   // bases in this word, right-aligned
            for (uint32_t o = 0; o < r; o++, p++) {
                const uint64_t b = (x >> (2 * (r - 1 - o))) & 3ull;
                fw = ((fw << 2) | b) & mmask;
                rc = (rc >> 2) | ((3ull - b) << (2 * m - 2));
                if (p + 1 >= m) best = min(best, rank_of(fw, rc, m, order, rank_table));
            }
        }
        uint32_t bin = bin_map ? bin_map[best & (uint32_t)mmask] : best % n_bins;
        if (bin >= n_bins) bin = n_bins - 1;   // defensive, as in the tile kernel
        bins[i] = bin;
    }
}

hipError_t launch_key_bins(const uint64_t* keys, uint64_t n, const BinArgs& a, uint32_t* bins, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const uint64_t g = (n + 255) / 256;
    hipLaunchKernelGGL(k_key_bins, dim3((uint32_t)(g < 65536 ? g : 65536)), dim3(256), 0, s, keys, n, a.k,
                       (a.k + 31) / 32, a.m, a.order, a.rank_table, a.bin_map, a.n_bins, bins);
    return hipGetLastError();
}

hipError_t launch_bin(const BinArgs& a, uint32_t max_grid, uint32_t cus, hipStream_t s) {
    size_t sh_tiles = (size_t)a.n_bins * sizeof(uint32_t);
    // as many workgroups as are resident at once (a second, partial wave of
    // workgroups would double the time of a grid-stride kernel)
    const uint32_t w = a.k - a.m + 1;
    if (w > kMaxWLong) return hipErrorInvalidValue;
    const bool shrt = w <= kMaxWShort;
    int per_cu = 0;
    const hipError_t oe = shrt ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_bin_tiles<kMaxWShort>,
                                                                              kBinBlock, sh_tiles)
                               : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_bin_tiles<kMaxWLong>,
                                                                              kBinBlock, sh_tiles);
    if (oe != hipSuccess || per_cu < 1) per_cu = 1;
    uint64_t grid = (uint64_t)cus * (uint32_t)per_cu;
    if (grid > max_grid) grid = max_grid;
    if (grid < 1) grid = 1;
    if (shrt)
        hipLaunchKernelGGL(k_bin_tiles<kMaxWShort>, dim3((uint32_t)grid), dim3(kBinBlock), sh_tiles, s, a);
    else
        hipLaunchKernelGGL(k_bin_tiles<kMaxWLong>, dim3((uint32_t)grid), dim3(kBinBlock), sh_tiles, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(1024), 0, s, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    size_t sh_sc = (3 * (size_t)a.n_bins + (a.n_bins & 1u)) * sizeof(uint32_t) + (size_t)a.n_bins * sizeof(uint64_t);
    if (sh_sc > 65536) {   // above the default limit of dynamic LDS per workgroup (n_bins > 3276)
        e = hipFuncSetAttribute((const void*)k_bin_scatter, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh_sc);
        if (e != hipSuccess) return e;
    }
    uint64_t chunks = (a.list_cap + (uint64_t)kBinBlock * kScatterPer - 1) / ((uint64_t)kBinBlock * kScatterPer);
    uint32_t g = (uint32_t)(chunks < 2048 ? (chunks ? chunks : 1) : 2048);
    hipLaunchKernelGGL(k_bin_scatter, dim3(g), dim3(kBinBlock), sh_sc, s, a);
    return hipGetLastError();
}

}  // namespace gerbil

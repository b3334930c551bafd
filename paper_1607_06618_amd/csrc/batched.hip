// Batched schedule of the counting step: all bins of a run in ONE
// persistent launch.
//
// The paper counts its temporary files one after another and re-balances
// hashers per file (Sec. 2.3.2, Sec. 3.3.2, Sec. 3.4.1). On one GPU the bins
// are instead turned into a queue of work items that persistent workgroups
// steal with an atomic cursor:
//   * bins are ranked largest first (longest-processing-time order), so the
//     big bins start early and the small ones fill the tail;
//   * rank i owns table (i mod Q) of a pool of Q tables; its items are
//     "insert" items (ins_chunk descriptors each) and "dump" items (cmp_chunk
//     slots each: emit, histogram, reset);
//   * the queue is INS(0..lag-1), then INS(i), CMP(i-lag) alternately, then
//     the remaining CMP; a dump of rank i waits for all inserts of rank i, an
//     insert of rank i waits for the dump of rank i-Q (its table must be
//     clean). Every dependency points to an earlier item, and items are
//     popped in order by running workgroups, so the earliest unfinished item
//     never waits: the schedule cannot deadlock. Every wait is bounded and
//     flags a device error when it gives up.
// Inserts of one bin and dumps of another overlap on the device, and no
// launch gaps or per-bin tails remain.
#include <atomic>

#include "table.h"

namespace gerbil {

constexpr uint32_t kPlanBlock = 1024;
constexpr uint32_t kWaitLimit = 1u << 25;   // about two seconds of s_sleep(2)

// ------------------------------------------------------------------ plan
// One workgroup: LPT order by bitonic sort of (k-mers, bin) in LDS, item
// counts per rank, queue segments and their prefix.
__global__ void __launch_bounds__(kPlanBlock) k_plan(PersistArgs q) {
    __shared__ uint64_t skey[kMaxBins];
    __shared__ uint32_t sval[kMaxBins];
    __shared__ uint64_t part[kPlanBlock];
    __shared__ uint32_t segn[2 * kMaxBins];   // items per queue segment
    const uint32_t tid = threadIdx.x, n = q.n_bins;
    uint32_t N = 1;
    while (N < n) N <<= 1;
    for (uint32_t i = tid; i < N; i += kPlanBlock) {
        skey[i] = i < n ? q.bin_kmers[i] : 0ull;
        sval[i] = i;
    }
    __syncthreads();
    // sort descending by k-mers, ties by bin id ascending
    for (uint32_t size = 2; size <= N; size <<= 1) {
        for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
            for (uint32_t i = tid; i < N / 2; i += kPlanBlock) {
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
    uint64_t max_nb = 1;   // largest power of two of buckets that fits a pool table
    while (max_nb * 2 <= q.slots / kBucket) max_nb *= 2;
    const uint32_t L = q.lag < n ? q.lag : n;
    // descriptors beyond the capacity were never stored: schedule nothing
    const bool overfull = *q.n_superm > q.superm_cap;
    if (overfull && tid == 0) set_status(q.status, ST_SUPERM_CAP);
    // per-rank items and their queue positions
    for (uint32_t i = tid; i < n; i += kPlanBlock) {
        uint32_t b = sval[i];
        uint64_t nd = q.bin_off[b + 1] - q.bin_off[b];
        uint64_t km = q.bin_kmers[b];
        uint64_t want = (uint64_t)((double)km / (double)q.load / kBucket) + 1;
        uint64_t p2 = 1;
        while (p2 < want) p2 *= 2;
        uint32_t nbk = (uint32_t)(p2 < max_nb ? p2 : max_nb);
        uint32_t ni = overfull ? 0u : (uint32_t)((nd + q.ins_chunk - 1) / q.ins_chunk);
        uint32_t nc = (nd && !overfull) ? (uint32_t)(((uint64_t)nbk * kBucket + q.cmp_chunk - 1) / q.cmp_chunk) : 0u;
        q.order[i] = b;
        q.nb[i] = nbk;
        q.n_ins[i] = ni;
        q.n_cmp[i] = nc;
        q.ins_done[i] = 0;
        q.cmp_done[i] = 0;
        uint32_t pos_ins = i < L ? i : L + 2 * (i - L);
        uint32_t pos_cmp = (i + L <= n - 1) ? L + 2 * i + 1 : n + i;
        q.seg_code[pos_ins] = i;
        q.seg_code[pos_cmp] = 0x80000000u | i;
        segn[pos_ins] = ni;
        segn[pos_cmp] = nc;
    }
    __syncthreads();
    // exclusive prefix over the 2n segment counts
    const uint32_t ns = 2 * n, per = (ns + kPlanBlock - 1) / kPlanBlock;
    uint64_t s = 0;
    for (uint32_t e = 0; e < per; e++) {
        uint32_t j = tid * per + e;
        if (j < ns) s += segn[j];
    }
    part[tid] = s;
    __syncthreads();
    for (uint32_t off = 1; off < kPlanBlock; off <<= 1) {
        uint64_t y = tid >= off ? part[tid - off] : 0ull;
        __syncthreads();
        part[tid] += y;
        __syncthreads();
    }
    uint64_t run = tid ? part[tid - 1] : 0ull;
    for (uint32_t e = 0; e < per; e++) {
        uint32_t j = tid * per + e;
        if (j < ns) {
            q.seg_start[j] = run;
            run += segn[j];
        }
    }
    if (tid == kPlanBlock - 1) q.seg_start[ns] = part[kPlanBlock - 1];
    if (tid == 0) *q.cursor = 0;
}

hipError_t launch_plan(const PersistArgs& q, hipStream_t s) {
    hipLaunchKernelGGL(k_plan, dim3(1), dim3(kPlanBlock), 0, s, q);
    return hipGetLastError();
}

template <int W, uint32_t B>
__global__ void __launch_bounds__(B) k_count_persistent(CountArgs a, PersistArgs q) {
    __shared__ int64_t sstart[B];
    __shared__ uint32_t spre[B];
    __shared__ uint32_t wsum[17];
    __shared__ uint32_t lh[kLdsHist];
    __shared__ uint64_t s_item;
    __shared__ uint32_t s_seg;
    const uint32_t tid = threadIdx.x;
    if (tid == 0) s_seg = 0;
    for (uint32_t b = tid; b < kLdsHist; b += B) lh[b] = 0;
    uint32_t wmax = 0;
    const uint32_t ns = 2 * q.n_bins;
    const uint64_t total = q.seg_start[ns];
    for (;;) {
        if (tid == 0) {
            uint64_t item = add_dev(q.cursor, 1ull);
            s_item = item;
            if (item < total) s_seg = find_segment(q.seg_start, ns, item, s_seg);
        }
        __syncthreads();
        const uint64_t item = s_item;
        if (item >= total) break;
        const uint32_t seg = s_seg;
        const uint32_t code = q.seg_code[seg];
        const uint32_t rank = code & 0x7FFFFFFFu;
        const uint64_t local = item - q.seg_start[seg];
        const uint32_t bin = q.order[rank];
        const uint32_t nb = q.nb[rank];
        const Table t = pool_table(q.pool, q.slots, W, rank % q.Q);
        if (!(code >> 31)) {
            // insert item: needs a clean table
            if (tid == 0 && rank >= q.Q) wait_done(q.cmp_done + (rank - q.Q), q.n_cmp[rank - q.Q], kWaitLimit, a.status, ST_SPIN);
            __syncthreads();
            const uint64_t d_end = q.bin_off[bin + 1];
            const uint64_t i = q.bin_off[bin] + local * q.ins_chunk + tid;
            uint32_t n = 0;
            int64_t st = 0;
            if (i < d_end) {
                uint64_t d = a.desc[i];
                st = (int64_t)(d >> 24);
                n = (uint32_t)(d & 0xFFFFFFu);
            }
            uint32_t tot;
            uint32_t pre = block_excl_scan(n, wsum, tot);
            sstart[tid] = st;
            spre[tid] = pre;
            __syncthreads();
            for (uint32_t idx = tid; idx < tot; idx += B) {
                uint32_t lo = 0, hi = B;
                while (hi - lo > 1) {
                    uint32_t mid = (lo + hi) >> 1;
                    if (spre[mid] <= idx) lo = mid; else hi = mid;
                }
                count_position<W>(a, t, nb, sstart[lo] + (int64_t)(idx - spre[lo]));
            }
            signal_done(q.ins_done + rank);
        } else {
            // dump item: needs every insert of this rank
            if (tid == 0) wait_done(q.ins_done + rank, q.n_ins[rank], kWaitLimit, a.status, ST_SPIN);
            __syncthreads();
            const uint64_t s0 = local * q.cmp_chunk;
            uint64_t s1 = s0 + q.cmp_chunk;
            const uint64_t used = (uint64_t)nb * kBucket;
            if (s1 > used) s1 = used;
            for (uint64_t base = s0; base < s1; base += B) {
                uint64_t slot = base + tid;
                compact_slot<W>(a, t, slot, slot < s1, lh, wmax);
            }
            signal_done(q.cmp_done + rank);
        }
        __syncthreads();
    }
    flush_max(a.max_count, wmax);
    __syncthreads();
    for (uint32_t b = tid; b < kLdsHist; b += B)
        if (lh[b]) add_dev(&a.hist[b], (uint64_t)lh[b]);
}

template <int W, uint32_t B>
static hipError_t persistent_w(const CountArgs& a, const PersistArgs& q, uint32_t grid, hipStream_t s) {
    hipLaunchKernelGGL((k_count_persistent<W, B>), dim3(grid), dim3(B), 0, s, a, q);
    return hipGetLastError();
}

template <uint32_t B>
static hipError_t persistent_b(const CountArgs& a, const PersistArgs& q, uint32_t grid, hipStream_t s) {
    switch (a.W) {
        case 1: return persistent_w<1, B>(a, q, grid, s);
        case 2: return persistent_w<2, B>(a, q, grid, s);
        case 3: return persistent_w<3, B>(a, q, grid, s);
        case 4: return persistent_w<4, B>(a, q, grid, s);
        case 5: return persistent_w<5, B>(a, q, grid, s);
        case 6: return persistent_w<6, B>(a, q, grid, s);
        case 7: return persistent_w<7, B>(a, q, grid, s);
        case 8: return persistent_w<8, B>(a, q, grid, s);
        case 9: return persistent_w<9, B>(a, q, grid, s);
        case 10: return persistent_w<10, B>(a, q, grid, s);
        case 11: return persistent_w<11, B>(a, q, grid, s);
        case 12: return persistent_w<12, B>(a, q, grid, s);
        case 13: return persistent_w<13, B>(a, q, grid, s);
        case 14: return persistent_w<14, B>(a, q, grid, s);
        case 15: return persistent_w<15, B>(a, q, grid, s);
    }
    return hipErrorInvalidValue;
}

// One insert item is one descriptor per thread, so ins_chunk equals the block.
hipError_t launch_count_persistent(const CountArgs& a, const PersistArgs& q, uint32_t grid, uint32_t block,
                                   hipStream_t s) {
    if (q.ins_chunk != block) return hipErrorInvalidValue;
    switch (block) {
        case 256: return persistent_b<256>(a, q, grid, s);
        case 512: return persistent_b<512>(a, q, grid, s);
        case 1024: return persistent_b<1024>(a, q, grid, s);
    }
    return hipErrorInvalidValue;
}

template <int W, uint32_t B>
static uint32_t occupancy_wb() {
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_count_persistent<W, B>, B, 0) != hipSuccess ||
        blocks < 1)
        blocks = 1;
    return (uint32_t)blocks;
}

template <int W>
static uint32_t occupancy_w(uint32_t block) {
    return block == 1024 ? occupancy_wb<W, 1024>() : block == 512 ? occupancy_wb<W, 512>() : occupancy_wb<W, 256>();
}

uint32_t persistent_blocks_per_cu(uint32_t W, uint32_t block) {
    // zero-initialised; the same value from any thread (per device of one kind)
    static std::atomic<uint32_t> cached[3][GERBIL_MAX_W + 1];
    if (W < 1 || W > GERBIL_MAX_W) return 1;
    const uint32_t bi = block == 1024 ? 2 : block == 512 ? 1 : 0;
    if (const uint32_t c = cached[bi][W].load(std::memory_order_relaxed)) return c;
    uint32_t r = 1;
    switch (W) {
        case 1: r = occupancy_w<1>(block); break;
        case 2: r = occupancy_w<2>(block); break;
        case 3: r = occupancy_w<3>(block); break;
        case 4: r = occupancy_w<4>(block); break;
        case 5: r = occupancy_w<5>(block); break;
        case 6: r = occupancy_w<6>(block); break;
        case 7: r = occupancy_w<7>(block); break;
        case 8: r = occupancy_w<8>(block); break;
        case 9: r = occupancy_w<9>(block); break;
        case 10: r = occupancy_w<10>(block); break;
        case 11: r = occupancy_w<11>(block); break;
        case 12: r = occupancy_w<12>(block); break;
        case 13: r = occupancy_w<13>(block); break;
        case 14: r = occupancy_w<14>(block); break;
        case 15: r = occupancy_w<15>(block); break;
    }
    cached[bi][W].store(r, std::memory_order_relaxed);
    return r;
}

}  // namespace gerbil

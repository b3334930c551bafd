/*
 * gerbil.h -- C ABI of the MI355X (gfx950) k-mer counting library.
 *
 * The library implements the counting step of Gerbil (Erbert, Rechner and
 * Mueller-Hannemann, "Gerbil: A fast and memory-efficient k-mer counter with
 * GPU-support", arXiv 1607.06618): reads and k go in; canonical (k-mer, count)
 * pairs above a threshold and the count-of-counts histogram come out
 * (Sec. 1, problem statement; Sec. 2, two-phase method).
 *
 *   gerbil_encode     2-bit encoding of the reads and the table of valid
 *                     k-mer windows (Sec. 2.3.1 parser step; Sec. 2.4.1:
 *                     windows with an undetermined base are ignored).
 *   gerbil_bin        minimizer signatures and super-mers distributed over
 *                     bins (Sec. 2.1, Fig. 1; Sec. 3.1 ordering; App. A `-f`).
 *                     The paper's temporary files become device-resident bins.
 *   gerbil_count      each bin cut into canonical k-mers (Sec. 2.4.2) and
 *                     counted in open-addressing hash tables with double
 *                     hashing and at most theta trials (Sec. 2.2, Alg. 1;
 *                     Sec. 3.3.1 bucket scan; Sec. 3.4.3 emergency area with
 *                     sort-and-compress); output iff count >= threshold
 *                     (App. A `-l`).
 *   gerbil_histogram  number of distinct canonical k-mers per count value.
 *
 * Conventions shared by every call
 *   Memory      Every pointer argument named "device" is device memory owned
 *               by the caller. The library never allocates or frees device
 *               memory; workspaces are sized by the *_workspace queries and
 *               must stay alive (and untouched) while results that point
 *               into them are used.
 *   Streams     Calls enqueue work on `stream` (NULL = the default stream)
 *               and return without waiting, except where a call says it
 *               synchronises.
 *   Errors      Argument errors (GERBIL_EINVAL, GERBIL_EUNSUPPORTED) are
 *               returned before anything is enqueued. Data-dependent capacity
 *               errors are recorded in a device status word and reported by
 *               gerbil_result() as GERBIL_ECAPACITY together with the size
 *               that would have sufficed; results are then incomplete and
 *               must not be used. Launch failures return GERBIL_EDEVICE.
 *   Concurrency Calls on different streams with disjoint workspaces may run
 *               concurrently.
 *   Key layout  W = ceil(k/32) uint64 words per key; words 0..W-2 hold 32
 *               bases each with the first base in bits 63:62; word W-1 holds
 *               the remaining k-32(W-1) bases right-aligned. Bases use the
 *               2-bit code of App. C (A=0, C=1, G=2, T=3), so numeric order of
 *               keys (word 0 first) is lexicographic order.
 */
#ifndef GERBIL_H
#define GERBIL_H

#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GERBIL_OK = 0,
    GERBIL_EINVAL = -1,       /* bad argument or workspace too small          */
    GERBIL_EUNSUPPORTED = -2, /* valid in the paper, not compiled here        */
    GERBIL_ECAPACITY = -3,    /* a device-side capacity was exceeded          */
    GERBIL_EDEVICE = -4       /* launch failure or a device wait gave up      */
} gerbil_status;

/* Counting schedule. PLAIN: one launch sequence per bin, bins in order, the
 * host reads the bin sizes once. BATCHED: every bin of the run in one
 * persistent launch with work stealing over bins (no host synchronisation). */
enum { GERBIL_PLAIN = 0, GERBIL_BATCHED = 1 };

/* Total order on minimizers (Sec. 3.1). KMC2: canonical m-mers in A<C<G<T
 * order with those starting AAA or ACA moved behind all others. LEX: plain
 * lexicographic order (Fig. 1). TABLE: the rank of each canonical m-mer is
 * read from gerbil_params.rank_table (made by gerbil_order_table for the
 * other orders of Sec. 3.1, or by the caller); bin = rank mod n_bins. */
enum { GERBIL_ORDER_KMC2 = 0, GERBIL_ORDER_LEX = 1, GERBIL_ORDER_TABLE = 2 };

/* Where hash tables live. LDS (and AUTO): every bin, or hash slice of a large
 * bin, is split by key hash into sub-tables that one workgroup counts in LDS
 * (the hasher threads of Sec. 2.3.2 with their own tables). HBM: one
 * open-addressing table per bin in device memory, probed by every workgroup. */
enum { GERBIL_TABLE_AUTO = 0, GERBIL_TABLE_HBM = 1, GERBIL_TABLE_LDS = 2 };

/* Run parameters; mirrors the command line of App. A. Zero means default. */
typedef struct {
    uint32_t k;              /* k-mer length, 2 <= k <= 480 (App. A `-k`: 8..479). LDS tables take
                                k <= 256; AUTO uses HBM tables above that, and TABLE_LDS with
                                k > 256 is GERBIL_EUNSUPPORTED                                    */
    uint32_t m;              /* minimizer length, 1 <= m <= 15, m < k (App. A `-m`)              */
    uint32_t n_bins;         /* number of bins, 1..4096 (App. A `-f`, default 512)               */
    uint32_t threshold;      /* output iff count >= threshold, >= 1 (App. A `-l`, default 3)     */
    uint32_t canonical;      /* 1: count canonical k-mers (Sec. 2.4.2); 0: count each strand's  */
                             /* k-mers as read (`-d`, App. A). Other values: GERBIL_EINVAL.    */
    uint32_t order;          /* GERBIL_ORDER_*                                                   */
    const uint32_t* bin_map; /* device [4^m] canonical m-mer code -> bin, or NULL for
                                bin = rank mod n_bins                                             */
    uint32_t mode;           /* GERBIL_PLAIN or GERBIL_BATCHED                                   */
    uint32_t table;          /* GERBIL_TABLE_*                                                   */
    float load_factor;       /* k-mers per table slot when tables are sized: HBM tables (0, 0.95]
                                (k-mers bound the distinct keys), default 0.5; LDS sub-tables
                                (0, 4], default 0.8 (occurrences repeat, so more than one per
                                slot can fit; distinct keys beyond the slots take the emergency
                                area)                                                             */
    uint32_t max_probes;     /* theta of Alg. 1: trials before the emergency path; 0 = default
                                (8 buckets of 8 slots in HBM tables, 64 slots in LDS tables)     */
    uint32_t block;          /* threads per workgroup for counting, 64..1024 in steps of 64. HBM
                                tables: 0 = 256. LDS tables, BATCHED: 512 runs two 512-thread
                                workgroups per CU with 80 KB of LDS each (half-size tables whose
                                stages overlap on the CU); any other value one 1024-thread
                                workgroup per CU with 160 KB. LDS tables, PLAIN: always 1024     */
    uint32_t pool;           /* BATCHED: hash tables resident at once. LDS tables: key slots (ranks
                                scattered and not yet counted), 0 = 16, best a multiple of 8 (one
                                work queue per XCD); HBM tables: 0 = chosen from budget          */
    uint64_t overflow_cap;   /* emergency-area capacity in k-mer occurrences, rounded up to a power
                                of two, at most 2^31; 0 = 2^20. The workspace holds the area and
                                its counting table of twice as many slots                        */
    uint64_t superm_cap;     /* super-mer descriptor capacity; 0 = default estimate              */
    uint64_t table_budget;   /* bytes of workspace for hash tables; 0 = default                  */
    hipEvent_t* timing_events; /* optional hipEvent_t[2] recorded on the stream just before and just
                                  after the main counting kernel(s): the persistent kernel (BATCHED)
                                  or the per-bin insert and dump launches (PLAIN); NULL = none      */
    uint64_t* stage_clocks;  /* optional device uint64[8], zeroed by the caller: busy time (in
                                units of the 100 MHz wall clock) of the four LDS stages (count,
                                scan, scatter, table) in [0..3] and their item counts in [4..7];
                                NULL = none                                                       */
    uint32_t size_sample;    /* LDS tables: sub-table runs are sized from a sample, every
                                size_sample-th segment of 32/size_sample k-mers (a run holds
                                size_sample x its sampled keys plus a four-sigma margin; if a run
                                still overflows, all of its keys take the emergency area, so
                                results stay exact); 1 = count every k-mer; 0 = default 8       */
    uint32_t reserved0;
    const uint32_t* rank_table; /* order TABLE: device uint32 [4^m], the rank of each canonical m-mer
                                code (distinct ranks below 0xFFFFFFFF; entries of other codes are
                                never read). bin_map must be NULL with this order.               */
    uint64_t* probe_hist;    /* optional device uint64[GERBIL_PROBE_HIST], zeroed by the caller; LDS
                                tables, BATCHED: entry t (1 <= t < GERBIL_PROBE_HIST - 1) counts the
                                k-mer occurrences whose insert ended at its t-th probe, the last
                                entry those that needed more or took the emergency area, entry 0
                                the occurrences sent to the emergency area without a probe (the
                                probe statistic of Sec. 3.3.1). NULL = none (no cost)             */
} gerbil_params;

#define GERBIL_PROBE_HIST 32

/* Output of gerbil_encode. All pointers point into the encode workspace. */
typedef struct {
    uint64_t n_reads;
    uint64_t n_bytes;        /* total ASCII bytes = offsets[n_reads]                  */
    uint32_t k;
    uint32_t reserved;
    uint64_t n_words;        /* ceil(n_bytes / 32) packed words                       */
    uint64_t n_mask;         /* ceil(n_bytes / 64) bitmask words                      */
    uint64_t* packed;        /* device [n_words]; packed[-1] and packed[n_words..+1]
                                exist and are zero. Byte i -> word i/32, bits
                                63-2(i%32)..62-2(i%32); non-ACGT bytes are code 0     */
    uint64_t* valid;         /* device bitmask [n_mask+1]: bit i = byte i is ACGT/acgt */
    uint64_t* read_start;    /* device bitmask [n_mask+1]: bit i = a read starts at i  */
    uint64_t* kmer_ok;       /* device bitmask [n_mask+1]: bit p = window [p, p+k) is
                                inside one read and has only valid bases              */
    uint64_t* n_valid;       /* device scalar: number of valid windows               */
    uint32_t* status;        /* device scalar: error bits                              */
} gerbil_encoded;

/* Output of gerbil_bin: super-mers grouped by bin (the temporary files of
 * Sec. 2.1). A super-mer is stored as a descriptor into the packed reads:
 * desc = (global position of its first base << 24) | number of k-mers. */
typedef struct {
    uint32_t k, m, n_bins, tile;
    uint64_t cap_superm;     /* capacity of desc                                      */
    uint64_t n_bytes;
    const uint64_t* packed;  /* the encoded reads (not owned)                         */
    uint64_t* desc;          /* device [cap_superm], bin-ordered                      */
    uint64_t* bin_off;       /* device [n_bins+1]: bin b owns desc[bin_off[b]..bin_off[b+1]) */
    uint64_t* bin_kmers;     /* device [n_bins]: k-mers per bin                       */
    uint64_t* n_superm;      /* device scalar: super-mers found (may exceed cap)      */
    uint32_t* status;        /* device scalar: error bits (shared with the encoding)  */
} gerbil_bins;

/* State of one gerbil_count call; pointers point into the count workspace. */
typedef struct {
    uint32_t k, W, threshold, hist_len;
    uint64_t cap;            /* capacity of the caller's output arrays (pairs)        */
    uint64_t overflow_cap;
    uint64_t* n_out;         /* device scalar: pairs emitted (or needed, if > cap)    */
    uint64_t* hist;          /* device [hist_len]: internal count-of-counts           */
    uint64_t* n_overflow;    /* device scalar: k-mer occurrences sent to the emergency area */
    uint64_t* max_count;     /* device scalar                                         */
    uint32_t* status;        /* device scalar: error bits                             */
    uint64_t* n_superm;      /* copied from the bins                                  */
    uint32_t* bin_status;
} gerbil_counted;

/* What gerbil_result reads back from the device. */
typedef struct {
    uint64_t n_valid;        /* valid windows of the input                            */
    uint64_t n_superm;       /* super-mers (descriptors needed)                       */
    uint64_t n_out;          /* pairs emitted (or needed)                             */
    uint64_t n_overflow;     /* k-mer occurrences that used the emergency area        */
    uint64_t max_count;      /* largest count seen                                    */
    uint32_t status;         /* device error bits                                     */
    uint32_t reserved;
} gerbil_report;

/* Library version as 0xMMmmpp. */
uint32_t gerbil_version(void);

/* Static text for a status code. */
const char* gerbil_status_string(int32_t status);

/* Workspace bytes gerbil_encode needs for n_bytes of ASCII and n_reads reads.
 * Errors: GERBIL_EINVAL if bytes is NULL or k is out of range. */
int32_t gerbil_encode_workspace(uint64_t n_reads, uint64_t n_bytes, uint32_t k, uint64_t* bytes);

/* 2-bit encode reads and mark every valid k-mer window (Sec. 2.3.1 parser
 * step; Sec. 2.4.1 N handling; App. C base code).
 *   ascii    device uint8 [n_bytes]: concatenated reads (any bytes; only
 *            A/C/G/T in either case are bases, anything else invalidates the
 *            windows that contain it)
 *   offsets  device uint64 [n_reads+1]: read r is ascii[offsets[r], offsets[r+1]);
 *            offsets[0] = 0, non-decreasing, offsets[n_reads] = n_bytes
 *   k        window length (2..480)
 *   ws       device workspace of at least gerbil_encode_workspace() bytes,
 *            256-byte aligned
 *   out      host struct filled with pointers into ws
 * A mismatch between offsets[n_reads] and n_bytes is reported by
 * gerbil_result (GERBIL_EINVAL). */
int32_t gerbil_encode(const uint8_t* ascii, const uint64_t* offsets, uint64_t n_reads, uint64_t n_bytes,
                      uint32_t k, void* ws, uint64_t ws_bytes, gerbil_encoded* out, hipStream_t stream);

/* Workspace bytes gerbil_bin needs. Errors: GERBIL_EINVAL on bad params. */
int32_t gerbil_bin_workspace(const gerbil_encoded* enc, const gerbil_params* p, uint64_t* bytes);

/* Split the encoded reads into super-mers by minimizer and group them by bin
 * (Sec. 2.1, Fig. 1; Sec. 3.1; Sec. 2.3.1 splitter step). The minimizer of a
 * k-mer is its smallest canonical m-mer under the chosen order; a super-mer
 * is a maximal run of consecutive k-mers with equal minimizers, additionally
 * cut every `tile` positions. enc must come from gerbil_encode with the same
 * k and stay alive. Exceeding p->superm_cap is reported as GERBIL_ECAPACITY
 * by gerbil_result, with the needed count in n_superm. */
int32_t gerbil_bin(const gerbil_encoded* enc, const gerbil_params* p, void* ws, uint64_t ws_bytes,
                   gerbil_bins* out, hipStream_t stream);

/* Workspace bytes gerbil_count needs for these bins. SYNCHRONISES `stream`
 * (only that stream): reads the per-bin k-mer counts from the device to size
 * the hash tables, so gerbil_bin must have been enqueued on `stream`. */
int32_t gerbil_count_workspace(const gerbil_bins* bins, const gerbil_params* p, uint64_t* bytes,
                               hipStream_t stream);

/* Count the canonical k-mers of every bin (Sec. 2.2, Alg. 1; Sec. 2.3.2;
 * Sec. 3.3.1; Sec. 3.4) and emit the pairs with count >= p->threshold.
 *   keys     device uint64 [cap * W]: pair i's key in keys[i*W .. i*W+W-1]
 *   counts   device uint32 [cap]
 *   cap      capacity in pairs; n_valid / threshold always suffices
 *   ws       workspace of gerbil_count_workspace() bytes (256-byte aligned)
 *   state    host struct filled with pointers into ws (n_out, histogram ...)
 * Pair order is unspecified. PLAIN mode synchronises once to read the bin
 * sizes; BATCHED mode does not synchronise. */
int32_t gerbil_count(const gerbil_bins* bins, const gerbil_params* p, void* ws, uint64_t ws_bytes,
                     uint64_t* keys, uint32_t* counts, uint64_t cap, gerbil_counted* state, hipStream_t stream);

/* Count-of-counts over every distinct canonical k-mer, before the threshold
 * (the k-mer histogram of the problem statement, Sec. 1, and of the `-x h`
 * option of App. A, read as the number of k-mers per count value so that
 * sum_c c * hist[c] equals the number of valid windows):
 * hist[c] = number of k-mers with count c for 1 <= c < len-1, hist[len-1] =
 * number with count >= len-1, hist[0] = 0.
 *   hist     device uint64 [len], 2 <= len <= 65536 */
int32_t gerbil_histogram(const gerbil_counted* state, uint64_t* hist, uint32_t len, hipStream_t stream);

/* Read the device-side counters and status of a finished run. SYNCHRONISES
 * on `stream`. Any of enc, bins, state may be NULL. Returns GERBIL_OK,
 * GERBIL_ECAPACITY (a capacity was exceeded; the report holds the needed
 * sizes), GERBIL_EINVAL (offsets inconsistent) or GERBIL_EDEVICE. */
int32_t gerbil_result(const gerbil_encoded* enc, const gerbil_bins* bins, const gerbil_counted* state,
                      gerbil_report* report, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Whole-path replay. The batched path (encode -> bin -> count -> histogram)
 * is a fixed sequence of kernel launches with no host synchronisation, so
 * for inputs of one shape it can be recorded once into a HIP graph and
 * replayed with a single launch per batch (the paper's pipeline of
 * Sec. 2.3 without per-step host work). Sizing needs the bin sizes, so
 * gerbil_count_workspace must be called beforehand (an eager first run).
 * ------------------------------------------------------------------------ */

/* Buffers of one run of the whole path (all device pointers owned by the caller). */
typedef struct {
    const uint8_t* ascii;      /* device uint8 [n_bytes]                                   */
    const uint64_t* offsets;   /* device uint64 [n_reads+1]                                */
    uint64_t n_reads;
    uint64_t n_bytes;
    void* ws_encode;           /* gerbil_encode_workspace() bytes                          */
    uint64_t ws_encode_bytes;
    void* ws_bin;              /* gerbil_bin_workspace() bytes                             */
    uint64_t ws_bin_bytes;
    void* ws_count;            /* gerbil_count_workspace() bytes                           */
    uint64_t ws_count_bytes;
    uint64_t* keys;            /* device uint64 [cap * W]                                  */
    uint32_t* counts;          /* device uint32 [cap]                                      */
    uint64_t cap;
    uint64_t* hist;            /* device uint64 [hist_len]                                 */
    uint32_t hist_len;
    uint32_t reserved;
} gerbil_pipeline;

typedef struct gerbil_graph gerbil_graph;

/* Record encode -> bin -> count -> histogram of `pl` into a graph (stream
 * capture on `stream`, which must not be the NULL stream; nothing runs
 * during the capture). p->mode must be GERBIL_BATCHED (GERBIL_EUNSUPPORTED
 * otherwise); p->timing_events is ignored. enc, bins and state are filled as
 * by the individual calls and describe the results of every replay. The
 * graph holds kernel nodes only (no memset or copy nodes); any other node
 * makes the call fail with GERBIL_EUNSUPPORTED. On success *out owns a host
 * object released by gerbil_graph_destroy; the buffers of `pl` must outlive it. */
int32_t gerbil_graph_capture(const gerbil_pipeline* pl, const gerbil_params* p, gerbil_encoded* enc,
                             gerbil_bins* bins, gerbil_counted* state, hipStream_t stream, gerbil_graph** out);

/* Enqueue one replay on `stream`. Results and status are read with
 * gerbil_result as after the individual calls. Replays on one graph must not
 * overlap (they share the workspaces). */
int32_t gerbil_graph_launch(const gerbil_graph* g, hipStream_t stream);

/* Number of nodes, and of kernel nodes, in the recorded graph. */
int32_t gerbil_graph_info(const gerbil_graph* g, uint32_t* n_nodes, uint32_t* n_kernel_nodes);

/* Release the graph (NULL is ignored). The caller ensures no replay is still running. */
int32_t gerbil_graph_destroy(gerbil_graph* g);

/* ------------------------------------------------------------------------
 * Autotuner. The paper chooses thread counts at run time and re-estimates
 * table sizes from the data (Sec. 2.3; Sec. 3.4.1); here the schedule's
 * free parameters are chosen by timing them on the caller's bins.
 * ------------------------------------------------------------------------ */

/* What gerbil_autotune chose. */
typedef struct {
    uint32_t table;          /* GERBIL_TABLE_LDS or GERBIL_TABLE_HBM                     */
    float load_factor;       /* chosen gerbil_params.load_factor                         */
    uint32_t pool;           /* chosen gerbil_params.pool (0 in PLAIN mode)              */
    uint32_t candidates;     /* candidates timed (0 when the choice came from the cache) */
    uint32_t cached;         /* 1 if the choice came from the cache                      */
    float best_ms;           /* time of one gerbil_count with the choice                 */
    uint32_t block;          /* chosen gerbil_params.block (LDS: 1024 or 512 threads per
                                workgroup; HBM: 256, 512 or 1024)                            */
} gerbil_tune_result;

/* Workspace bytes that fit every candidate of gerbil_autotune for these
 * bins (the largest gerbil_count_workspace over them). SYNCHRONISES `stream`. */
int32_t gerbil_autotune_workspace(const gerbil_bins* bins, const gerbil_params* p, uint64_t* bytes,
                                  hipStream_t stream);

/* Time gerbil_count on `bins` for each candidate of the grid (LDS tables:
 * load_factor 0.6/0.8/1.0/1.2 x pool 8/16/24 x block 1024/512; HBM tables:
 * load_factor 0.4/0.6 x pool 8/32 x block 256/512/1024; p->table = LDS or
 * HBM restricts the grid to that placement; PLAIN mode has no pool and LDS
 * tables only block 1024) and write into *best a copy of *p with table,
 * load_factor, pool and block of the fastest candidate that finished without
 * a capacity error (one warm-up run, then one timed run per candidate). Candidates whose workspace exceeds ws_bytes are skipped.
 * keys/counts/cap serve as the output of the trial runs (their contents are
 * overwritten). The choice is cached per (device, ceil(k/32), m, n_bins,
 * mode, p->table, and the total, largest and median bin size in quarter
 * octaves); a later call with the same profile returns the cached choice
 * without running anything (info->cached = 1). SYNCHRONISES `stream`.
 * Errors: GERBIL_EINVAL (bad arguments, or no candidate fits ws_bytes),
 * GERBIL_ECAPACITY (cap too small, or every candidate ran out of a
 * capacity), GERBIL_EDEVICE. */
int32_t gerbil_autotune(const gerbil_bins* bins, const gerbil_params* p, void* ws, uint64_t ws_bytes,
                        uint64_t* keys, uint32_t* counts, uint64_t cap, gerbil_params* best,
                        gerbil_tune_result* info, hipStream_t stream);

/* Forget every cached autotuner choice. */
int32_t gerbil_autotune_reset(void);

/* ------------------------------------------------------------------------
 * Output records (App. C): the binary file format of the counted pairs.
 * ------------------------------------------------------------------------ */

/* Workspace bytes gerbil_records needs for n pairs. */
int32_t gerbil_records_workspace(uint64_t n, uint64_t* bytes);

/* Encode n pairs as the binary records of App. C, back to back in pair order:
 * the counter (one byte if it is below 255, else the byte 0xFF and the count
 * as a big-endian 32-bit word), then the k-mer with four bases per byte, the
 * first base in the two top bits, and the last byte padded with zero bits.
 *   keys       device uint64 [n * W] (the layout gerbil_count emits)
 *   counts     device uint32 [n]
 *   ws         device workspace of gerbil_records_workspace(n) bytes, 256-byte aligned
 *   out        device byte buffer of out_cap bytes
 *   out_bytes  device uint64: receives the size of the whole stream. Bytes
 *              past out_cap are not written; a caller whose buffer was too
 *              small calls again with out_cap >= *out_bytes.
 * Asynchronous on `stream`. Errors: GERBIL_EINVAL (bad arguments or
 * workspace), GERBIL_EDEVICE (launch). */
int32_t gerbil_records(const uint64_t* keys, const uint32_t* counts, uint64_t n, uint32_t k, void* ws,
                       uint64_t ws_bytes, uint8_t* out, uint64_t out_cap, uint64_t* out_bytes, hipStream_t stream);

/* Largest n that gerbil_records_noalloc takes: 2^29 pairs (65536 tiles of 8192). */
#define GERBIL_RECORDS_NOALLOC_MAX 536870912ull

/* gerbil_records without a workspace, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation. Nothing is allocated by this call or by the library for
 * it (no hipMalloc, no allocating library routine): the per-tile scratch that
 * gerbil_records keeps in its workspace lives in one static device array of
 * the library, 786,688 bytes on each GPU that calls it, held until the process
 * ends. Arguments and results are those of gerbil_records (the caller still
 * provides keys, counts, out and out_bytes), with n <= GERBIL_RECORDS_NOALLOC_MAX.
 * The scratch of a GPU is shared by every call on that GPU and keeps the last
 * call's contents (each call writes every entry it reads): calls that overlap
 * on one GPU (on different streams, or from different threads) race and must
 * be serialised by the caller. The first call on a device looks up the
 * array's address on that device (synchronous; not a stream operation).
 * Errors: GERBIL_EINVAL (bad arguments, n above the maximum), GERBIL_EDEVICE. */
int32_t gerbil_records_noalloc(const uint64_t* keys, const uint32_t* counts, uint64_t n, uint32_t k, uint8_t* out,
                               uint64_t out_cap, uint64_t* out_bytes, hipStream_t stream);

/* Bin of each of n keys (the layout gerbil_count emits) under the binning of
 * `p` (k, m, n_bins, order, bin_map, rank_table): the bin that gerbil_bin
 * sends every occurrence of the key to (Sec. 2.1, Sec. 3.1). With counts of
 * every key (threshold 1) this gives the distinct k-mers of each bin, the
 * quantity the table-size estimate of Sec. 3.4.1 predicts.
 *   keys   device uint64 [n * W];  bins  device uint32 [n]
 * Asynchronous on `stream`. Errors: GERBIL_EINVAL, GERBIL_EUNSUPPORTED, GERBIL_EDEVICE. */
int32_t gerbil_key_bins(const uint64_t* keys, uint64_t n, const gerbil_params* p, uint32_t* bins,
                        hipStream_t stream);

/* HyperLogLog sketch of the distinct k-mers of every bin, from the k-mer
 * occurrences of its super-mers: the alternative to the ratio estimate of
 * Sec. 3.4.1 (it needs no counting). Register j of bin b is the largest
 * rank of the first set bit, after the top log2_regs bits, of the 64-bit
 * hash of a key whose top bits are j (the usual HyperLogLog update); the
 * estimate is formed by the caller.
 *   bins       the output of gerbil_bin (its workspace still valid)
 *   p          the parameters the bins were made with (k, canonical)
 *   log2_regs  4..15 registers per bin as a power of two
 *   regs       device uint32 [n_bins << log2_regs], every register written
 * Asynchronous on `stream`. Errors: GERBIL_EINVAL, GERBIL_EUNSUPPORTED, GERBIL_EDEVICE. */
int32_t gerbil_hll_bins(const gerbil_bins* bins, const gerbil_params* p, uint32_t log2_regs, uint32_t* regs,
                        hipStream_t stream);

/* ------------------------------------------------------------------------
 * Minimizer orders (Sec. 3.1) as rank tables for GERBIL_ORDER_TABLE.
 * ------------------------------------------------------------------------ */

enum {
    GERBIL_RANKS_KMC2 = 0,    /* the KMC2 order (also built into GERBIL_ORDER_KMC2)               */
    GERBIL_RANKS_LEX = 1,     /* A<C<G<T (also built into GERBIL_ORDER_LEX)                        */
    GERBIL_RANKS_CGAT = 2,    /* lexicographic with C<G<A<T                                        */
    GERBIL_RANKS_ROBERTS = 3, /* Roberts et al.: bases at even positions (counting from 1)
                                 complemented, then lexicographic with C<A<T<G                     */
    GERBIL_RANKS_RANDOM = 4,  /* canonical m-mers sorted by the top 30 bits of SplitMix64 output
                                 number `code` of `seed` (ties by code); rank = position          */
    GERBIL_RANKS_DFP = 5      /* dfp(pivot): canonical m-mers sorted by sampled frequency (ties by
                                 code), re-sorted by distance of the position from
                                 floor(pivot * M), M = number of canonical m-mers (ties: lower
                                 position first); rank = final position                          */
};

/* Workspace bytes of gerbil_order_table (0 for the orders without a sort). */
int32_t gerbil_order_table_workspace(uint32_t kind, uint32_t m, uint64_t* bytes);

/* Rank table of one minimizer order: table[c] is the rank of canonical m-mer
 * code c; every other entry is 0xFFFFFFFF.
 *   kind     GERBIL_RANKS_*; m in 1..15 (RANDOM and DFP: 1..12)
 *   seed     RANDOM: generator seed
 *   pivot    DFP: pivot factor in [0, 1]
 *   stride, enc
 *            DFP: the frequency sample is the canonical m-mer that starts
 *            each valid k-mer window (gerbil_encode's bitmap, m < enc->k)
 *            whose position is a multiple of stride (0 = 16)
 *   ws       device workspace of gerbil_order_table_workspace bytes, 256-byte aligned
 *   table    device uint32 [4^m]
 * Asynchronous on `stream`. Errors: GERBIL_EINVAL, GERBIL_EDEVICE. */
int32_t gerbil_order_table(uint32_t kind, uint32_t m, uint64_t seed, float pivot, uint32_t stride,
                           const gerbil_encoded* enc, void* ws, uint64_t ws_bytes, uint32_t* table,
                           hipStream_t stream);

/* ------------------------------------------------------------------------
 * Input parsing (the formats of App. B): FASTA or FASTQ text in device
 * memory to the CSR reads gerbil_encode takes.
 * ------------------------------------------------------------------------ */

enum { GERBIL_FORMAT_DETECT = 0, GERBIL_FORMAT_FASTQ = 1, GERBIL_FORMAT_FASTA = 2 };

/* Status bits of a parse (gerbil_parsed.status); 0 = the reads are valid. */
#define GERBIL_PARSE_EHEADER 0x001u  /* FASTQ: a record's first line is empty or lacks '@'        */
#define GERBIL_PARSE_EPLUS 0x002u    /* FASTQ: a record's third line does not start with '+'     */
#define GERBIL_PARSE_EQUAL 0x004u    /* FASTQ: quality and sequence lengths differ               */
#define GERBIL_PARSE_ELINES 0x008u   /* FASTQ: line count not a multiple of four                 */
#define GERBIL_PARSE_EORPHAN 0x010u  /* FASTA: sequence bytes before the first '>' header        */
#define GERBIL_PARSE_EBYTES 0x020u   /* sequence bytes exceed seq_cap (nothing written past it)  */
#define GERBIL_PARSE_EREADS 0x040u   /* reads exceed reads_cap (nothing written past it)         */
#define GERBIL_PARSE_EFORMAT 0x080u  /* detection: the text starts with neither '@' nor '>'      */
#define GERBIL_PARSE_ELINECAP 0x100u /* more lines than lines_cap: no read was produced          */

typedef struct {
    uint64_t n_reads;  /* reads found (FASTQ sequence lines, FASTA '>' headers)              */
    uint64_t n_bytes;  /* sequence bytes over all sequence lines                              */
    uint64_t n_lines;  /* lines of the text (a final line without a newline counts)          */
    uint32_t status;   /* GERBIL_PARSE_* bits                                                  */
    uint32_t format;   /* the format parsed (0: empty text or not detected)                   */
} gerbil_parsed;

/* Workspace bytes of gerbil_parse for n text bytes and up to lines_cap lines. */
int32_t gerbil_parse_workspace(uint64_t n, uint64_t lines_cap, uint64_t* bytes);

/* Parse FASTA or FASTQ text (the input formats named in App. B; compressed
 * and staden inputs are not handled). Lines end at '\n'; a final line may
 * lack it; one '\r' right before a line's end is dropped. FASTQ: records of
 * four lines ('@' header, sequence, '+' line, quality of the sequence's
 * length); each sequence line is one read. FASTA: a line starting with '>'
 * starts a read and every other line is appended to the current read. Read
 * bytes are copied unchanged; gerbil_encode decides which are bases.
 *   text       device bytes [n], any alignment, n < 2^40
 *   format     GERBIL_FORMAT_*; DETECT looks at the first byte ('@' or '>')
 *   ws         device workspace of gerbil_parse_workspace(n, lines_cap) bytes,
 *              256-byte aligned
 *   seq        device bytes [seq_cap]: the reads back to back (seq_cap = n
 *              always suffices)
 *   offsets    device uint64 [reads_cap + 1]: read r is seq[offsets[r],
 *              offsets[r+1])
 *   out        device gerbil_parsed: counts and status, written by the parse
 * Asynchronous on `stream`; the caller reads *out after synchronising. The
 * reads are defined when out->status is 0; with EBYTES, EREADS or ELINECAP
 * the counts in *out tell the capacities to call again with. Errors returned
 * here: GERBIL_EINVAL (bad arguments or workspace), GERBIL_EDEVICE. */
int32_t gerbil_parse(const uint8_t* text, uint64_t n, uint32_t format, void* ws, uint64_t ws_bytes,
                     uint64_t lines_cap, uint8_t* seq, uint64_t seq_cap, uint64_t* offsets, uint64_t reads_cap,
                     gerbil_parsed* out, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Device ceilings (measurement only; nothing on the counting path uses
 * them). Alg. 1 and the bucket scan of Sec. 3.3.1 are bound by random
 * accesses and atomics, not by streaming, so inserts per second are
 * reported next to the rates the device sustains for the same access kinds.
 * ------------------------------------------------------------------------ */

enum {
    GERBIL_CEIL_LDS_CAS = 0,  /* 64-bit compare-and-swap with return, random slots of a 16384-slot
                                 LDS table per workgroup (the claim of an LDS table insert)         */
    GERBIL_CEIL_LDS_ADD = 1,  /* 32-bit add without return, random words of a 32768-word LDS array
                                 per workgroup (the counter update)                                 */
    GERBIL_CEIL_HBM_ADD = 2,  /* 32-bit device-scope add without return, random 64-byte lines of buf */
    GERBIL_CEIL_HBM_CAS = 3,  /* 64-bit device-scope compare-and-swap with return, random lines     */
    GERBIL_CEIL_HBM_LOAD = 4, /* 64-bit device-coherent load, random lines                           */
    GERBIL_CEIL_ONE_ADDR = 5  /* device-scope add with return on the first word of buf, by lane 0 of
                                 every wave (a shared work-queue cursor)                            */
};

/* One launch of `grid` workgroups of 1024 threads; each thread performs
 * `iters` operations of `kind` at pseudo-random positions (ONE_ADDR: lane 0
 * of each of the 16 waves of a workgroup performs `iters` dependent adds).
 * Operations in the launch: grid * 1024 * iters (ONE_ADDR: grid * 16 * iters);
 * the caller times the launch on `stream`.
 *   buf    device memory for the HBM kinds and ONE_ADDR: buf_bytes >= 64, a
 *          multiple of 64, 64-byte aligned; overwritten. NULL for the LDS kinds.
 *   sink   device uint64 [grid * 1024]: one checksum per thread (so that no
 *          operation is optimised away); overwritten.
 * Asynchronous on `stream`. Errors: GERBIL_EINVAL (kind, sizes or pointers),
 * GERBIL_EDEVICE (launch). */
int32_t gerbil_ceiling(uint32_t kind, void* buf, uint64_t buf_bytes, uint32_t grid, uint32_t iters, uint64_t* sink,
                       hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* GERBIL_H */

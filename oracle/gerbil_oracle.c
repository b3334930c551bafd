/*
 * CPU oracle for canonical k-mer counting (Gerbil, arXiv 1607.06618).
 *
 * TEST INFRASTRUCTURE ONLY. Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may call this code. The GPU library never links
 * it and shares no code with it.
 *
 * Everything here is the plain definition, written for a reader to check by
 * eye, single-threaded and slow on purpose:
 *
 *   oracle_count      Sec. 1 (problem statement), Sec. 2.4.1 (k-mers with an
 *                     undetermined base are ignored), Sec. 2.4.2 (canonical
 *                     form = lexicographically smaller of a k-mer and its
 *                     reverse complement), App. A `-l` (output iff count >=
 *                     threshold). Bins, minimizers and hash tables reach this
 *                     same result (Sec. 2.1: all occurrences of a k-mer land in
 *                     one temporary file; Sec. 3.4.3: the emergency path loses
 *                     nothing), so the oracle uses none of them: windows ->
 *                     strings -> canonical string -> packed key -> qsort ->
 *                     run-length.
 *   oracle_encode     App. C 2-bit code (A=00, C=01, G=10, T=11), first base
 *                     most significant; which windows are valid (Sec. 2.4.1).
 *   oracle_supermers  Sec. 2.1 and Fig. 1: the minimizer of a k-mer is its
 *                     smallest m-mer under a total order; a super-mer is a
 *                     maximal run of consecutive k-mers sharing a minimizer.
 *                     Order of Sec. 3.1 (KMC2 item) as read below.
 *   oracle_record     App. C output record (variable-length counter + k-mer,
 *                     four bases per byte).
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *   - valid bases are A, C, G, T in either case; any other byte invalidates
 *     every window that contains it;
 *   - windows never span two reads;
 *   - key layout: W = ceil(k/32) 64-bit words; words 0..W-2 hold 32 bases each
 *     with the first base in bits 63:62; word W-1 holds the remaining
 *     r = k - 32(W-1) bases right-aligned;
 *   - minimizers use canonical m-mers (the smaller of the m-mer and its reverse
 *     complement), so that a k-mer and its reverse complement fall in the same
 *     bin; the KMC2-style order ranks a canonical m-mer code c as c + 4^m when
 *     it starts with AAA or ACA, else c; the plain order ranks it c;
 *   - bin = rank mod n_bins, or bin_map[c] when a map is given;
 *   - a count of 2^32 - 1 or more is an error (counters are 32-bit, App. C).
 */
#define _GNU_SOURCE
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_EINVAL -1
#define ORACLE_ENOMEM -2
#define ORACLE_ECOUNT -3
#define ORACLE_ECAP -4

/* ---------------------------------------------------------------- bases -- */

static int base_ok(uint8_t c) {
    return c == 'A' || c == 'C' || c == 'G' || c == 'T' || c == 'a' || c == 'c' || c == 'g' || c == 't';
}

static char upper(uint8_t c) { return (c >= 'a' && c <= 'z') ? (char)(c - 'a' + 'A') : (char)c; }

/* Watson-Crick complement: A<->T, C<->G (Sec. 2.4.2). */
static char complement(char c) {
    switch (c) {
        case 'A': return 'T';
        case 'T': return 'A';
        case 'C': return 'G';
        case 'G': return 'C';
    }
    return '?';
}

/* 2-bit code of App. C: A=00, C=01, G=10, T=11. */
static uint64_t code2(char c) {
    switch (c) {
        case 'A': return 0;
        case 'C': return 1;
        case 'G': return 2;
        case 'T': return 3;
    }
    return 0;
}

static uint32_t words_for(uint32_t k) { return (k + 31) / 32; }

/* Pack k uppercase bases: base j goes into word j/32, shifted in from the
 * right, so the first base of each word ends up most significant and the last
 * word is right-aligned. */
static void pack(const char* s, uint32_t k, uint64_t* w) {
    uint32_t W = words_for(k);
    for (uint32_t i = 0; i < W; i++) w[i] = 0;
    for (uint32_t j = 0; j < k; j++) w[j / 32] = (w[j / 32] << 2) | code2(s[j]);
}

/* Reverse complement of the string s (length n) into t. */
static void reverse_complement(const char* s, uint32_t n, char* t) {
    for (uint32_t j = 0; j < n; j++) t[n - 1 - j] = complement(s[j]);
}

/* The window ascii[p, p+n) is valid iff every byte is A, C, G or T. */
static int window_ok(const uint8_t* p, uint32_t n) {
    for (uint32_t j = 0; j < n; j++)
        if (!base_ok(p[j])) return 0;
    return 1;
}

/* --------------------------------------------------------- shard filter -- */

/* FNV-1a over the key's bytes, used only to split the oracle's work into
 * memory-bounded passes and to select the same keys on the GPU side. */
uint64_t oracle_shard_of(const uint64_t* key, uint32_t W, uint64_t shard_mod) {
    uint64_t h = 1469598103934665603ull;
    for (uint32_t i = 0; i < W; i++)
        for (int b = 0; b < 8; b++) {
            h ^= (key[i] >> (8 * b)) & 0xFF;
            h *= 1099511628211ull;
        }
    return shard_mod ? h % shard_mod : 0;
}

/* ------------------------------------------------------------- counting -- */

typedef struct {
    uint64_t n_valid;       /* all valid windows of the input                  */
    uint64_t n_valid_shard; /* valid windows whose canonical key is in shard   */
    uint64_t n_distinct;    /* distinct canonical keys in the shard            */
    uint64_t n_pairs;       /* distinct keys with count >= threshold           */
    uint64_t* keys;         /* [n_pairs * W], ascending                        */
    uint32_t* counts;       /* [n_pairs]                                       */
    uint64_t* hist;         /* [hist_len]; hist[c] = #distinct with count c    */
    uint64_t hist_len;      /* max_count + 1                                   */
    uint64_t max_count;
} oracle_result;

static int cmp_keys(const void* a, const void* b, void* ctx) {
    uint32_t W = *(const uint32_t*)ctx;
    const uint64_t* x = (const uint64_t*)a;
    const uint64_t* y = (const uint64_t*)b;
    for (uint32_t i = 0; i < W; i++)
        if (x[i] != y[i]) return x[i] < y[i] ? -1 : 1;
    return 0;
}

void oracle_free(oracle_result* r) {
    free(r->keys); free(r->counts); free(r->hist);
    memset(r, 0, sizeof(*r));
}

/*
 * A growable array of keys of W words each. Used to hand the keys of one
 * shard from the collecting step to the counting step.
 */
typedef struct {
    uint64_t* keys;   /* [cap * W] */
    uint64_t n;       /* keys held */
    uint64_t cap;     /* keys allocated; a caller may preset it before the first push */
} oracle_keys;

void oracle_keys_free(oracle_keys* a) {
    free(a->keys);
    a->keys = NULL;
    a->n = a->cap = 0;
}

static int keys_push(oracle_keys* a, const uint64_t* key, uint32_t W) {
    if (!a->keys || a->n == a->cap) {
        uint64_t cap = a->keys ? a->cap + a->cap / 4 + 1024 : (a->cap ? a->cap : 1024);
        uint64_t* grown = (uint64_t*)realloc(a->keys, cap * 8 * W);
        if (!grown) return ORACLE_ENOMEM;
        a->keys = grown;
        a->cap = cap;
    }
    memcpy(a->keys + a->n * W, key, 8 * W);
    a->n++;
    return ORACLE_OK;
}

/*
 * Steps 1-5 of the definition over reads [r0, r1): every window of every read
 * (windows never span two reads); windows holding a byte other than A, C, G, T
 * (either case) are skipped (Sec. 2.4.1); the key is the lexicographically
 * smaller of the window and its reverse complement (Sec. 2.4.2), or the window
 * itself when canonical == 0 (App. A `-d`); it is packed into W words.
 * A key whose shard s = oracle_shard_of(key, W, shard_mod) lies in
 * [s_lo, s_hi) is appended to outs[s - s_lo]. *n_valid receives the number of
 * valid windows of the range (all shards).
 */
int oracle_collect(const uint8_t* ascii, const uint64_t* offsets, uint64_t r0, uint64_t r1, uint32_t k,
                   uint32_t canonical, uint64_t shard_mod, uint64_t s_lo, uint64_t s_hi,
                   oracle_keys* outs /* [s_hi - s_lo] */, uint64_t* n_valid) {
    *n_valid = 0;
    if (k < 1 || k > 1024 || s_hi <= s_lo) return ORACLE_EINVAL;
    uint32_t W = words_for(k);
    char* s = (char*)malloc(k);
    char* t = (char*)malloc(k);
    uint64_t* key = (uint64_t*)malloc(8 * W);
    if (!s || !t || !key) { free(s); free(t); free(key); return ORACLE_ENOMEM; }
    int status = ORACLE_OK;
    for (uint64_t r = r0; r < r1 && status == ORACLE_OK; r++) {
        const uint8_t* R = ascii + offsets[r];
        uint64_t L = offsets[r + 1] - offsets[r];
        for (uint64_t i = 0; i + k <= L; i++) {
            if (!window_ok(R + i, k)) continue;
            (*n_valid)++;
            for (uint32_t j = 0; j < k; j++) s[j] = upper(R[i + j]);
            const char* c = s;
            if (canonical) {
                reverse_complement(s, k, t);
                if (memcmp(t, s, k) < 0) c = t;
            }
            pack(c, k, key);
            uint64_t sh = oracle_shard_of(key, W, shard_mod);
            if (sh < s_lo || sh >= s_hi) continue;
            status = keys_push(&outs[sh - s_lo], key, W);
            if (status != ORACLE_OK) break;
        }
    }
    free(s); free(t); free(key);
    return status;
}

/*
 * Steps 6-9 of the definition over a multiset of n keys (sorted in place):
 * sort, run-length, the pairs with count >= threshold (App. A `-l`) in
 * ascending key order, and the histogram of the counts of every distinct key.
 */
int oracle_count_multiset(uint64_t* all, uint64_t n, uint32_t W, uint32_t threshold, oracle_result* out) {
    memset(out, 0, sizeof(*out));
    if (W < 1) return ORACLE_EINVAL;
    out->n_valid_shard = n;

    /* Step 6: sort the multiset, then run-length it. */
    if (n) qsort_r(all, n, 8 * W, cmp_keys, &W);   /* an empty shard may come with no array at all */
    uint64_t n_distinct = 0, max_count = 0;
    for (uint64_t i = 0; i < n;) {
        uint64_t j = i + 1;
        while (j < n && cmp_keys(all + i * W, all + j * W, &W) == 0) j++;
        n_distinct++;
        if (j - i > max_count) max_count = j - i;
        i = j;
    }
    /* Step 9: counters are 32-bit. */
    if (max_count >= 0xFFFFFFFFull) return ORACLE_ECOUNT;

    /* Steps 7-8: pairs with count >= threshold; histogram of all counts. */
    out->hist_len = max_count + 1;
    out->hist = (uint64_t*)calloc(out->hist_len, 8);
    uint64_t n_pairs = 0;
    for (uint64_t i = 0; i < n;) {
        uint64_t j = i + 1;
        while (j < n && cmp_keys(all + i * W, all + j * W, &W) == 0) j++;
        out->hist[j - i]++;
        if (j - i >= threshold) n_pairs++;
        i = j;
    }
    out->keys = (uint64_t*)malloc((n_pairs ? n_pairs : 1) * 8 * W);
    out->counts = (uint32_t*)malloc((n_pairs ? n_pairs : 1) * 4);
    if (!out->hist || !out->keys || !out->counts) { oracle_free(out); return ORACLE_ENOMEM; }
    uint64_t o = 0;
    for (uint64_t i = 0; i < n;) {
        uint64_t j = i + 1;
        while (j < n && cmp_keys(all + i * W, all + j * W, &W) == 0) j++;
        if (j - i >= threshold) {
            memcpy(out->keys + o * W, all + i * W, 8 * W);
            out->counts[o] = (uint32_t)(j - i);
            o++;
        }
        i = j;
    }
    out->n_distinct = n_distinct;
    out->n_pairs = n_pairs;
    out->max_count = max_count;
    return ORACLE_OK;
}

/*
 * Count canonical k-mers (canonical != 0) or plain k-mers (canonical == 0,
 * the paper's `-d`): steps 1-5 over every read, then steps 6-9. Keeps only
 * keys with oracle_shard_of(key) == shard_id when shard_mod > 1. Output pairs
 * are those with count >= threshold; the histogram covers every distinct key
 * of the shard.
 */
int oracle_count(const uint8_t* ascii, const uint64_t* offsets, uint64_t n_reads, uint32_t k,
                 uint32_t threshold, uint32_t canonical, uint64_t shard_mod, uint64_t shard_id,
                 oracle_result* out) {
    memset(out, 0, sizeof(*out));
    if (k < 1 || k > 1024) return ORACLE_EINVAL;
    if (shard_mod <= 1) shard_id = 0;
    oracle_keys keys = {NULL, 0, 0};
    uint64_t n_valid = 0;
    int status = oracle_collect(ascii, offsets, 0, n_reads, k, canonical, shard_mod, shard_id, shard_id + 1, &keys,
                                &n_valid);
    if (status == ORACLE_OK) status = oracle_count_multiset(keys.keys, keys.n, words_for(k), threshold, out);
    out->n_valid = n_valid;
    oracle_keys_free(&keys);
    return status;
}

/* Shard of each of n keys (oracle_shard_of), for splitting a large result the
 * way the oracle splits its work. */
void oracle_shard_of_many(const uint64_t* keys, uint64_t n, uint32_t W, uint64_t shard_mod, uint64_t* out) {
    for (uint64_t i = 0; i < n; i++) out[i] = oracle_shard_of(keys + i * W, W, shard_mod);
}

/*
 * Count how often each of the given canonical keys occurs in the input: one
 * pass over every window, each canonical window key looked up by binary
 * search in the sorted query list. Used to check sampled outputs of a large
 * run one by one.
 */
int oracle_count_keys(const uint8_t* ascii, const uint64_t* offsets, uint64_t n_reads, uint32_t k,
                      const uint64_t* query /* [n_query * W], sorted ascending */, uint64_t n_query,
                      uint64_t* counts /* [n_query] */) {
    if (k < 1 || k > 1024) return ORACLE_EINVAL;
    uint32_t W = words_for(k);
    char* s = (char*)malloc(k);
    char* t = (char*)malloc(k);
    uint64_t* key = (uint64_t*)malloc(8 * W);
    memset(counts, 0, n_query * 8);
    for (uint64_t r = 0; r < n_reads; r++) {
        const uint8_t* R = ascii + offsets[r];
        uint64_t L = offsets[r + 1] - offsets[r];
        for (uint64_t i = 0; i + k <= L; i++) {
            if (!window_ok(R + i, k)) continue;
            for (uint32_t j = 0; j < k; j++) s[j] = upper(R[i + j]);
            reverse_complement(s, k, t);
            pack(memcmp(t, s, k) < 0 ? t : s, k, key);
            uint64_t lo = 0, hi = n_query;
            while (lo < hi) {
                uint64_t mid = (lo + hi) / 2;
                int c = cmp_keys(query + mid * W, key, &W);
                if (c == 0) { counts[mid]++; break; }
                if (c < 0) lo = mid + 1; else hi = mid;
            }
        }
    }
    free(s); free(t); free(key);
    return ORACLE_OK;
}

/* The same counts over reads [r0, r1) only, for queries against very large
 * read sets (callers split the reads between threads and add the results).
 * A window is canonicalised only when the first f = min(16, k) bases of its
 * forward strand or of its reverse complement begin some query key: the
 * canonical form is one of the two strands, so no window that matches a
 * query is skipped. Windows are tested for undetermined bases with the end
 * of the run of valid bases they start in (Sec. 2.4.1). */
static int cmp_u32(const void* a, const void* b) {
    uint32_t x = *(const uint32_t*)a, y = *(const uint32_t*)b;
    return x < y ? -1 : x > y;
}

static int has_u32(const uint32_t* v, uint64_t n, uint32_t x) {
    uint64_t lo = 0, hi = n;
    while (lo < hi) {
        uint64_t mid = (lo + hi) / 2;
        if (v[mid] == x) return 1;
        if (v[mid] < x) lo = mid + 1; else hi = mid;
    }
    return 0;
}

int oracle_count_keys_range(const uint8_t* ascii, const uint64_t* offsets, uint64_t r0, uint64_t r1, uint32_t k,
                            const uint64_t* query /* [n_query * W], sorted ascending */, uint64_t n_query,
                            uint64_t* counts /* [n_query], added to */) {
    if (k < 1 || k > 1024) return ORACLE_EINVAL;
    uint32_t W = words_for(k);
    uint32_t f = k < 16 ? k : 16;
    uint32_t r_last = k - 32 * (W - 1);
    /* prefix code of every query key: its first f bases, 2 bits each */
    uint32_t* pre = (uint32_t*)malloc(4 * (n_query ? n_query : 1));
    for (uint64_t q = 0; q < n_query; q++) {
        const uint64_t* key = query + q * W;
        uint32_t c = 0;
        for (uint32_t j = 0; j < f; j++) {
            uint32_t wi = j / 32, bi = j % 32;
            uint32_t bases_in_word = (wi == W - 1) ? r_last : 32;
            c = (c << 2) | (uint32_t)((key[wi] >> (2 * (bases_in_word - 1 - bi))) & 3);
        }
        pre[q] = c;
    }
    qsort(pre, n_query, 4, cmp_u32);
    char* s = (char*)malloc(k);
    char* t = (char*)malloc(k);
    uint64_t* key = (uint64_t*)malloc(8 * W);
    for (uint64_t r = r0; r < r1; r++) {
        const uint8_t* R = ascii + offsets[r];
        uint64_t L = offsets[r + 1] - offsets[r];
        uint64_t run_end = 0;   /* first invalid position at or after i */
        for (uint64_t i = 0; i + k <= L; i++) {
            if (run_end <= i) {
                run_end = i;
                while (run_end < L && base_ok(R[run_end])) run_end++;
            }
            if (run_end < i + k) continue;   /* the window holds an undetermined base */
            uint32_t cf = 0, cr = 0;
            for (uint32_t j = 0; j < f; j++) {
                cf = (cf << 2) | (uint32_t)code2(upper(R[i + j]));
                cr = (cr << 2) | (uint32_t)code2(complement(upper(R[i + k - 1 - j])));
            }
            if (!has_u32(pre, n_query, cf) && !has_u32(pre, n_query, cr)) continue;
            for (uint32_t j = 0; j < k; j++) s[j] = upper(R[i + j]);
            reverse_complement(s, k, t);
            pack(memcmp(t, s, k) < 0 ? t : s, k, key);
            uint64_t lo = 0, hi = n_query;
            while (lo < hi) {
                uint64_t mid = (lo + hi) / 2;
                int c = cmp_keys(query + mid * W, key, &W);
                if (c == 0) { counts[mid]++; break; }
                if (c < 0) lo = mid + 1; else hi = mid;
            }
        }
    }
    free(s); free(t); free(key); free(pre);
    return ORACLE_OK;
}

/* ------------------------------------------------------------- encoding -- */

/*
 * 2-bit packing of the whole byte stream (byte i -> word i/32, bits
 * 63-2(i%32) .. 62-2(i%32)); bytes that are not A/C/G/T are stored as code 0.
 * kmer_ok bit p (word p/64, bit p%64) is set iff the window [p, p+k) lies
 * inside one read and holds only valid bases. Returns the number of set bits
 * in *n_valid.
 */
int oracle_encode(const uint8_t* ascii, const uint64_t* offsets, uint64_t n_reads, uint32_t k,
                  uint64_t* packed /* [ceil(n_bytes/32)] */, uint64_t* kmer_ok /* [ceil(n_bytes/64)] */,
                  uint64_t* n_valid) {
    if (k < 1) return ORACLE_EINVAL;
    uint64_t n_bytes = offsets[n_reads];
    memset(packed, 0, ((n_bytes + 31) / 32) * 8);
    memset(kmer_ok, 0, ((n_bytes + 63) / 64) * 8);
    for (uint64_t i = 0; i < n_bytes; i++) {
        uint64_t c = base_ok(ascii[i]) ? code2(upper(ascii[i])) : 0;
        packed[i / 32] |= c << (62 - 2 * (i % 32));
    }
    uint64_t nv = 0;
    for (uint64_t r = 0; r < n_reads; r++) {
        uint64_t L = offsets[r + 1] - offsets[r];
        for (uint64_t i = 0; i + k <= L; i++) {
            uint64_t p = offsets[r] + i;
            if (window_ok(ascii + p, k)) {
                kmer_ok[p / 64] |= 1ull << (p % 64);
                nv++;
            }
        }
    }
    *n_valid = nv;
    return ORACLE_OK;
}

/* ----------------------------------------------------------- minimizers -- */

/* Rank of an m-mer string u under the chosen total order, using its
 * canonical form. order 0: KMC2-style (codes of canonical m-mers starting with
 * AAA or ACA are moved behind all others); order 1: plain lexicographic;
 * order 2: table[canonical code] (any order of Sec. 3.1 given as a table).
 * The canonical code is returned in *code. */
static const uint32_t* g_rank_table = NULL;
static uint64_t mmer_rank(const char* u, uint32_t m, uint32_t order, uint64_t* code) {
    char v[64], c[64];
    reverse_complement(u, m, v);
    memcpy(c, memcmp(v, u, m) < 0 ? v : u, m);
    uint64_t x = 0;
    for (uint32_t j = 0; j < m; j++) x = (x << 2) | code2(c[j]);
    *code = x;
    if (order == 2) return g_rank_table[x];
    if (order == 0 && m >= 3 && (memcmp(c, "AAA", 3) == 0 || memcmp(c, "ACA", 3) == 0))
        return x + (1ull << (2 * m));
    return x;
}

/* Minimizer rank of the k-mer s (uppercase, valid): the smallest rank over
 * its k-m+1 m-mers. */
static uint64_t minimizer_rank(const char* s, uint32_t k, uint32_t m, uint32_t order, uint64_t* code) {
    uint64_t best = ~0ull, best_code = 0;
    for (uint32_t j = 0; j + m <= k; j++) {
        uint64_t c;
        uint64_t r = mmer_rank(s + j, m, order, &c);
        if (r < best) { best = r; best_code = c; }
    }
    *code = best_code;
    return best;
}

/*
 * Super-mers of every read: maximal runs of consecutive valid windows whose
 * minimizers are equal. Each is reported as (global byte position of its
 * first base, number of k-mers, bin, minimizer rank).
 */
int oracle_supermers(const uint8_t* ascii, const uint64_t* offsets, uint64_t n_reads, uint32_t k, uint32_t m,
                     uint32_t order, uint32_t n_bins, const uint32_t* bin_map /* [4^m] or NULL */,
                     const uint32_t* rank_table /* [4^m], order 2 */, uint64_t* start, uint32_t* n_kmers,
                     uint32_t* bin, uint64_t* rank, uint64_t cap, uint64_t* n_out) {
    if (m < 1 || m > 15 || m >= k || n_bins < 1 || order > 2 || (order == 2 && !rank_table)) return ORACLE_EINVAL;
    g_rank_table = rank_table;
    char* s = (char*)malloc(k);
    uint64_t n = 0;
    int status = ORACLE_OK;
    for (uint64_t r = 0; r < n_reads; r++) {
        const uint8_t* R = ascii + offsets[r];
        uint64_t L = offsets[r + 1] - offsets[r];
        int open = 0;
        uint64_t cur = 0;
        for (uint64_t i = 0; i + k <= L; i++) {
            if (!window_ok(R + i, k)) { open = 0; continue; }
            for (uint32_t j = 0; j < k; j++) s[j] = upper(R[i + j]);
            uint64_t code;
            uint64_t mr = minimizer_rank(s, k, m, order, &code);
            if (open && mr == cur) {
                n_kmers[n - 1]++;
                continue;
            }
            if (n == cap) { status = ORACLE_ECAP; open = 0; continue; }
            start[n] = offsets[r] + i;
            n_kmers[n] = 1;
            bin[n] = bin_map ? bin_map[code] : (uint32_t)(mr % n_bins);
            rank[n] = mr;
            n++;
            open = 1;
            cur = mr;
        }
    }
    *n_out = n;
    free(s);
    return status;
}

/* ---------------------------------------------------------- output codec -- */

/*
 * One output record of App. C: the counter in one byte if it is below 255,
 * otherwise 0xFF followed by the counter as a big-endian 32-bit integer; then
 * the k-mer string, four bases per byte, first base in the two most
 * significant bits, unused low bits of the last byte set to zero. Returns the
 * record length in bytes.
 */
uint32_t oracle_record(const char* kmer, uint32_t k, uint32_t count, uint8_t* out) {
    uint32_t o = 0;
    if (count < 255) {
        out[o++] = (uint8_t)count;
    } else {
        out[o++] = 0xFF;
        out[o++] = (uint8_t)(count >> 24);
        out[o++] = (uint8_t)(count >> 16);
        out[o++] = (uint8_t)(count >> 8);
        out[o++] = (uint8_t)count;
    }
    for (uint32_t j = 0; j < k; j += 4) {
        uint8_t byte = 0;
        for (uint32_t q = 0; q < 4; q++) {
            uint64_t c = (j + q < k) ? code2(upper((uint8_t)kmer[j + q])) : 0;
            byte |= (uint8_t)(c << (6 - 2 * q));
        }
        out[o++] = byte;
    }
    return o;
}

/*
 * Test driver: runs the C oracle and the C read generator on small seeded
 * inputs under AddressSanitizer and UndefinedBehaviorSanitizer (built and run
 * by tests/test_sanitizers.py with gcc; host code only, no GPU). Exits 0 when
 * every call succeeds and the counts are consistent; any out-of-bounds
 * access, leak or undefined behaviour aborts the run.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    uint64_t n_valid, n_valid_shard, n_distinct, n_pairs;
    uint64_t* keys;
    uint32_t* counts;
    uint64_t* hist;
    uint64_t hist_len, max_count;
} oracle_result;
typedef struct {
    uint64_t* keys;
    uint64_t n, cap;
} oracle_keys;

int synth_genome(uint64_t G, double gc, double rep_frac, double rep_div, uint64_t seed, uint8_t* out);
uint64_t synth_read_offsets(uint64_t n, double median, double sigma, uint64_t len_min, uint64_t len_max,
                            uint64_t seed, uint64_t* offsets);
int synth_reads(const uint8_t* genome, uint64_t G, const uint64_t* offsets, uint64_t n, double err, double p_n,
                uint64_t seed, int threads, uint8_t* out);
int oracle_count(const uint8_t* ascii, const uint64_t* offsets, uint64_t n_reads, uint32_t k, uint32_t threshold,
                 uint32_t canonical, uint64_t shard_mod, uint64_t shard_id, oracle_result* out);
void oracle_free(oracle_result* r);
int oracle_collect(const uint8_t* ascii, const uint64_t* offsets, uint64_t r0, uint64_t r1, uint32_t k,
                   uint32_t canonical, uint64_t shard_mod, uint64_t s_lo, uint64_t s_hi, oracle_keys* outs,
                   uint64_t* n_valid);
int oracle_count_multiset(uint64_t* all, uint64_t n, uint32_t W, uint32_t threshold, oracle_result* out);
void oracle_keys_free(oracle_keys* a);
int oracle_count_keys(const uint8_t* ascii, const uint64_t* offsets, uint64_t n_reads, uint32_t k,
                      const uint64_t* query, uint64_t n_query, uint64_t* counts);
int oracle_count_keys_range(const uint8_t* ascii, const uint64_t* offsets, uint64_t r0, uint64_t r1, uint32_t k,
                            const uint64_t* query, uint64_t n_query, uint64_t* counts);
int oracle_encode(const uint8_t* ascii, const uint64_t* offsets, uint64_t n_reads, uint32_t k, uint64_t* packed,
                  uint64_t* kmer_ok, uint64_t* n_valid);
int oracle_supermers(const uint8_t* ascii, const uint64_t* offsets, uint64_t n_reads, uint32_t k, uint32_t m,
                     uint32_t order, uint32_t n_bins, const uint32_t* bin_map, const uint32_t* rank_table,
                     uint64_t* start, uint32_t* n_kmers, uint32_t* bin, uint64_t* rank, uint64_t cap,
                     uint64_t* n_out);
uint32_t oracle_record(const char* kmer, uint32_t k, uint32_t count, uint8_t* out);

#define CHECK(c)                                                         \
    do {                                                                 \
        if (!(c)) {                                                      \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            return 1;                                                    \
        }                                                                \
    } while (0)

int main(void) {
    const uint64_t G = 30000, n = 400;
    uint8_t* genome = malloc(G);
    uint64_t* offsets = malloc(8 * (n + 1));
    CHECK(synth_genome(G, 0.41, 0.05, 0.02, 7, genome) == 0);
    const uint64_t bytes = synth_read_offsets(n, 150, 0.5, 20, 600, 7, offsets);
    CHECK(bytes == offsets[n]);
    uint8_t* ascii = malloc(bytes);
    CHECK(synth_reads(genome, G, offsets, n, 0.01, 0.01, 7, 2, ascii) == 0);
    ascii[3] = 'n';   /* lower case and an undetermined base */
    ascii[5] = 'a';

    const uint32_t ks[] = {1, 15, 31, 32, 33, 64, 65, 99, 200, 479};
    for (unsigned t = 0; t < sizeof(ks) / sizeof(ks[0]); t++) {
        const uint32_t k = ks[t], W = (k + 31) / 32;
        for (uint32_t canon = 0; canon < 2; canon++) {
            oracle_result r;
            CHECK(oracle_count(ascii, offsets, n, k, 2, canon, 1, 0, &r) == 0);
            uint64_t sum = 0;
            for (uint64_t c = 1; c < r.hist_len; c++) sum += c * r.hist[c];
            CHECK(sum == r.n_valid);
            /* the same count from the collecting and counting steps, in three shards */
            uint64_t pairs = 0;
            for (uint64_t s = 0; s < 3; s++) {
                oracle_keys keys = {NULL, 0, 0};
                uint64_t nv = 0;
                CHECK(oracle_collect(ascii, offsets, 0, n, k, canon, 3, s, s + 1, &keys, &nv) == 0);
                CHECK(nv == r.n_valid);
                oracle_result q;
                CHECK(oracle_count_multiset(keys.keys, keys.n, W, 2, &q) == 0);
                pairs += q.n_pairs;
                oracle_free(&q);
                oracle_keys_free(&keys);
            }
            CHECK(pairs == r.n_pairs);
            if (canon && r.n_pairs) {
                uint64_t* got = calloc(r.n_pairs, 8);
                uint64_t* got2 = calloc(r.n_pairs, 8);
                CHECK(oracle_count_keys(ascii, offsets, n, k, r.keys, r.n_pairs, got) == 0);
                CHECK(oracle_count_keys_range(ascii, offsets, 0, n / 2, k, r.keys, r.n_pairs, got2) == 0);
                CHECK(oracle_count_keys_range(ascii, offsets, n / 2, n, k, r.keys, r.n_pairs, got2) == 0);
                for (uint64_t i = 0; i < r.n_pairs; i++) CHECK(got[i] == r.counts[i] && got2[i] == r.counts[i]);
                free(got);
                free(got2);
            }
            oracle_free(&r);
        }
        const uint64_t nw = (bytes + 31) / 32 + 1, nm = (bytes + 63) / 64 + 1;
        uint64_t* packed = calloc(nw, 8);
        uint64_t* ok = calloc(nm, 8);
        uint64_t nv = 0;
        CHECK(oracle_encode(ascii, offsets, n, k, packed, ok, &nv) == 0);
        free(packed);
        free(ok);
        if (k > 7) {
            const uint64_t cap = bytes;
            uint64_t* start = malloc(8 * cap);
            uint32_t* nk = malloc(4 * cap);
            uint32_t* bin = malloc(4 * cap);
            uint64_t* rank = malloc(8 * cap);
            for (uint32_t order = 0; order < 2; order++) {
                uint64_t ns = 0, total = 0;
                CHECK(oracle_supermers(ascii, offsets, n, k, 7, order, 64, NULL, NULL, start, nk, bin, rank, cap,
                                       &ns) == 0);
                for (uint64_t i = 0; i < ns; i++) total += nk[i];
                CHECK(total == nv);
            }
            free(start);
            free(nk);
            free(bin);
            free(rank);
        }
    }
    uint8_t rec[8];
    CHECK(oracle_record("AACGTG", 6, 67, rec) == 3);
    CHECK(oracle_record("TGGATC", 6, 345, rec) == 7);
    free(ascii);
    free(offsets);
    free(genome);
    printf("sanitized oracle and generator runs: ok\n");
    return 0;
}

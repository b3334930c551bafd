/*
 * Seeded synthetic genomes and sequencing reads.
 *
 * This module only draws random DNA: it holds none of the counting method's
 * arithmetic (no 2-bit code, no k-mers, no minimizers, no hashing of keys).
 * Both the CPU oracle and the GPU path read its output, so it must stay free
 * of anything either of them computes.
 *
 * Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014) used as a counter-based
 * generator: every draw is splitmix64(key(seed, stream) + index), so a value
 * depends only on (seed, stream, index) and the output is identical for any
 * thread count.
 *
 * Workload model (the paper measures on real read sets that are not
 * available; these stand in for them):
 *   genome  : i.i.d. bases with P(G) = P(C) = gc/2, plus repeat copies: a
 *             uniform source segment of length U[300, 5000] is copied in
 *             forward orientation with per-base substitution probability
 *             `rep_div` and inserted at a uniform position, until a fraction
 *             `rep_frac` of the genome length is inserted.
 *   reads   : start uniform in [0, G - L]; strand chosen with p = 1/2 (the
 *             read is reverse-complemented); each base substituted with
 *             probability `err` by one of the three other bases; then each
 *             base replaced by 'N' with probability `p_n`.
 *   lengths : fixed, or log-normal with a given median and sigma, resampled
 *             until inside [len_min, len_max].
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static inline uint64_t sm64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Stream identifiers: each kind of draw has its own counter space. */
enum {
    ST_GENOME = 1, ST_REP_LEN, ST_REP_SRC, ST_REP_POS, ST_REP_MUT,
    ST_READ_LEN, ST_READ_POS, ST_READ_STRAND, ST_READ_ERR, ST_READ_N
};

static inline uint64_t stream_key(uint64_t seed, uint64_t stream) {
    return sm64(sm64(seed) ^ (stream * 0xD1B54A32D192ED03ull));
}
static inline uint64_t draw(uint64_t key, uint64_t idx) { return sm64(key + idx * 0x9E3779B97F4A7C15ull); }
static inline double unit(uint64_t r) { return (double)(r >> 11) * (1.0 / 9007199254740992.0); }
/* Uniform integer in [0, n) by 128-bit multiply (Lemire's range reduction). */
static inline uint64_t below(uint64_t r, uint64_t n) { return (uint64_t)(((__uint128_t)r * n) >> 64); }

static const char ACGT[4] = {'A', 'C', 'G', 'T'};

static inline char random_base(double u, double gc) {
    double a = (1.0 - gc) * 0.5, c = gc * 0.5;
    if (u < a) return 'A';
    if (u < a + c) return 'C';
    if (u < a + 2 * c) return 'G';
    return 'T';
}

static inline char substitute(char b, uint64_t r) {
    /* one of the three other bases, uniformly */
    int idx = b == 'A' ? 0 : b == 'C' ? 1 : b == 'G' ? 2 : 3;
    int alt = (int)below(r, 3);
    return ACGT[(idx + 1 + alt) & 3];
}

static inline char complement(char b) {
    switch (b) {
        case 'A': return 'T';
        case 'C': return 'G';
        case 'G': return 'C';
        case 'T': return 'A';
        default: return b;
    }
}

typedef struct { uint64_t pos; uint64_t src; uint64_t len; uint64_t id; } repeat_t;

static int cmp_repeat(const void* a, const void* b) {
    const repeat_t* x = (const repeat_t*)a;
    const repeat_t* y = (const repeat_t*)b;
    if (x->pos != y->pos) return x->pos < y->pos ? -1 : 1;
    return x->id < y->id ? -1 : (x->id > y->id);
}

/* Number of repeat copies the genome model inserts for (G, rep_frac, seed). */
static uint64_t repeat_plan(uint64_t G, double rep_frac, uint64_t seed, repeat_t** out, uint64_t* total) {
    uint64_t target = (uint64_t)(rep_frac * (double)G);
    uint64_t klen = stream_key(seed, ST_REP_LEN);
    uint64_t cap = 16, n = 0, sum = 0;
    repeat_t* r = (repeat_t*)malloc(cap * sizeof(repeat_t));
    while (sum < target) {
        uint64_t len = 300 + below(draw(klen, n), 4701);
        if (sum + len > target) len = target - sum;
        if (n == cap) { cap *= 2; r = (repeat_t*)realloc(r, cap * sizeof(repeat_t)); }
        r[n].len = len; r[n].id = n;
        sum += len; n++;
    }
    *out = r; *total = sum;
    return n;
}

/*
 * synth_genome: write an uppercase ACGT genome of exactly G bases to `out`.
 * Returns 0 on success, -1 on bad arguments.
 */
int synth_genome(uint64_t G, double gc, double rep_frac, double rep_div, uint64_t seed, uint8_t* out) {
    if (G < 10000 || gc < 0 || gc > 1 || rep_frac < 0 || rep_frac >= 0.5) return -1;
    repeat_t* reps = NULL; uint64_t rep_total = 0;
    uint64_t n_rep = repeat_plan(G, rep_frac, seed, &reps, &rep_total);
    uint64_t B = G - rep_total;                     /* backbone length */
    uint8_t* bb = (uint8_t*)malloc(B);
    uint64_t kg = stream_key(seed, ST_GENOME);
    for (uint64_t i = 0; i < B; i++) bb[i] = (uint8_t)random_base(unit(draw(kg, i)), gc);
    uint64_t ksrc = stream_key(seed, ST_REP_SRC), kpos = stream_key(seed, ST_REP_POS);
    for (uint64_t j = 0; j < n_rep; j++) {
        reps[j].src = below(draw(ksrc, j), B - reps[j].len + 1);
        reps[j].pos = below(draw(kpos, j), B + 1);
    }
    qsort(reps, n_rep, sizeof(repeat_t), cmp_repeat);
    uint64_t kmut = stream_key(seed, ST_REP_MUT);
    uint64_t o = 0, prev = 0;
    for (uint64_t j = 0; j < n_rep; j++) {
        memcpy(out + o, bb + prev, reps[j].pos - prev); o += reps[j].pos - prev; prev = reps[j].pos;
        for (uint64_t t = 0; t < reps[j].len; t++) {
            char b = (char)bb[reps[j].src + t];
            uint64_t idx = (reps[j].id << 16) ^ t;  /* copies are < 2^16 bases long */
            if (unit(draw(kmut, 2 * idx)) < rep_div) b = substitute(b, draw(kmut, 2 * idx + 1));
            out[o++] = (uint8_t)b;
        }
    }
    memcpy(out + o, bb + prev, B - prev); o += B - prev;
    free(bb); free(reps);
    return o == G ? 0 : -1;
}

/*
 * synth_read_lengths: lengths of n reads. If sigma <= 0 every read has length
 * `median`; otherwise LogNormal(ln(median), sigma) rounded, resampled until in
 * [len_min, len_max]. Writes offsets[0..n] (CSR, offsets[0] = 0) and returns
 * the total number of bytes.
 */
uint64_t synth_read_offsets(uint64_t n, double median, double sigma, uint64_t len_min, uint64_t len_max,
                            uint64_t seed, uint64_t* offsets) {
    uint64_t kl = stream_key(seed, ST_READ_LEN);
    offsets[0] = 0;
    for (uint64_t r = 0; r < n; r++) {
        uint64_t L;
        if (sigma <= 0) {
            L = (uint64_t)median;
        } else {
            for (uint64_t a = 0;; a++) {
                uint64_t idx = (r << 8) | (a & 0xFF);
                double u1 = unit(draw(kl, 2 * idx)), u2 = unit(draw(kl, 2 * idx + 1));
                if (u1 < 1e-300) u1 = 1e-300;
                double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);  /* Box-Muller */
                double x = floor(exp(log(median) + sigma * z) + 0.5);
                if (x >= (double)len_min && x <= (double)len_max) { L = (uint64_t)x; break; }
                if (a == 255) { L = (uint64_t)median; break; }
            }
        }
        offsets[r + 1] = offsets[r] + L;
    }
    return offsets[n];
}

typedef struct {
    const uint8_t* genome; uint64_t G;
    const uint64_t* offsets; uint64_t r0, r1;
    double err, p_n; uint64_t seed; uint8_t* out;
} read_job;

static void* read_worker(void* arg) {
    read_job* j = (read_job*)arg;
    uint64_t kp = stream_key(j->seed, ST_READ_POS), ks = stream_key(j->seed, ST_READ_STRAND);
    uint64_t ke = stream_key(j->seed, ST_READ_ERR), kn = stream_key(j->seed, ST_READ_N);
    for (uint64_t r = j->r0; r < j->r1; r++) {
        uint64_t o = j->offsets[r], L = j->offsets[r + 1] - o;
        if (L > j->G) L = j->G;
        uint64_t start = below(draw(kp, r), j->G - L + 1);
        int rev = (int)(draw(ks, r) >> 63);
        uint8_t* d = j->out + o;
        for (uint64_t t = 0; t < L; t++) {
            char b = rev ? complement((char)j->genome[start + L - 1 - t]) : (char)j->genome[start + t];
            uint64_t idx = o + t;  /* global byte index: unique per base */
            if (j->err > 0 && unit(draw(ke, 2 * idx)) < j->err) b = substitute(b, draw(ke, 2 * idx + 1));
            if (j->p_n > 0 && unit(draw(kn, idx)) < j->p_n) b = 'N';
            d[t] = (uint8_t)b;
        }
    }
    return NULL;
}

/*
 * synth_reads: fill out[offsets[0]..offsets[n]) with n reads sampled from the
 * genome (see the model above), using `threads` POSIX threads.
 */
int synth_reads(const uint8_t* genome, uint64_t G, const uint64_t* offsets, uint64_t n, double err, double p_n,
                uint64_t seed, int threads, uint8_t* out) {
    if (threads < 1) threads = 1;
    if (threads > 256) threads = 256;
    pthread_t th[256];
    read_job jobs[256];
    for (int t = 0; t < threads; t++) {
        jobs[t].genome = genome; jobs[t].G = G; jobs[t].offsets = offsets;
        jobs[t].r0 = n * (uint64_t)t / (uint64_t)threads;
        jobs[t].r1 = n * (uint64_t)(t + 1) / (uint64_t)threads;
        jobs[t].err = err; jobs[t].p_n = p_n; jobs[t].seed = seed; jobs[t].out = out;
    }
    for (int t = 1; t < threads; t++) pthread_create(&th[t], NULL, read_worker, &jobs[t]);
    read_worker(&jobs[0]);
    for (int t = 1; t < threads; t++) pthread_join(th[t], NULL);
    return 0;
}

/* Uniform double in [0,1) for the Python side (job parameters, Poisson arrivals). */
double synth_unit(uint64_t seed, uint64_t stream, uint64_t idx) {
    return unit(draw(stream_key(seed, stream), idx));
}

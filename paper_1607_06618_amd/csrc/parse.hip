// FASTA / FASTQ text to CSR reads, on the device (the input formats of
// App. B; the paper's parser stage feeds the counting pipeline, Sec. 2.3.1).
//
// The text is cut into lines by a newline compaction; every later step works
// on lines, never on the text again, except for the copy of the sequence
// bytes:
//   1. newlines per byte tile (64 KB: sixteen rounds of 4 KB, 16 B per lane);
//   2. one workgroup scans the tile counts (line count, final line);
//   3. each newline writes a line word: its position (40 bits), whether the
//      byte before it is '\r' (bit 40), and the first byte of the next line
//      (bits 48-55);
//   4. per line tile: sequence bytes kept and reads started, from the format
//      (FASTQ: line index mod 4; FASTA: a '>' first byte), plus the format
//      checks;
//   5. one workgroup scans the tile sums;
//   6. per line: the offset of its kept bytes, and the read offsets;
//   7. per line tile, the kept bytes are gathered into aligned 16-byte
//      chunks of the output.
#include "../../include/gerbil.h"
#include "common.h"
#include "internal.h"

namespace gerbil {
namespace {

constexpr uint32_t kPB = 256;                        // threads of the tile kernels
constexpr uint32_t kChunk = 16;                      // text bytes per lane and round
constexpr uint32_t kRounds = 16;                     // a multiple of 4: four rounds share one scan
constexpr uint64_t kByteTile = (uint64_t)kPB * kChunk * kRounds;   // 64 KB
constexpr uint32_t kLinesPer = 8;                    // lines per lane
constexpr uint64_t kLineTile = (uint64_t)kPB * kLinesPer;          // 2048 lines
constexpr uint32_t kScanBlock = 1024;                // threads of the one-workgroup scans
constexpr uint64_t kPosMask = (1ull << 40) - 1;

constexpr uint32_t kMaxTileGridParse = 8192;

struct Ws {
    uint64_t* tile_nl;     // [n_btiles + 1]
    uint64_t* line;        // [lines_cap] line words
    uint64_t* line_off;    // [lines_cap]
    uint64_t* lt_kept;     // [n_ltiles + 1]
    uint64_t* lt_reads;    // [n_ltiles + 1]
};

__host__ __device__ inline uint64_t n_btiles_of(uint64_t n) { return (n + kByteTile - 1) / kByteTile; }
__host__ __device__ inline uint64_t n_ltiles_of(uint64_t lines) { return (lines + kLineTile - 1) / kLineTile; }

inline uint64_t ws_layout(uint64_t n, uint64_t lines_cap, uint8_t* base, Ws* w) {
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) {
        uint8_t* p = base ? base + off : nullptr;
        off += align256(bytes);
        return (uint64_t*)p;
    };
    Ws x;
    x.tile_nl = take(8 * (n_btiles_of(n) + 1));
    x.line = take(8 * (lines_cap + 1));
    x.line_off = take(8 * (lines_cap + 1));
    x.lt_kept = take(8 * (n_ltiles_of(lines_cap) + 1));
    x.lt_reads = take(8 * (n_ltiles_of(lines_cap) + 1));
    if (w) *w = x;
    return off;
}

// 0x80 in every byte of x that equals 0x0A, else 0 (exact, no carries).
__device__ __forceinline__ uint32_t nl_bytes(uint32_t x) {
    const uint32_t y = x ^ 0x0A0A0A0Au;
    return ~(((y & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | y | 0x7F7F7F7Fu);
}

// The 16 bytes of chunk c (c * 16 .. c * 16 + 15 of the text) as four words;
// bytes outside [0, n) read as 0. Whole chunks use one 16-byte load when the
// text is 16-byte aligned, else byte loads.
__device__ __forceinline__ void load_chunk(const uint8_t* __restrict__ text, uint64_t n, uint64_t c, bool aligned,
                                           uint32_t (&w)[4]) {
    const uint64_t b = c * kChunk;
    if (aligned && b + kChunk <= n) {
        const uint4 v = *(const uint4*)(text + b);
        w[0] = v.x; w[1] = v.y; w[2] = v.z; w[3] = v.w;
        return;
    }
#pragma unroll
    for (int i = 0; i < 4; i++) {
        uint32_t x = 0;
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const uint64_t p = b + 4 * i + j;
            x |= (uint32_t)(p < n ? text[p] : 0u) << (8 * j);
        }
        w[i] = x;
    }
}

__device__ __forceinline__ uint32_t chunk_newlines(const uint32_t (&w)[4]) {
    uint32_t c = 0;
#pragma unroll
    for (int i = 0; i < 4; i++) c += __builtin_popcount(nl_bytes(w[i]));
    return c;
}

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
    const uint32_t lane = __lane_id();
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const T y = __shfl_up(v, off);
        if (lane >= (uint32_t)off) v += y;
    }
    return v;
}

// Exclusive scan of one uint64 per thread over the block; wsum holds
// blockDim/64 + 1 entries.
__device__ __forceinline__ uint64_t block_scan64(uint64_t v, uint64_t* wsum, uint64_t& total) {
    const uint32_t lane = __lane_id(), wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const uint64_t incl = wave_incl_scan<uint64_t>(v);
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    if (wave == 0) {
        const uint64_t s = lane < nw ? wsum[lane] : 0ull;
        const uint64_t si = wave_incl_scan<uint64_t>(s);
        if (lane < nw) wsum[lane] = si - s;
        if (lane == 63) wsum[nw] = si;
    }
    __syncthreads();
    const uint64_t r = wsum[wave] + incl - v;
    total = wsum[nw];
    __syncthreads();   // wsum is reused by the next call
    return r;
}

// In-place exclusive scan of v[0..n) by one workgroup of kScanBlock threads;
// returns the total to every thread.
__device__ uint64_t wg_scan_inplace(uint64_t* v, uint64_t n, uint64_t* wsum) {
    const uint32_t tid = threadIdx.x;
    const uint64_t per = (n + kScanBlock - 1) / kScanBlock;
    const uint64_t lo = tid * per, hi = lo + per < n ? lo + per : n;
    uint64_t s = 0;
    for (uint64_t i = lo; i < hi; i++) s += v[i];
    uint64_t total;
    uint64_t run = block_scan64(s, wsum, total);
    for (uint64_t i = lo; i < hi; i++) {
        const uint64_t x = v[i];
        v[i] = run;
        run += x;
    }
    return total;
}

// --------------------------------------------------------------- kernels

__global__ void k_parse_init(const uint8_t* __restrict__ text, uint64_t n, uint32_t format, gerbil_parsed* out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    uint32_t fmt = format, status = 0;
    if (fmt == GERBIL_FORMAT_DETECT && n) {
        const uint8_t c = text[0];
        fmt = c == '@' ? GERBIL_FORMAT_FASTQ : c == '>' ? GERBIL_FORMAT_FASTA : 0u;
        if (!fmt) status = GERBIL_PARSE_EFORMAT;
    }
    out->n_reads = 0;
    out->n_bytes = 0;
    out->n_lines = 0;
    out->status = status;
    out->format = fmt;
}

// 1. newlines per byte tile
__global__ void __launch_bounds__(kPB) k_nl_count(const uint8_t* __restrict__ text, uint64_t n, bool aligned,
                                                  uint64_t* __restrict__ tile_nl) {
    __shared__ uint64_t wsum[kPB / 64 + 1];
    const uint64_t nt = n_btiles_of(n);
    for (uint64_t t = blockIdx.x; t < nt; t += gridDim.x) {
        uint32_t c = 0;
#pragma unroll
        for (uint32_t r = 0; r < kRounds; r++) {
            uint32_t w[4];
            load_chunk(text, n, (t * kRounds + r) * kPB + threadIdx.x, aligned, w);
            c += chunk_newlines(w);
        }
        uint64_t total;
        (void)block_scan64(c, wsum, total);
        if (threadIdx.x == 0) tile_nl[t] = total;
    }
}

// 2. scan of the tile counts; the final line without a newline
__global__ void __launch_bounds__(kScanBlock) k_nl_scan(const uint8_t* __restrict__ text, uint64_t n,
                                                        uint64_t* __restrict__ tile_nl, uint64_t* __restrict__ line,
                                                        uint64_t lines_cap, gerbil_parsed* out) {
    __shared__ uint64_t wsum[kScanBlock / 64 + 1];
    const uint64_t nt = n_btiles_of(n);
    const uint64_t nl = wg_scan_inplace(tile_nl, nt, wsum);
    if (threadIdx.x != 0) return;
    const bool open_end = n > 0 && text[n - 1] != '\n';
    const uint64_t lines = nl + (open_end ? 1 : 0);
    out->n_lines = lines;
    if (lines > lines_cap) {
        out->status |= GERBIL_PARSE_ELINECAP;
        return;
    }
    if (open_end) line[nl] = n | ((uint64_t)(text[n - 1] == '\r') << 40);   // no next line: first byte 0
}

// 3. the line words. Four rounds share one block scan: their newline counts
// (at most 16 per lane and round, at most 4096 per round) ride in 16-bit
// fields of one 64-bit value.
__device__ __forceinline__ uint32_t chunk_byte(const uint32_t (&w)[4], uint32_t idx) {
    const uint32_t x = idx < 4 ? w[0] : idx < 8 ? w[1] : idx < 12 ? w[2] : w[3];
    return (x >> (8 * (idx & 3))) & 0xFFu;
}

__global__ void __launch_bounds__(kPB) k_nl_write(const uint8_t* __restrict__ text, uint64_t n, bool aligned,
                                                  const uint64_t* __restrict__ tile_nl, uint64_t* __restrict__ line,
                                                  uint64_t lines_cap) {
    __shared__ uint64_t wsum[kPB / 64 + 1];
    const uint64_t nt = n_btiles_of(n);
    for (uint64_t t = blockIdx.x; t < nt; t += gridDim.x) {
        uint64_t base = tile_nl[t];
        uint32_t w[4][4], nx[4][4];   // this group's chunks, the next group's (loaded ahead)
#pragma unroll
        for (uint32_t rr = 0; rr < 4; rr++) load_chunk(text, n, (t * kRounds + rr) * kPB + threadIdx.x, aligned, nx[rr]);
#pragma unroll 1
        for (uint32_t g = 0; g < kRounds; g += 4) {
            uint64_t packed = 0;
#pragma unroll
            for (uint32_t rr = 0; rr < 4; rr++) {
#pragma unroll
                for (int i = 0; i < 4; i++) w[rr][i] = nx[rr][i];
                packed |= (uint64_t)chunk_newlines(w[rr]) << (16 * rr);
            }
            if (g + 4 < kRounds) {
#pragma unroll
                for (uint32_t rr = 0; rr < 4; rr++)
                    load_chunk(text, n, (t * kRounds + g + 4 + rr) * kPB + threadIdx.x, aligned, nx[rr]);
            }
            uint64_t total;
            const uint64_t excl = block_scan64(packed, wsum, total);
#pragma unroll
            for (uint32_t rr = 0; rr < 4; rr++) {
                const uint64_t c = (t * kRounds + g + rr) * kPB + threadIdx.x;
                uint64_t idx = base + ((excl >> (16 * rr)) & 0xFFFFull);
#pragma unroll
                for (int i = 0; i < 4; i++) {
                    uint32_t m = nl_bytes(w[rr][i]);
                    while (m) {
                        const uint32_t j = 4 * i + ((uint32_t)__builtin_ctz(m) >> 3);   // byte of the chunk
                        m &= m - 1;
                        const uint64_t p = c * kChunk + j;   // < n: bytes past n read as 0
                        const uint32_t before = j ? chunk_byte(w[rr], j - 1) : (p ? (uint32_t)text[p - 1] : 0u);
                        const uint32_t after = j < kChunk - 1 ? chunk_byte(w[rr], j + 1)
                                                              : (p + 1 < n ? (uint32_t)text[p + 1] : 0u);
                        if (idx < lines_cap)
                            line[idx] = p | ((uint64_t)(before == '\r') << 40) | ((uint64_t)after << 48);
                        idx++;
                    }
                }
                base += (total >> (16 * rr)) & 0xFFFFull;
            }
        }
    }
}

struct LineInfo {
    uint64_t kept;    // sequence bytes of the line
    uint32_t starts;  // 1 if the line starts a read
    uint32_t err;     // GERBIL_PARSE_* bits found at this line
};

__device__ __forceinline__ uint64_t line_start(const uint64_t* line, uint64_t i) {
    return i ? (line[i - 1] & kPosMask) + 1 : 0ull;
}
__device__ __forceinline__ uint64_t line_body(const uint64_t* line, uint64_t i) {
    const uint64_t w = line[i];
    const uint64_t e = w & kPosMask, s = line_start(line, i);
    return e - s - ((w >> 40) & 1ull);
}
__device__ __forceinline__ uint32_t line_first(const uint64_t* line, uint64_t i, uint32_t first0) {
    return i ? (uint32_t)(line[i - 1] >> 48) & 0xFFu : first0;
}

__device__ __forceinline__ LineInfo classify(const uint64_t* line, uint64_t i, uint64_t lines, uint32_t fmt,
                                             uint32_t first0) {
    LineInfo x{0, 0, 0};
    if (fmt == GERBIL_FORMAT_FASTQ) {
        if ((i & 3) != 1) return x;
        x.starts = 1;
        x.kept = line_body(line, i);
        // an empty header line has the newline itself as "first byte"
        if (line_first(line, i - 1, first0) != '@') x.err |= GERBIL_PARSE_EHEADER;
        if (i + 1 < lines && line_first(line, i + 1, first0) != '+') x.err |= GERBIL_PARSE_EPLUS;
        if (i + 2 < lines && line_body(line, i + 2) != x.kept) x.err |= GERBIL_PARSE_EQUAL;
    } else {
        const bool empty = (line[i] & kPosMask) == line_start(line, i);
        if (!empty && line_first(line, i, first0) == '>') {
            x.starts = 1;
        } else {
            x.kept = line_body(line, i);
        }
    }
    return x;
}

__device__ __forceinline__ bool lines_usable(const gerbil_parsed* out, uint64_t& lines, uint32_t& fmt) {
    const uint32_t st = out->status;
    fmt = out->format;
    lines = out->n_lines;
    return fmt != 0 && !(st & (GERBIL_PARSE_ELINECAP | GERBIL_PARSE_EFORMAT));
}

// 4. kept bytes and reads per line tile; format checks
__global__ void __launch_bounds__(kPB) k_line_sums(const uint8_t* __restrict__ text, const uint64_t* __restrict__ line,
                                                   uint64_t* __restrict__ lt_kept, uint64_t* __restrict__ lt_reads,
                                                   gerbil_parsed* out) {
    __shared__ uint64_t wsum[kPB / 64 + 1];
    __shared__ uint32_t err_s;
    uint64_t lines;
    uint32_t fmt;
    if (!lines_usable(out, lines, fmt)) return;
    const uint32_t first0 = lines ? text[0] : 0u;
    const uint64_t nt = n_ltiles_of(lines);
    for (uint64_t t = blockIdx.x; t < nt; t += gridDim.x) {
        if (threadIdx.x == 0) err_s = 0;
        uint64_t kept = 0, reads = 0;
        uint32_t err = 0;
        const uint64_t i0 = t * kLineTile + (uint64_t)threadIdx.x * kLinesPer;
        for (uint32_t j = 0; j < kLinesPer; j++) {
            const uint64_t i = i0 + j;
            if (i >= lines) break;
            const LineInfo x = classify(line, i, lines, fmt, first0);
            kept += x.kept;
            reads += x.starts;
            err |= x.err;
        }
        uint64_t tk, tr;
        (void)block_scan64(kept, wsum, tk);
        (void)block_scan64(reads, wsum, tr);
        if (err) atomicOr(&err_s, err);
        __syncthreads();
        if (threadIdx.x == 0) {
            lt_kept[t] = tk;
            lt_reads[t] = tr;
            if (err_s) set_status(&out->status, err_s);
        }
    }
}

// 5. scan of the line tile sums; totals and capacity checks
__global__ void __launch_bounds__(kScanBlock) k_line_scan(uint64_t* __restrict__ lt_kept, uint64_t* __restrict__ lt_reads,
                                                          uint64_t* __restrict__ offsets, uint64_t seq_cap,
                                                          uint64_t reads_cap, gerbil_parsed* out) {
    __shared__ uint64_t wsum[kScanBlock / 64 + 1];
    uint64_t lines;
    uint32_t fmt;
    if (!lines_usable(out, lines, fmt)) return;
    const uint64_t nt = n_ltiles_of(lines);
    const uint64_t bytes = wg_scan_inplace(lt_kept, nt, wsum);
    const uint64_t reads = wg_scan_inplace(lt_reads, nt, wsum);
    if (threadIdx.x != 0) return;
    uint32_t st = 0;
    if (fmt == GERBIL_FORMAT_FASTQ && (lines & 3)) st |= GERBIL_PARSE_ELINES;
    if (fmt == GERBIL_FORMAT_FASTA && reads == 0 && bytes > 0) st |= GERBIL_PARSE_EORPHAN;
    if (bytes > seq_cap) st |= GERBIL_PARSE_EBYTES;
    if (reads > reads_cap) st |= GERBIL_PARSE_EREADS;
    else offsets[reads] = bytes;
    out->n_bytes = bytes;
    out->n_reads = reads;
    if (st) set_status(&out->status, st);
}

// 6. line offsets and read offsets
__global__ void __launch_bounds__(kPB) k_line_apply(const uint8_t* __restrict__ text, const uint64_t* __restrict__ line,
                                                    const uint64_t* __restrict__ lt_kept,
                                                    const uint64_t* __restrict__ lt_reads,
                                                    uint64_t* __restrict__ line_off, uint64_t* __restrict__ offsets,
                                                    uint64_t reads_cap, gerbil_parsed* out) {
    __shared__ uint64_t wsum[kPB / 64 + 1];
    uint64_t lines;
    uint32_t fmt;
    if (!lines_usable(out, lines, fmt)) return;
    const uint32_t first0 = lines ? text[0] : 0u;
    const uint64_t nt = n_ltiles_of(lines);
    for (uint64_t t = blockIdx.x; t < nt; t += gridDim.x) {
        const uint64_t i0 = t * kLineTile + (uint64_t)threadIdx.x * kLinesPer;
        LineInfo x[kLinesPer];
        uint64_t kept = 0, reads = 0;
#pragma unroll
        for (uint32_t j = 0; j < kLinesPer; j++) {
            x[j] = i0 + j < lines ? classify(line, i0 + j, lines, fmt, first0) : LineInfo{0, 0, 0};
            kept += x[j].kept;
            reads += x[j].starts;
        }
        uint64_t tk, tr;
        uint64_t ko = lt_kept[t] + block_scan64(kept, wsum, tk);
        uint64_t ro = lt_reads[t] + block_scan64(reads, wsum, tr);
        bool orphan = false;
#pragma unroll
        for (uint32_t j = 0; j < kLinesPer; j++) {
            if (i0 + j >= lines) break;
            line_off[i0 + j] = ko;
            if (x[j].starts) {
                if (ro < reads_cap) offsets[ro] = ko;
                orphan |= fmt == GERBIL_FORMAT_FASTA && ro == 0 && ko != 0;
                ro++;
            }
            ko += x[j].kept;
        }
        if (orphan) set_status(&out->status, GERBIL_PARSE_EORPHAN);
    }
}

// 7. per line tile: the tile's lines own the output range [O0, O1); each
// lane fills aligned 16-byte chunks of it (two at a time, so that their loads
// overlap). The line holding a chunk's first byte is found by binary search
// in the tile's offsets, which sit in LDS with the line starts. A chunk that
// lies inside one line is two aligned 16-byte loads and a byte funnel shift;
// one that spans lines, or is cut by the range ends or seq_cap, is gathered
// and written byte by byte (its bytes outside the range belong to
// neighbouring tiles).
constexpr uint32_t kCopyBatch = 2;
constexpr uint32_t kCopyTile = 2 * kPB;   // lines per copy tile: 8 KB of LDS, many workgroups per CU

// bytes [o, o + 16) of the 32 bytes a, b (o < 16)
__device__ __forceinline__ uint4 funnel16(const uint4 a, const uint4 b, uint32_t o) {
    const uint32_t r = o & 3;
    uint32_t e0, e1, e2, e3, e4;
    switch (o >> 2) {
        case 0: e0 = a.x; e1 = a.y; e2 = a.z; e3 = a.w; e4 = b.x; break;
        case 1: e0 = a.y; e1 = a.z; e2 = a.w; e3 = b.x; e4 = b.y; break;
        case 2: e0 = a.z; e1 = a.w; e2 = b.x; e3 = b.y; e4 = b.z; break;
        default: e0 = a.w; e1 = b.x; e2 = b.y; e3 = b.z; e4 = b.w; break;
    }
    return make_uint4(__builtin_amdgcn_alignbyte(e1, e0, r), __builtin_amdgcn_alignbyte(e2, e1, r),
                      __builtin_amdgcn_alignbyte(e3, e2, r), __builtin_amdgcn_alignbyte(e4, e3, r));
}

__global__ void __launch_bounds__(kPB) k_line_copy(const uint8_t* __restrict__ text, uint64_t n,
                                                   const uint64_t* __restrict__ line,
                                                   const uint64_t* __restrict__ line_off, uint8_t* __restrict__ seq,
                                                   uint64_t seq_cap, gerbil_parsed* out) {
    __shared__ uint64_t s_off[kCopyTile + 1];
    __shared__ uint64_t s_start[kCopyTile];
    uint64_t lines;
    uint32_t fmt;
    if (!lines_usable(out, lines, fmt)) return;
    const uint64_t total = out->n_bytes;
    const uint64_t ms = ((uintptr_t)seq) & 15;   // chunks are aligned in the address space
    const uintptr_t t_lo = (uintptr_t)text, t_hi = (uintptr_t)text + n;
    const uint64_t nt = (lines + kCopyTile - 1) / kCopyTile;
    for (uint64_t t = blockIdx.x; t < nt; t += gridDim.x) {
        const uint64_t i0 = t * kCopyTile;
        const uint32_t cnt = (uint32_t)(lines - i0 < kCopyTile ? lines - i0 : kCopyTile);
        // the tables: every load issued before any is used
        uint64_t o_v[kCopyTile / kPB + 1], s_v[kCopyTile / kPB];
#pragma unroll
        for (uint32_t r = 0; r <= kCopyTile / kPB; r++) {
            const uint32_t j = threadIdx.x + r * kPB;
            const uint64_t i = i0 + j;
            o_v[r] = j <= cnt ? (i < lines ? line_off[i] : total) : 0ull;
            if (r < kCopyTile / kPB) s_v[r] = j < cnt && i ? line[i - 1] : 0ull;
        }
#pragma unroll
        for (uint32_t r = 0; r <= kCopyTile / kPB; r++) {
            const uint32_t j = threadIdx.x + r * kPB;
            if (j <= cnt) s_off[j] = o_v[r];
            if (r < kCopyTile / kPB && j < cnt) s_start[j] = i0 + j ? (s_v[r] & kPosMask) + 1 : 0ull;
        }
        __syncthreads();
        const uint64_t O0 = s_off[0], O1 = s_off[cnt];
        if (O1 > O0) {
            const uint64_t c0 = (O0 + ms) / kChunk, c1 = (O1 + ms + kChunk - 1) / kChunk;
            for (uint64_t cb = c0 + threadIdx.x; cb < c1; cb += (uint64_t)kPB * kCopyBatch) {
                uint4 v[kCopyBatch];
                bool fast[kCopyBatch];
#pragma unroll
                for (uint32_t b = 0; b < kCopyBatch; b++) {
                    const uint64_t c = cb + (uint64_t)b * kPB;
                    fast[b] = false;
                    v[b] = make_uint4(0u, 0u, 0u, 0u);
                    if (c >= c1) continue;
                    // byte k of the chunk is output byte a0 + k - ms; it belongs to this
                    // tile iff O0 + ms <= a0 + k < O1 + ms (never negative: no wrap)
                    const uint64_t a0 = c * kChunk;
                    const uint64_t qs = (a0 > O0 + ms ? a0 : O0 + ms) - ms;
                    // last line whose offset is <= qs: the line holding byte qs
                    uint32_t lo = 0, hi = cnt;
                    while (hi - lo > 1) {
                        const uint32_t mid = (lo + hi) >> 1;
                        if (s_off[mid] <= qs) lo = mid; else hi = mid;
                    }
                    uint32_t j = lo;
                    uint64_t lend = s_off[j + 1];
                    const bool whole = a0 >= O0 + ms && a0 + kChunk <= O1 + ms && a0 + kChunk <= seq_cap + ms;
                    const uint64_t q0 = whole ? a0 - ms : 0;
                    if (whole && q0 + kChunk <= lend) {
                        const uintptr_t src = (uintptr_t)(text + s_start[j] + (q0 - s_off[j]));
                        const uintptr_t A = src & ~(uintptr_t)15;
                        if (A >= t_lo && A + 32 <= t_hi) {
                            const uint4 x = *(const uint4*)A, y = *(const uint4*)(A + 16);
                            v[b] = funnel16(x, y, (uint32_t)(src & 15));
                            fast[b] = true;
                            continue;
                        }
                    }
                    uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
                    for (uint32_t k = 0; k < kChunk; k++) {
                        if (a0 + k >= O0 + ms && a0 + k < O1 + ms) {
                            const uint64_t q = a0 + k - ms;
                            while (q >= lend) lend = s_off[++j + 1];
                            w[k >> 2] |= (uint32_t)text[s_start[j] + (q - s_off[j])] << (8 * (k & 3));
                        }
                    }
                    v[b] = make_uint4(w[0], w[1], w[2], w[3]);
                }
#pragma unroll
                for (uint32_t b = 0; b < kCopyBatch; b++) {
                    const uint64_t c = cb + (uint64_t)b * kPB;
                    if (c >= c1) continue;
                    const uint64_t a0 = c * kChunk;
                    if (fast[b] || (a0 >= O0 + ms && a0 + kChunk <= O1 + ms && a0 + kChunk <= seq_cap + ms)) {
                        *(uint4*)(seq + (a0 - ms)) = v[b];
                    } else {
                        const uint32_t w[4] = {v[b].x, v[b].y, v[b].z, v[b].w};
#pragma unroll
                        for (uint32_t k = 0; k < kChunk; k++) {
                            if (a0 + k >= O0 + ms && a0 + k < O1 + ms && a0 + k < seq_cap + ms)
                                seq[a0 + k - ms] = (uint8_t)(w[k >> 2] >> (8 * (k & 3)));
                        }
                    }
                }
            }
        }
        __syncthreads();   // the LDS tables are refilled for the next tile
    }
}

uint32_t grid_of(uint64_t tiles) {
    return (uint32_t)(tiles == 0 ? 1 : tiles < kMaxTileGridParse ? tiles : kMaxTileGridParse);
}

}  // namespace
}  // namespace gerbil

using namespace gerbil;

extern "C" {

int32_t gerbil_parse_workspace(uint64_t n, uint64_t lines_cap, uint64_t* bytes) {
    if (!bytes || n >= (1ull << 40) || lines_cap > n + 1) return GERBIL_EINVAL;
    *bytes = ws_layout(n, lines_cap, nullptr, nullptr);
    return GERBIL_OK;
}

int32_t gerbil_parse(const uint8_t* text, uint64_t n, uint32_t format, void* ws, uint64_t ws_bytes,
                     uint64_t lines_cap, uint8_t* seq, uint64_t seq_cap, uint64_t* offsets, uint64_t reads_cap,
                     gerbil_parsed* out, hipStream_t stream) {
    if (!out || !offsets || !ws || (n && !text) || (seq_cap && !seq)) return GERBIL_EINVAL;
    if (format > GERBIL_FORMAT_FASTA || n >= (1ull << 40) || lines_cap > n + 1) return GERBIL_EINVAL;
    if (((uintptr_t)ws) & 255) return GERBIL_EINVAL;
    Ws w;
    if (ws_bytes < ws_layout(n, lines_cap, (uint8_t*)ws, &w)) return GERBIL_EINVAL;
    const bool aligned = (((uintptr_t)text) & 15) == 0;
    const uint64_t bt = n_btiles_of(n), lt = n_ltiles_of(lines_cap);
    hipLaunchKernelGGL(k_parse_init, dim3(1), dim3(64), 0, stream, text, n, format, out);
    hipLaunchKernelGGL(k_nl_count, dim3(grid_of(bt)), dim3(kPB), 0, stream, text, n, aligned, w.tile_nl);
    hipLaunchKernelGGL(k_nl_scan, dim3(1), dim3(kScanBlock), 0, stream, text, n, w.tile_nl, w.line, lines_cap, out);
    hipLaunchKernelGGL(k_nl_write, dim3(grid_of(bt)), dim3(kPB), 0, stream, text, n, aligned, w.tile_nl, w.line,
                       lines_cap);
    hipLaunchKernelGGL(k_line_sums, dim3(grid_of(lt)), dim3(kPB), 0, stream, text, w.line, w.lt_kept, w.lt_reads, out);
    hipLaunchKernelGGL(k_line_scan, dim3(1), dim3(kScanBlock), 0, stream, w.lt_kept, w.lt_reads, offsets, seq_cap,
                       reads_cap, out);
    hipLaunchKernelGGL(k_line_apply, dim3(grid_of(lt)), dim3(kPB), 0, stream, text, w.line, w.lt_kept, w.lt_reads,
                       w.line_off, offsets, reads_cap, out);
    hipLaunchKernelGGL(k_line_copy, dim3(grid_of((lines_cap + kCopyTile - 1) / kCopyTile)), dim3(kPB), 0, stream, text,
                       n, w.line, w.line_off, seq, seq_cap, out);
    return hipGetLastError() == hipSuccess ? GERBIL_OK : GERBIL_EDEVICE;
}

}  // extern "C"

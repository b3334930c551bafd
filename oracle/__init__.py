"""CPU oracle for canonical k-mer counting -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The GPU library never uses it.

Thin ctypes wrapper over ``gerbil_oracle.c``; every function's arithmetic is
in the C file, which cites the passages of the paper it follows. The
exceptions, written here in plain Python from their definitions, are
``parse_reads`` (FASTA/FASTQ text to reads) and ``order_table`` (the
minimizer orders of Sec. 3.1 as rank tables).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gerbil_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# A test may point the oracle at another build of gerbil_oracle.c (the
# mutation test loads deliberately broken copies this way); it is never built here.
_LIB_OVERRIDE = os.environ.get("ORACLE_LIBRARY")
_lib = None


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (plain C, single-threaded)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", _SRC, "-o", tmp], check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Keys(ctypes.Structure):
    _fields_ = [("keys", ctypes.POINTER(ctypes.c_uint64)), ("n", ctypes.c_uint64), ("cap", ctypes.c_uint64)]


class _Result(ctypes.Structure):
    _fields_ = [("n_valid", ctypes.c_uint64), ("n_valid_shard", ctypes.c_uint64),
                ("n_distinct", ctypes.c_uint64), ("n_pairs", ctypes.c_uint64),
                ("keys", ctypes.POINTER(ctypes.c_uint64)), ("counts", ctypes.POINTER(ctypes.c_uint32)),
                ("hist", ctypes.POINTER(ctypes.c_uint64)), ("hist_len", ctypes.c_uint64),
                ("max_count", ctypes.c_uint64)]


def _load():
    global _lib
    if _lib is None:
        if _LIB_OVERRIDE:
            lib = ctypes.CDLL(_LIB_OVERRIDE)
        else:
            if not os.path.exists(_LIB):
                build(force=True)
            lib = ctypes.CDLL(_LIB)
        vp, u64, u32, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
        lib.oracle_count.argtypes = [vp, vp, u64, u32, u32, u32, u64, u64, ctypes.POINTER(_Result)]
        lib.oracle_count.restype = i32
        lib.oracle_free.argtypes = [ctypes.POINTER(_Result)]
        lib.oracle_free.restype = None
        lib.oracle_count_keys.argtypes = [vp, vp, u64, u32, vp, u64, vp]
        lib.oracle_count_keys.restype = i32
        lib.oracle_count_keys_range.argtypes = [vp, vp, u64, u64, u32, vp, u64, vp]
        lib.oracle_count_keys_range.restype = i32
        lib.oracle_encode.argtypes = [vp, vp, u64, u32, vp, vp, vp]
        lib.oracle_encode.restype = i32
        lib.oracle_supermers.argtypes = [vp, vp, u64, u32, u32, u32, u32, vp, vp, vp, vp, vp, vp, u64, vp]
        lib.oracle_supermers.restype = i32
        lib.oracle_shard_of.argtypes = [vp, u32, u64]
        lib.oracle_shard_of.restype = u64
        lib.oracle_shard_of_many.argtypes = [vp, u64, u32, u64, vp]
        lib.oracle_shard_of_many.restype = None
        lib.oracle_collect.argtypes = [vp, vp, u64, u64, u32, u32, u64, u64, u64, vp, vp]
        lib.oracle_collect.restype = i32
        lib.oracle_count_multiset.argtypes = [vp, u64, u32, u32, ctypes.POINTER(_Result)]
        lib.oracle_count_multiset.restype = i32
        lib.oracle_keys_free.argtypes = [vp]
        lib.oracle_keys_free.restype = None
        lib.oracle_record.argtypes = [ctypes.c_char_p, u32, u32, vp]
        lib.oracle_record.restype = u32
        _lib = lib
    return _lib


def words(k: int) -> int:
    return (k + 31) // 32


def _c(a: np.ndarray, dtype) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=dtype)


@dataclass
class Counted:
    """Oracle result: sorted pairs (count >= threshold) and the full histogram."""
    k: int
    n_valid: int            # valid windows of the whole input
    n_valid_shard: int      # valid windows whose canonical key is in the shard
    n_distinct: int
    keys: np.ndarray        # uint64 [n_pairs, W], ascending
    counts: np.ndarray      # uint32 [n_pairs]
    hist: np.ndarray        # uint64 [max_count + 1]; hist[c] = #distinct keys with count c

    def folded_hist(self, length: int) -> np.ndarray:
        """Histogram folded to ``length`` buckets, last bucket = counts >= length-1."""
        h = np.zeros(length, dtype=np.uint64)
        n = min(length - 1, self.hist.size)
        h[:n] = self.hist[:n]
        if self.hist.size > length - 1:
            h[length - 1] = self.hist[length - 1:].sum()
        h[0] = 0
        return h


def count(ascii: np.ndarray, offsets: np.ndarray, k: int, threshold: int = 1, canonical: bool = True,
          shard_mod: int = 1, shard_id: int = 0) -> Counted:
    """Sort-and-count of (canonical) k-mers; see ``oracle_count`` in the C file."""
    lib = _load()
    a, o = _c(ascii, np.uint8), _c(offsets, np.uint64)
    r = _Result()
    rc = lib.oracle_count(a.ctypes.data, o.ctypes.data, o.size - 1, k, threshold, int(canonical),
                          shard_mod, shard_id, ctypes.byref(r))
    if rc != 0:
        raise RuntimeError(f"oracle_count failed with status {rc}")
    try:
        return _counted(k, r)
    finally:
        lib.oracle_free(ctypes.byref(r))


def _counted(k: int, r: "_Result") -> Counted:
    W = words(k)
    n = r.n_pairs
    keys = np.ctypeslib.as_array(r.keys, shape=(max(n, 1) * W,))[: n * W].reshape(n, W).copy()
    counts = np.ctypeslib.as_array(r.counts, shape=(max(n, 1),))[:n].copy()
    hist = np.ctypeslib.as_array(r.hist, shape=(r.hist_len,)).copy() if r.hist_len else \
        np.zeros(1, dtype=np.uint64)
    return Counted(k, int(r.n_valid), int(r.n_valid_shard), int(r.n_distinct), keys, counts, hist)


def count_multiset(keys: np.ndarray, k: int, threshold: int = 1) -> Counted:
    """Steps 6-9 of the definition over a multiset of packed keys ([n, W]
    uint64, sorted in place): see ``oracle_count_multiset`` in the C file."""
    lib = _load()
    W = words(k)
    ks = keys.reshape(-1, W)
    assert ks.dtype == np.uint64 and ks.flags["C_CONTIGUOUS"]
    r = _Result()
    rc = lib.oracle_count_multiset(ks.ctypes.data, ks.shape[0], W, threshold, ctypes.byref(r))
    if rc != 0:
        lib.oracle_free(ctypes.byref(r))
        raise RuntimeError(f"oracle_count_multiset failed with status {rc}")
    try:
        return _counted(k, r)
    finally:
        lib.oracle_free(ctypes.byref(r))


def count_sharded(ascii: np.ndarray, offsets: np.ndarray, k: int, threshold: int, shard_mod: int,
                  on_shard, canonical: bool = True, group: int = 0, threads: int = 8, sort_workers: int = 2) -> int:
    """The result of ``count`` split into ``shard_mod`` shards by
    ``oracle_shard_of``, for read sets whose keys do not fit in memory at once.

    Shards are taken ``group`` at a time (0: all at once). For each group the
    reads are cut into ``threads`` ranges whose keys are collected
    concurrently (steps 1-5, ``oracle_collect``); then each shard's keys are
    joined and counted (steps 6-9, ``oracle_count_multiset``), and
    ``on_shard(s, Counted)`` is called once per shard, in shard order within a
    group. Every key lands in exactly one shard, so the shards' pairs are the
    pairs of ``count`` and their histograms add up to its histogram. Returns the
    number of valid windows of the input. Memory: the keys of one group, plus
    about two shards per sort worker."""
    import concurrent.futures as cf
    lib = _load()
    W = words(k)
    a, o = _c(ascii, np.uint8), _c(offsets, np.uint64)
    n_reads = o.size - 1
    group = shard_mod if group <= 0 else min(group, shard_mod)
    cuts = np.linspace(0, n_reads, max(1, threads) + 1).astype(np.int64)
    L = np.diff(o.astype(np.int64))
    win = np.maximum(L - k + 1, 0)
    win_cum = np.concatenate([[0], np.cumsum(win)])
    n_valid_total = None
    for s_lo in range(0, shard_mod, group):
        s_hi = min(shard_mod, s_lo + group)
        G = s_hi - s_lo
        outs = []
        for t in range(len(cuts) - 1):
            arr = (_Keys * G)()
            expect = int(win_cum[cuts[t + 1]] - win_cum[cuts[t]]) / max(1, shard_mod)
            for i in range(G):
                arr[i].cap = int(expect * 1.02) + 4096
            outs.append(arr)
        nv = [np.zeros(1, dtype=np.uint64) for _ in outs]

        def collect(t):
            return lib.oracle_collect(a.ctypes.data, o.ctypes.data, int(cuts[t]), int(cuts[t + 1]), k,
                                      int(canonical), shard_mod, s_lo, s_hi, ctypes.addressof(outs[t]),
                                      nv[t].ctypes.data)

        try:
            with cf.ThreadPoolExecutor(max_workers=len(outs)) as ex:
                rcs = list(ex.map(collect, range(len(outs))))
            if any(rc != 0 for rc in rcs):
                raise RuntimeError(f"oracle_collect failed with status {rcs}")
            n_valid = int(sum(int(x[0]) for x in nv))
            if n_valid_total is None:
                n_valid_total = n_valid
            assert n_valid == n_valid_total

            def count_shard(i):
                n = sum(int(outs[t][i].n) for t in range(len(outs)))
                joined = np.empty((max(n, 1), W), dtype=np.uint64)
                pos = 0
                for t in range(len(outs)):
                    part = outs[t][i]
                    if part.n:
                        src = np.ctypeslib.as_array(part.keys, shape=(int(part.n) * W,))
                        joined.reshape(-1)[pos * W: (pos + int(part.n)) * W] = src
                        pos += int(part.n)
                    lib.oracle_keys_free(ctypes.byref(part))
                res = count_multiset(joined[:n], k, threshold)
                del joined
                res.n_valid = n_valid
                return res

            with cf.ThreadPoolExecutor(max_workers=max(1, sort_workers)) as ex:
                futs = [ex.submit(count_shard, i) for i in range(G)]
                for i, f in enumerate(futs):
                    on_shard(s_lo + i, f.result())
        finally:
            for arr in outs:
                for i in range(G):
                    lib.oracle_keys_free(ctypes.byref(arr[i]))
    return int(n_valid_total or 0)


def count_keys(ascii: np.ndarray, offsets: np.ndarray, k: int, query: np.ndarray) -> np.ndarray:
    """Occurrences of each canonical key in ``query`` ([n, W] uint64)."""
    lib = _load()
    W = words(k)
    q = _c(query, np.uint64).reshape(-1, W)
    order = np.lexsort(q.T[::-1])
    qs = np.ascontiguousarray(q[order])
    out = np.zeros(qs.shape[0], dtype=np.uint64)
    a, o = _c(ascii, np.uint8), _c(offsets, np.uint64)
    rc = lib.oracle_count_keys(a.ctypes.data, o.ctypes.data, o.size - 1, k, qs.ctypes.data, qs.shape[0],
                               out.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"oracle_count_keys failed with status {rc}")
    res = np.empty_like(out)
    res[order] = out
    return res


def count_keys_parallel(ascii: np.ndarray, offsets: np.ndarray, k: int, query: np.ndarray,
                        threads: int = 16) -> np.ndarray:
    """Same result as ``count_keys`` for large read sets: the reads are split
    into ``threads`` ranges counted concurrently (the C code runs without the
    interpreter lock), and a window is canonicalised only when one of its
    strands begins like a query key."""
    import concurrent.futures as cf
    lib = _load()
    W = words(k)
    q = _c(query, np.uint64).reshape(-1, W)
    order = np.lexsort(q.T[::-1])
    qs = np.ascontiguousarray(q[order])
    a, o = _c(ascii, np.uint8), _c(offsets, np.uint64)
    n_reads = o.size - 1
    cuts = np.linspace(0, n_reads, max(1, threads) + 1).astype(np.int64)
    parts = [np.zeros(qs.shape[0], dtype=np.uint64) for _ in range(len(cuts) - 1)]

    def run(i):
        return lib.oracle_count_keys_range(a.ctypes.data, o.ctypes.data, int(cuts[i]), int(cuts[i + 1]), k,
                                           qs.ctypes.data, qs.shape[0], parts[i].ctypes.data)

    with cf.ThreadPoolExecutor(max_workers=len(parts)) as ex:
        rcs = list(ex.map(run, range(len(parts))))
    if any(rc != 0 for rc in rcs):
        raise RuntimeError(f"oracle_count_keys_range failed with status {rcs}")
    out = np.sum(parts, axis=0, dtype=np.uint64) if parts else np.zeros(qs.shape[0], np.uint64)
    res = np.empty_like(out)
    res[order] = out
    return res


def encode(ascii: np.ndarray, offsets: np.ndarray, k: int):
    """(packed uint64[ceil(n/32)], kmer_ok uint64[ceil(n/64)], n_valid)."""
    lib = _load()
    a, o = _c(ascii, np.uint8), _c(offsets, np.uint64)
    n = int(o[-1])
    packed = np.zeros((n + 31) // 32, dtype=np.uint64)
    ok = np.zeros((n + 63) // 64, dtype=np.uint64)
    nv = np.zeros(1, dtype=np.uint64)
    rc = lib.oracle_encode(a.ctypes.data, o.ctypes.data, o.size - 1, k, packed.ctypes.data, ok.ctypes.data,
                           nv.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"oracle_encode failed with status {rc}")
    return packed, ok, int(nv[0])


def supermers(ascii: np.ndarray, offsets: np.ndarray, k: int, m: int, n_bins: int, order: int = 0,
              bin_map: Optional[np.ndarray] = None, rank_table: Optional[np.ndarray] = None):
    """Super-mers as a dict of arrays: start, n_kmers, bin, rank (in read order).
    order 2 ranks canonical m-mers by ``rank_table`` (see ``order_table``)."""
    lib = _load()
    a, o = _c(ascii, np.uint8), _c(offsets, np.uint64)
    cap = max(1, int(o[-1]))
    start = np.empty(cap, dtype=np.uint64)
    nk = np.empty(cap, dtype=np.uint32)
    b = np.empty(cap, dtype=np.uint32)
    rank = np.empty(cap, dtype=np.uint64)
    n = np.zeros(1, dtype=np.uint64)
    bm = _c(bin_map, np.uint32) if bin_map is not None else None
    rt = _c(rank_table, np.uint32) if rank_table is not None else None
    rc = lib.oracle_supermers(a.ctypes.data, o.ctypes.data, o.size - 1, k, m, order, n_bins,
                              bm.ctypes.data if bm is not None else None, rt.ctypes.data if rt is not None else None,
                              start.ctypes.data, nk.ctypes.data, b.ctypes.data, rank.ctypes.data, cap,
                              n.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"oracle_supermers failed with status {rc}")
    c = int(n[0])
    return {"start": start[:c].copy(), "n_kmers": nk[:c].copy(), "bin": b[:c].copy(), "rank": rank[:c].copy()}


def shard_of(keys: np.ndarray, k: int, shard_mod: int) -> np.ndarray:
    """Shard id of each key row (the oracle's memory-bounding partition)."""
    import concurrent.futures as cf
    lib = _load()
    W = words(k)
    ks = _c(keys, np.uint64).reshape(-1, W)
    n = ks.shape[0]
    out = np.empty(n, dtype=np.uint64)
    cuts = np.linspace(0, n, 17).astype(np.int64) if n > (1 << 20) else np.array([0, n])

    def part(i):
        lo, hi = int(cuts[i]), int(cuts[i + 1])
        if hi > lo:
            lib.oracle_shard_of_many(ks[lo:hi].ctypes.data, hi - lo, W, shard_mod, out[lo:hi].ctypes.data)

    with cf.ThreadPoolExecutor(max_workers=len(cuts) - 1) as ex:
        list(ex.map(part, range(len(cuts) - 1)))
    return out


def record(kmer: str, count: int) -> bytes:
    """One output record of the paper's binary format (App. C)."""
    buf = (ctypes.c_uint8 * (5 + (len(kmer) + 3) // 4))()
    n = _load().oracle_record(kmer.encode(), len(kmer), count, ctypes.addressof(buf))
    return bytes(buf[:n])


def decode_key(key: np.ndarray, k: int) -> str:
    """String of a packed key (test helper: inverse of the key layout)."""
    W = words(k)
    out = []
    for i in range(W):
        nb = 32 if i < W - 1 else k - 32 * (W - 1)
        w = int(key[i])
        for j in range(nb):
            out.append("ACGT"[(w >> (2 * (nb - 1 - j))) & 3])
    return "".join(out)


# ------------------------------------------------------------------ input parsing

FASTQ, FASTA = 1, 2
PARSE_EHEADER = 1    # FASTQ: a record's first line is empty or does not start with '@'
PARSE_EPLUS = 2      # FASTQ: a record's third line does not start with '+'
PARSE_EQUAL = 4      # FASTQ: quality and sequence lengths differ
PARSE_ELINES = 8     # FASTQ: the number of lines is not a multiple of four
PARSE_EORPHAN = 16   # FASTA: sequence bytes before the first header
PARSE_EFORMAT = 128  # format to be detected, and the text starts with neither '@' nor '>'


@dataclass
class Parsed:
    ascii: np.ndarray     # uint8: the reads back to back
    offsets: np.ndarray   # uint64 [n_reads + 1]
    status: int           # PARSE_* bits; the reads are defined only when it is 0
    fmt: int              # FASTQ, FASTA, or 0 (empty text or undetected)
    n_lines: int
    n_bytes: int          # sequence bytes over every sequence line (also when status != 0)


def parse_reads(text: bytes, fmt: int = 0) -> Parsed:
    """Reads of a FASTA or FASTQ text (the input formats of App. B), as the
    CSR arrays the encoder takes.

    Lines end at a newline; a final line may lack one; one carriage return
    right before a line's end is not part of the line. FASTQ records are four
    lines (header starting with '@', sequence, a line starting with '+',
    quality of the sequence's length) and each sequence line is one read.
    FASTA: a non-empty line starting with '>' starts a read; every other line
    is sequence and is appended to the current read (multi-line records).
    Sequence bytes are kept as they are (the encoder decides which are
    bases). fmt 0 detects the format from the first byte.
    """
    lines = text.split(b"\n")
    if not text or text.endswith(b"\n"):
        lines.pop()   # the piece after the final newline is not a line
    n_lines = len(lines)
    status = 0
    if fmt == 0 and text:
        fmt = FASTQ if text[:1] == b"@" else FASTA if text[:1] == b">" else 0
        if fmt == 0:
            status |= PARSE_EFORMAT

    def body(line: bytes) -> bytes:
        return line[:-1] if line.endswith(b"\r") else line

    reads = []
    n_bytes = 0
    if fmt == FASTQ:
        if n_lines % 4:
            status |= PARSE_ELINES
        for i in range(1, n_lines, 4):
            head = lines[i - 1]
            if not head.startswith(b"@"):
                status |= PARSE_EHEADER
            if i + 1 < n_lines and not lines[i + 1].startswith(b"+"):
                status |= PARSE_EPLUS
            seq = body(lines[i])
            if i + 2 < n_lines and len(body(lines[i + 2])) != len(seq):
                status |= PARSE_EQUAL
            reads.append(seq)
            n_bytes += len(seq)
    elif fmt == FASTA:
        for line in lines:
            if line.startswith(b">"):
                reads.append(bytearray())
                continue
            seq = body(line)
            n_bytes += len(seq)
            if not reads:
                if seq:
                    status |= PARSE_EORPHAN
                continue
            reads[-1] += seq
    joined = b"".join(bytes(r) for r in reads)
    offsets = np.zeros(len(reads) + 1, dtype=np.uint64)
    if reads:
        offsets[1:] = np.cumsum([len(r) for r in reads], dtype=np.uint64)
    return Parsed(np.frombuffer(joined, dtype=np.uint8).copy(), offsets, status, fmt, n_lines, n_bytes)


# ------------------------------------------------------------ minimizer orders

RANKS_KMC2, RANKS_LEX, RANKS_CGAT, RANKS_ROBERTS, RANKS_RANDOM, RANKS_DFP = 0, 1, 2, 3, 4, 5
NOT_CANONICAL = 0xFFFFFFFF
_BASES = "ACGT"
_MASK64 = (1 << 64) - 1
_GAMMA = 0x9E3779B97F4A7C15


def splitmix64(seed: int, i: int) -> int:
    """Output i (from 0) of the SplitMix64 generator seeded with `seed`
    (Steele, Lea and Flood, 2014): the state advances by the golden-ratio
    increment and each state value is passed through a fixed 64-bit mixer."""
    z = (seed + (i + 1) * _GAMMA) & _MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
    return z ^ (z >> 31)


def mmer_string(code: int, m: int) -> str:
    return "".join(_BASES[(code >> (2 * (m - 1 - i))) & 3] for i in range(m))


def revcomp(s: str) -> str:
    return s[::-1].translate(str.maketrans("ACGT", "TGCA"))


def canonical_codes(m: int) -> list:
    """Codes c of the m-mers that are their own canonical form (c <= rc(c))."""
    return [c for c in range(4 ** m) if mmer_string(c, m) <= revcomp(mmer_string(c, m))]


def mmer_frequencies(ascii: np.ndarray, offsets: np.ndarray, k: int, m: int, stride: int) -> dict:
    """Sampled minimizer frequencies for dfp: the canonical m-mer that starts
    each valid k-mer window whose global position is a multiple of `stride`."""
    freq = {}
    a = bytes(np.asarray(ascii, dtype=np.uint8))
    o = [int(x) for x in offsets]
    for r in range(len(o) - 1):
        read = a[o[r]:o[r + 1]].decode("latin-1")
        for i in range(len(read) - k + 1):
            p = o[r] + i
            if p % stride:
                continue
            win = read[i:i + k]
            if not all(ch in "ACGTacgt" for ch in win):
                continue
            u = win[:m].upper()
            c = min(u, revcomp(u))
            code = 0
            for ch in c:
                code = 4 * code + _BASES.index(ch)
            freq[code] = freq.get(code, 0) + 1
    return freq


def order_table(kind: int, m: int, seed: int = 0, pivot: float = 0.0, freq: Optional[dict] = None) -> np.ndarray:
    """Rank of every canonical m-mer code under one of the orders of Sec. 3.1
    (smaller rank = preferred minimizer); other codes get NOT_CANONICAL.

    KMC2 and LEX: as in the super-mer oracle. CGAT: lexicographic with
    C<G<A<T. ROBERTS: the bases at even positions (counting from 1) are
    complemented, then lexicographic with C<A<T<G. RANDOM: canonical codes
    sorted by the top 30 bits of SplitMix64 output number `code` (ties by
    code); the rank is the position. DFP: canonical codes sorted by sampled
    frequency (ties by code), then re-sorted by the distance of that position
    from the pivot position floor(pivot * M), M = number of canonical codes
    (ties: lower position first)."""
    table = np.full(4 ** m, NOT_CANONICAL, dtype=np.uint32)
    canon = canonical_codes(m)

    def lex_rank(s, alphabet):
        r = 0
        for ch in s:
            r = 4 * r + alphabet.index(ch)
        return r

    if kind in (RANKS_KMC2, RANKS_LEX, RANKS_CGAT, RANKS_ROBERTS):
        for c in canon:
            s = mmer_string(c, m)
            if kind == RANKS_LEX:
                r = c
            elif kind == RANKS_KMC2:
                r = c + (4 ** m if m >= 3 and s[:3] in ("AAA", "ACA") else 0)
            elif kind == RANKS_CGAT:
                r = lex_rank(s, "CGAT")
            else:
                t = "".join(revcomp(ch) if i % 2 == 1 else ch for i, ch in enumerate(s))
                r = lex_rank(t, "CATG")
            table[c] = r
        return table
    if kind == RANKS_RANDOM:
        order = sorted(canon, key=lambda c: (splitmix64(seed, c) >> 34, c))
        for pos, c in enumerate(order):
            table[c] = pos
        return table
    if kind == RANKS_DFP:
        freq = freq or {}
        by_freq = sorted(canon, key=lambda c: (freq.get(c, 0), c))
        M = len(canon)
        P = int(float(np.float32(pivot)) * M)   # the pivot is a 32-bit float on both sides
        by_dist = sorted(range(M), key=lambda pos: (abs(pos - P), pos))
        for rank, pos in enumerate(by_dist):
            table[by_freq[pos]] = rank
        return table
    raise ValueError(kind)

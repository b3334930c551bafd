"""Seeded synthetic reads for tests and benchmarks (no counting arithmetic here).

The C generator in ``synth.c`` draws genomes and reads from a counter-based
SplitMix64 stream, so a workload is a pure function of its parameters and seed.
This package is shared by the CPU oracle and the GPU path; it must never hold
any step of the counting method.

The named workloads stand in for the paper's real read sets (Tab. 1), which
are not available: uniform or GC-biased genomes with diverged repeat copies,
reads from both strands with substitution errors and undetermined bases.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field, replace
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB = os.path.join(_HERE, "libsynth.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile libsynth.so with gcc (host code only)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-pthread", _SRC, "-o", tmp, "-lm"],
                       check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        u64, f64, i32 = ctypes.c_uint64, ctypes.c_double, ctypes.c_int
        vp = ctypes.c_void_p
        lib.synth_genome.argtypes = [u64, f64, f64, f64, u64, vp]
        lib.synth_genome.restype = i32
        lib.synth_read_offsets.argtypes = [u64, f64, f64, u64, u64, u64, vp]
        lib.synth_read_offsets.restype = u64
        lib.synth_reads.argtypes = [vp, u64, vp, u64, f64, f64, u64, i32, vp]
        lib.synth_reads.restype = i32
        lib.synth_unit.argtypes = [u64, u64, u64]
        lib.synth_unit.restype = f64
        _lib = lib
    return _lib


def genome(G: int, gc: float = 0.5, rep_frac: float = 0.0, rep_div: float = 0.02, seed: int = 1) -> np.ndarray:
    """Uppercase ACGT genome of exactly ``G`` bases (uint8 ASCII)."""
    out = np.empty(G, dtype=np.uint8)
    rc = _load().synth_genome(G, gc, rep_frac, rep_div, seed, out.ctypes.data)
    if rc != 0:
        raise ValueError(f"synth_genome rejected G={G} gc={gc} rep_frac={rep_frac}")
    return out


def reads(gen: np.ndarray, n: int, median: float, sigma: float = 0.0, len_min: int = 0, len_max: int = 0,
          err: float = 0.01, p_n: float = 0.0005, seed: int = 1, threads: Optional[int] = None):
    """Sample ``n`` reads; returns (ascii uint8[n_bytes], offsets uint64[n+1])."""
    lib = _load()
    offsets = np.empty(n + 1, dtype=np.uint64)
    total = lib.synth_read_offsets(n, float(median), float(sigma), len_min, len_max, seed, offsets.ctypes.data)
    ascii_ = np.empty(int(total), dtype=np.uint8)
    if threads is None:
        threads = min(16, os.cpu_count() or 1)
    lib.synth_reads(gen.ctypes.data, gen.size, offsets.ctypes.data, n, err, p_n, seed, threads, ascii_.ctypes.data)
    return ascii_, offsets


def unit(seed: int, stream: int, idx: int) -> float:
    """Counter-based uniform draw in [0, 1) (same generator as the C side)."""
    return float(_load().synth_unit(seed, stream, idx))


@dataclass(frozen=True)
class Workload:
    """Parameters of one synthetic counting workload (genome, reads, k, m, bins, threshold)."""
    name: str
    G: int
    gc: float
    rep_frac: float
    read_median: float
    read_sigma: float
    len_min: int
    len_max: int
    coverage: float
    n_reads: int
    err: float
    p_n: float
    k: int
    m: int
    n_bins: int
    threshold: int
    seed: int
    skew_bins: bool = False
    note: str = ""

    def mean_read_len(self) -> float:
        if self.read_sigma <= 0:
            return self.read_median
        return self.read_median * math.exp(self.read_sigma ** 2 / 2)

    def scaled(self, factor: float, name: Optional[str] = None) -> "Workload":
        """Same shape with a genome (and read count) scaled by ``factor``."""
        G = max(20000, int(self.G * factor))
        n = max(1, int(math.ceil(self.coverage * G / self.mean_read_len()))) if self.coverage else \
            max(1, int(self.n_reads * factor))
        return replace(self, name=name or f"{self.name}@{factor:g}", G=G, n_reads=n)

    def bin_map(self) -> Optional[np.ndarray]:
        """Seeded minimizer -> bin map for the skewed-bins workload, else None.

        Bin weights are LogNormal(0, 0.97) (over 1024 bins the expected
        max/median weight is about 20); every m-mer code is given to a bin
        with probability proportional to its weight, so bin sizes follow the
        weights. Only the m-mer code space is used here, no m-mer arithmetic.
        """
        if not self.skew_bins:
            return None
        rng = np.random.default_rng(self.seed)
        nb, n_codes = self.n_bins, 4 ** self.m
        weights = np.exp(rng.normal(0.0, 0.97, nb))
        cdf = np.cumsum(weights / weights.sum())
        return np.searchsorted(cdf, rng.random(n_codes), side="right").clip(0, nb - 1).astype(np.uint32)

    def generate(self, threads: Optional[int] = None):
        """(ascii, offsets) for this workload."""
        g = genome(self.G, self.gc, self.rep_frac, 0.02, self.seed)
        return reads(g, self.n_reads, self.read_median, self.read_sigma, self.len_min, self.len_max,
                     self.err, self.p_n, self.seed, threads)


def _cov_reads(cov: float, G: int, mean_len: float) -> int:
    return int(math.ceil(cov * G / mean_len))


# The five workloads. Readings where the workload text is silent:
#  * c3 uses m = 9 and the error / N rates of c2 ("as above");
#  * c4 keeps k = 200 (seven 64-bit words: six full words and an 8-base tail);
#    its read lengths are LogNormal(median 2000, sigma 0.5) resampled into
#    [500, 10000];
#  * c3's bin skew is realised by a seeded minimizer -> bin map (skew_bins).
CONFIGS = {
    "c1_tiny": Workload("c1_tiny", G=1_000_000, gc=0.5, rep_frac=0.0, read_median=100, read_sigma=0.0,
                        len_min=0, len_max=0, coverage=0.0, n_reads=100_000, err=0.01, p_n=0.0005,
                        k=32, m=7, n_bins=64, threshold=2, seed=1,
                        note="1 Mbp uniform genome, 100k x 100 bp reads, k=32, m=7, 64 bins, t=2"),
    "c2_k65": Workload("c2_k65", G=100_000_000, gc=0.41, rep_frac=0.05, read_median=150, read_sigma=0.0,
                       len_min=0, len_max=0, coverage=30.0, n_reads=_cov_reads(30, 100_000_000, 150),
                       err=0.01, p_n=0.0005, k=65, m=9, n_bins=512, threshold=2, seed=2,
                       note="100 Mbp GC41% 5% repeats, 30x 150 bp, k=65, m=9, 512 bins, t=2"),
    "c3_skew": Workload("c3_skew", G=500_000_000, gc=0.41, rep_frac=0.15, read_median=250, read_sigma=0.0,
                        len_min=0, len_max=0, coverage=20.0, n_reads=_cov_reads(20, 500_000_000, 250),
                        err=0.01, p_n=0.0005, k=99, m=9, n_bins=1024, threshold=3, seed=3, skew_bins=True,
                        note="500 Mbp 15% repeats, 20x 250 bp, k=99, m=9, 1024 skewed bins, t=3"),
    "c4_longk": Workload("c4_longk", G=300_000_000, gc=0.41, rep_frac=0.05, read_median=2000, read_sigma=0.5,
                         len_min=500, len_max=10000, coverage=10.0,
                         n_reads=_cov_reads(10, 300_000_000, 2000 * math.exp(0.125)),
                         err=0.02, p_n=0.001, k=200, m=11, n_bins=2048, threshold=2, seed=4,
                         note="300 Mbp, 10x log-normal reads (median 2 kbp), k=200, m=11, 2048 bins, t=2"),
}

# Serving workload: a Poisson stream of independent jobs (seed 5; job j uses
# seed (5 << 32) | j). Each job: G ~ U[1, 50] Mbp, coverage ~ U[10, 40] of
# 150 bp reads, 1% errors, 0.05% N, GC 41% with 5% repeats, k ~ U{32, 55, 99},
# m = 7 for k = 32 and 9 otherwise, 256 bins, t = 2.
SERVING_SEED = 5
SERVING_RATE = 20.0  # jobs per second


def serving_job(j: int, scale: float = 1.0) -> Workload:
    """Parameters of serving job ``j`` (genome size scaled by ``scale``)."""
    s = (SERVING_SEED << 32) | j
    G = int((1_000_000 + unit(s, 100, 0) * 49_000_000) * scale)
    G = max(20000, G)
    cov = 10.0 + unit(s, 100, 1) * 30.0
    k = (32, 55, 99)[min(2, int(unit(s, 100, 2) * 3))]
    m = 7 if k == 32 else 9
    return Workload(f"job{j}", G=G, gc=0.41, rep_frac=0.05, read_median=150, read_sigma=0.0, len_min=0,
                    len_max=0, coverage=cov, n_reads=_cov_reads(cov, G, 150), err=0.01, p_n=0.0005,
                    k=k, m=m, n_bins=256, threshold=2, seed=s)


def arrival_times(n_jobs: int, rate: float = SERVING_RATE) -> np.ndarray:
    """Poisson arrival times (seconds) of the serving stream."""
    gaps = [-math.log(1.0 - unit(SERVING_SEED, 101, j)) / rate for j in range(n_jobs)]
    return np.cumsum(np.array(gaps))


# ------------------------------------------------------------ text renderings

def to_fastq(ascii: np.ndarray, offsets: np.ndarray, seed: int = 1, crlf: bool = False) -> bytes:
    """The reads as FASTQ text: Illumina-like header, sequence, '+', and a
    random quality string over '!'..'J' (which includes '@', '>' and '+', so
    a parser cannot take a line's first byte for its kind)."""
    rng = np.random.default_rng(seed)
    a = np.ascontiguousarray(ascii, dtype=np.uint8).tobytes()
    o = np.asarray(offsets, dtype=np.int64)
    n = o.size - 1
    qual = rng.integers(33, 75, size=int(o[-1]) if n else 0, dtype=np.uint8).tobytes()
    nl = b"\r\n" if crlf else b"\n"
    parts = []
    for r in range(n):
        s, e = int(o[r]), int(o[r + 1])
        parts.append(b"@SYN.%d %d/1 length=%d" % (r, r * 7 + 3, e - s) + nl + a[s:e] + nl + b"+" + nl + qual[s:e] + nl)
    return b"".join(parts)


def to_fasta(ascii: np.ndarray, offsets: np.ndarray, width: int = 60, crlf: bool = False,
             blank_lines: bool = False) -> bytes:
    """The reads as multi-line FASTA text, sequence lines of `width` bytes
    (0: one line per read); blank_lines adds an empty line after each record."""
    a = np.ascontiguousarray(ascii, dtype=np.uint8).tobytes()
    o = np.asarray(offsets, dtype=np.int64)
    nl = b"\r\n" if crlf else b"\n"
    parts = []
    for r in range(o.size - 1):
        s, e = int(o[r]), int(o[r + 1])
        parts.append(b">syn_%d some description" % r + nl)
        step = width if width > 0 else max(1, e - s)
        for x in range(s, e, step):
            parts.append(a[x:min(e, x + step)] + nl)
        if blank_lines:
            parts.append(nl)
    return b"".join(parts)

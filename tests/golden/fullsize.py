"""Oracle results of the named workloads at their full sizes, stored as
digests (written by the oracle only; read by the full-size parity tests).

A workload of billions of windows is far too large for the oracle to count
inside a test, and its (k-mer, count) pairs are gigabytes. So this script
counts it once, offline, with ``oracle.count_sharded`` (the oracle's plain
sort-and-count, split into hash shards to bound memory) and stores, per
workload, a small text file ``fullsize_<name>.txt`` holding:

* a fingerprint of the generated reads (so a changed generator is caught
  before any comparison);
* n_valid, the number of distinct keys, the number of pairs, the largest
  count;
* every non-zero entry of the count-of-counts histogram over all distinct
  keys (folded at 65535, the last bucket holding every larger count);
* for each shard ``s`` (``oracle.shard_of(key) == s``): its number of pairs
  and the SHA-256 of its pairs in ascending key order, keys as ``[n, W]``
  little-endian uint64 followed by counts as little-endian uint32.

Usage (CPU only; calls ``oracle`` and ``synth``, nothing else)::

    python tests/golden/fullsize.py c2_k65 [--threads 7] [--shards 16] [--group 8]
    python tests/golden/fullsize.py job199 ...      # serving job 199 at scale 1.0

Nothing here is used by the library; only tests import ``read`` and the
digest helpers.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
HIST_LEN = 65536
CHUNK = 256 << 20


def golden_path(name: str) -> str:
    return os.path.join(HERE, f"fullsize_{name}.txt")


def workload(name: str):
    """The named workload (``c2_k65`` ... or ``job<j>``: serving job j at scale 1)."""
    import synth
    if name.startswith("job"):
        return synth.serving_job(int(name[3:]), scale=1.0)
    return synth.CONFIGS[name]


def input_fingerprint(ascii: np.ndarray, offsets: np.ndarray, threads: int = 16) -> str:
    """SHA-256 over the SHA-256 digests of 256 MiB chunks of the reads' bytes,
    then of the offsets (chunks hashed in parallel)."""
    bufs = []
    for arr in (np.ascontiguousarray(ascii).view(np.uint8).reshape(-1),
                np.ascontiguousarray(offsets).view(np.uint8).reshape(-1)):
        bufs.extend(memoryview(arr[i: i + CHUNK]) for i in range(0, arr.size, CHUNK))

    def one(b):
        return hashlib.sha256(b).digest()

    with cf.ThreadPoolExecutor(threads) as ex:
        parts = list(ex.map(one, bufs))
    return hashlib.sha256(b"".join(parts)).hexdigest()


def pairs_digest(keys: np.ndarray, counts: np.ndarray) -> str:
    """SHA-256 of pairs in ascending key order (keys [n, W] uint64, counts uint32)."""
    h = hashlib.sha256()
    h.update(memoryview(np.ascontiguousarray(keys, dtype="<u8")).cast("B"))
    h.update(memoryview(np.ascontiguousarray(counts, dtype="<u4")).cast("B"))
    return h.hexdigest()


def write(name: str, threads: int, shards: int, group: int, sort_workers: int) -> str:
    sys.path.insert(0, ROOT)
    import oracle
    w = workload(name)
    t0 = time.time()
    a, o = w.generate(threads=threads)
    fp = input_fingerprint(a, o, threads)
    print(f"[{name}] {a.size / 1e9:.2f} GB of reads, fingerprint {fp[:16]} ({time.time() - t0:.0f} s)", flush=True)
    hist = np.zeros(HIST_LEN, dtype=np.uint64)
    rows = {}
    totals = {"n_distinct": 0, "n_pairs": 0, "max_count": 0}

    def on_shard(s, r):
        n = min(r.hist.size, HIST_LEN - 1)
        hist[:n] += r.hist[:n]
        if r.hist.size > HIST_LEN - 1:
            hist[HIST_LEN - 1] += r.hist[HIST_LEN - 1:].sum()
        totals["n_distinct"] += r.n_distinct
        totals["n_pairs"] += r.keys.shape[0]
        totals["max_count"] = max(totals["max_count"], r.hist.size - 1)
        rows[s] = (r.keys.shape[0], r.n_distinct, pairs_digest(r.keys, r.counts))
        print(f"[{name}] shard {s}/{shards}: {r.n_valid_shard} windows, {r.n_distinct} distinct, "
              f"{r.keys.shape[0]} pairs ({time.time() - t0:.0f} s)", flush=True)

    n_valid = oracle.count_sharded(a, o, w.k, w.threshold, shards, on_shard, canonical=True, group=group,
                                   threads=threads, sort_workers=sort_workers)
    hist[0] = 0
    assert int((np.arange(HIST_LEN, dtype=np.float64) * hist.astype(np.float64)).sum()) == n_valid or \
        hist[HIST_LEN - 1] > 0
    path = golden_path(name)
    with open(path, "w") as f:
        f.write(f"# Oracle result of workload {name} at full size: {w.note or w.name}\n")
        f.write(f"# written by tests/golden/fullsize.py with oracle.count_sharded ({shards} shards); "
                f"{time.time() - t0:.0f} s on {threads} threads\n")
        f.write(f"name {name}\nseed {w.seed}\nk {w.k}\nm {w.m}\nn_bins {w.n_bins}\nthreshold {w.threshold}\n")
        f.write(f"canonical 1\nreads {o.size - 1}\nbytes {a.size}\ninput {fp}\n")
        f.write(f"n_valid {n_valid}\nn_distinct {totals['n_distinct']}\nn_pairs {totals['n_pairs']}\n")
        f.write(f"max_count {totals['max_count']}\nshard_mod {shards}\nhist_len {HIST_LEN}\n")
        for s in range(shards):
            n, d, dig = rows[s]
            f.write(f"shard {s} {n} {d} {dig}\n")
        for c in np.nonzero(hist)[0]:
            f.write(f"hist {int(c)} {int(hist[c])}\n")
    print(f"[{name}] wrote {path} ({time.time() - t0:.0f} s)", flush=True)
    return path


class Golden:
    """Parsed ``fullsize_<name>.txt``."""

    def __init__(self, path: str):
        self.fields = {}
        self.shards = []      # (n_pairs, n_distinct, digest) per shard
        hist = {}
        with open(path) as f:
            for ln in f:
                if not ln.strip() or ln.startswith("#"):
                    continue
                p = ln.split()
                if p[0] == "shard":
                    assert int(p[1]) == len(self.shards)
                    self.shards.append((int(p[2]), int(p[3]), p[4]))
                elif p[0] == "hist":
                    hist[int(p[1])] = int(p[2])
                else:
                    self.fields[p[0]] = p[1]
        self.hist = np.zeros(int(self.fields["hist_len"]), dtype=np.uint64)
        for c, v in hist.items():
            self.hist[c] = v
        assert len(self.shards) == self.int("shard_mod")

    def int(self, key: str) -> int:
        return int(self.fields[key])


def read(name: str) -> Golden:
    return Golden(golden_path(name))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("names", nargs="+")
    ap.add_argument("--threads", type=int, default=7)
    ap.add_argument("--shards", type=int, default=16)
    ap.add_argument("--group", type=int, default=0, help="shards held in memory per pass (0: all)")
    ap.add_argument("--sort-workers", type=int, default=2)
    args = ap.parse_args()
    for name in args.names:
        write(name, args.threads, args.shards, args.group, args.sort_workers)


if __name__ == "__main__":
    main()

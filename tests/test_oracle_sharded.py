"""The oracle's sharded driver and the stored full-size results.

``oracle.count_sharded`` splits the plain sort-and-count into hash shards and
read ranges so that workloads of billions of windows fit in memory. These
tests pin it to ``oracle.count`` (itself pinned by brute force, closed forms
and invariants) and check that every stored golden file is consistent with
itself and, for the small workload, with a direct count.
"""
import collections
import glob
import os
import sys

import numpy as np
import pytest

import oracle
import synth

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import fullsize  # noqa: E402
from gpu_util import random_reads, reads_to_csr  # noqa: E402


def _join(parts, k):
    keys = np.concatenate([p.keys for p in parts])
    counts = np.concatenate([p.counts for p in parts])
    order = np.lexsort(keys.T[::-1]) if keys.shape[0] else np.zeros(0, np.int64)
    return keys[order], counts[order]


@pytest.mark.parametrize("k,canonical", [(5, True), (31, True), (33, False), (65, True), (99, True)])
@pytest.mark.parametrize("shards,group,threads", [(1, 0, 1), (5, 2, 3), (7, 0, 4), (3, 1, 16)])
def test_sharded_equals_plain(k, canonical, shards, group, threads):
    rng = np.random.default_rng(k * 100 + shards)
    a, o = reads_to_csr(random_reads(rng, 150, 0, 260, n_rate=0.01))
    full = oracle.count(a, o, k, threshold=2, canonical=canonical)
    got = {}
    nv = oracle.count_sharded(a, o, k, 2, shards, lambda s, r: got.__setitem__(s, r), canonical=canonical,
                              group=group, threads=threads)
    assert sorted(got) == list(range(shards))
    assert nv == full.n_valid
    keys, counts = _join([got[s] for s in range(shards)], k)
    assert np.array_equal(keys, full.keys) and np.array_equal(counts, full.counts)
    hist = np.zeros(full.hist.size + 1, dtype=np.uint64)
    for r in got.values():
        hist[: r.hist.size] += r.hist
    assert np.array_equal(hist[: full.hist.size], full.hist) and hist[full.hist.size:].sum() == 0
    assert sum(r.n_valid_shard for r in got.values()) == full.n_valid
    assert sum(r.n_distinct for r in got.values()) == full.n_distinct
    if full.keys.shape[0]:
        sh = oracle.shard_of(full.keys, k, shards)
        for s in range(shards):
            assert np.array_equal(got[s].keys, full.keys[sh == s])


def test_count_multiset_by_brute_force():
    rng = np.random.default_rng(3)
    for W in (1, 2, 4):
        keys = rng.integers(0, 6, size=(500, W)).astype(np.uint64) * np.uint64(0x9E3779B97F4A7C15)
        tally = collections.Counter(tuple(int(x) for x in row) for row in keys)
        k = 32 * W
        r = oracle.count_multiset(np.ascontiguousarray(keys), k, threshold=3)
        want = sorted((key, c) for key, c in tally.items() if c >= 3)
        assert [tuple(int(x) for x in row) for row in r.keys] == [key for key, _ in want]
        assert r.counts.tolist() == [c for _, c in want]
        hist = collections.Counter(tally.values())
        assert r.hist.tolist() == [hist.get(c, 0) for c in range(max(tally.values()) + 1)]
        assert r.n_distinct == len(tally)


def test_shard_of_vectorised_equals_scalar():
    rng = np.random.default_rng(5)
    for k in (20, 64, 200):
        W = (k + 31) // 32
        keys = rng.integers(0, 2 ** 63, size=(3000, W), dtype=np.int64).astype(np.uint64)
        many = oracle.shard_of(keys, k, 13)
        lib = oracle._load()
        one = [lib.oracle_shard_of(np.ascontiguousarray(keys[i]).ctypes.data, W, 13) for i in range(0, 3000, 97)]
        assert many[::97].tolist() == one


def test_small_golden_equals_direct_count():
    gold = fullsize.read("c1_tiny")
    w = synth.CONFIGS["c1_tiny"]
    a, o = w.generate()
    assert fullsize.input_fingerprint(a, o) == gold.fields["input"]
    ref = oracle.count(a, o, w.k, threshold=w.threshold)
    assert gold.int("n_valid") == ref.n_valid and gold.int("n_distinct") == ref.n_distinct
    assert np.array_equal(gold.hist, ref.folded_hist(gold.hist.size))
    sh = oracle.shard_of(ref.keys, w.k, gold.int("shard_mod"))
    for s, (n, _, dig) in enumerate(gold.shards):
        assert n == int((sh == s).sum())
        assert dig == fullsize.pairs_digest(ref.keys[sh == s], ref.counts[sh == s])


@pytest.mark.parametrize("path", sorted(glob.glob(os.path.join(HERE, "golden", "fullsize_*.txt"))),
                         ids=os.path.basename)
def test_golden_files_are_consistent(path):
    gold = fullsize.Golden(path)
    h = gold.hist.astype(np.float64)
    c = np.arange(h.size, dtype=np.float64)
    t = gold.int("threshold")
    if gold.int("max_count") < h.size - 1:
        assert int((c * h).sum()) == gold.int("n_valid"), "sum of c * h[c] must be the valid windows"
    assert int(h.sum()) == gold.int("n_distinct")
    assert int(h[t:].sum()) == gold.int("n_pairs")
    assert sum(n for n, _, _ in gold.shards) == gold.int("n_pairs")
    assert sum(d for _, d, _ in gold.shards) == gold.int("n_distinct")
    name = gold.fields["name"]
    w = fullsize.workload(name)
    assert (gold.int("k"), gold.int("threshold"), gold.int("seed")) == (w.k, w.threshold, w.seed)
    assert gold.int("reads") == w.n_reads

"""The `-d` mode (App. A): k-mers counted as read, without reverse-complement
normalisation, against the oracle's non-canonical count, element by element.

A k-mer and its reverse complement are then two keys, so the key that is all
T's (at k = 32) and keys whose first word is 32 T's (k >= 64), which a
canonical count never or rarely meets, occur here. The all-ones word marks an
empty table slot, so in this mode a key's first word is stored XORed with a
fixed constant: poly-T keys are counted in the tables, and the keys that start
with the one 32-mer the XOR maps onto the marker take the emergency area.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import random_reads, reads_to_csr
from paper_1607_06618_amd import gerbil as g

pytestmark = pytest.mark.gpu

TABLES = [pytest.param(g.GERBIL_TABLE_LDS, id="lds"), pytest.param(g.GERBIL_TABLE_HBM, id="hbm")]
MODES = [pytest.param(g.GERBIL_PLAIN, id="plain"), pytest.param(g.GERBIL_BATCHED, id="batched")]


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    g.load()


def compare_d(a, o, k, m, n_bins, t, hist_len=256, expect_overflow=None, **kw):
    res = g.count_kmers(a, o, k, m, n_bins, t, hist_len, canonical=False, **kw)
    ref = oracle.count(a, o, k, threshold=t, canonical=False)
    keys, counts = res.sorted()
    assert res.report.n_valid == ref.n_valid
    assert keys.shape == ref.keys.shape, (keys.shape, ref.keys.shape)
    assert np.array_equal(keys, ref.keys)
    assert np.array_equal(counts, ref.counts)
    assert np.array_equal(res.hist, ref.folded_hist(hist_len))
    if expect_overflow is True:
        assert res.report.n_overflow > 0
    return res, ref


def genome_reads(rng, k, n=400, glen=3000):
    gen = "".join(np.array(list("ACGT"))[rng.integers(0, 4, glen)].tolist())
    reads = []
    for _ in range(n):
        L = int(rng.integers(max(1, k - 5), k + 150))
        s = int(rng.integers(0, len(gen) - L))
        r = gen[s: s + L]
        if rng.random() < 0.5:
            r = r[::-1].translate(str.maketrans("ACGT", "TGCA"))
        reads.append("".join(c if rng.random() > 0.003 else "N" for c in r))
    return reads + random_reads(rng, 30, 0, 300)


@pytest.mark.parametrize("k,t", [(2, 1), (16, 2), (31, 1), (32, 1), (33, 2), (64, 1), (65, 2), (99, 1), (128, 2),
                                 (200, 1), (256, 2)])
@pytest.mark.parametrize("table", TABLES)
@pytest.mark.parametrize("mode", MODES)
def test_noncanonical_parity_random(k, t, table, mode):
    rng = np.random.default_rng(5000 + k)
    a, o = reads_to_csr(genome_reads(rng, k))
    compare_d(a, o, k, min(9, k - 1), 37, t, hist_len=64, table=table, mode=mode)


# the 32-mer whose first word, XORed with the stored-key constant of the
# `-d` mode (0x9E3779B97F4A7C15), is the all-ones empty-slot marker
MARKER_32MER = oracle.decode_key(np.array([~np.uint64(0x9E3779B97F4A7C15)], dtype=np.uint64), 32)


@pytest.mark.parametrize("k", [32, 64, 96])
@pytest.mark.parametrize("table", TABLES)
@pytest.mark.parametrize("mode", MODES)
def test_all_t_keys_are_counted_in_the_tables(k, table, mode):
    reads = ["T" * 300, "A" * 300, "T" * 40 + "ACGGT" * 30, "CA" + "T" * 120] * 10 + ["ACGTTGCA" * 30] * 5
    a, o = reads_to_csr(reads)
    res, ref = compare_d(a, o, k, 9, 8, 1, table=table, mode=mode)
    assert res.report.n_overflow == 0
    # the all-T k-mer and the all-A k-mer are two keys here
    words = g.words(k)
    all_t = [(1 << 64) - 1] * (words - 1) + [(1 << (2 * (k - 32 * (words - 1)))) - 1]
    hit = np.nonzero((res.sorted()[0] == np.array(all_t, dtype=np.uint64)).all(axis=1))[0]
    assert hit.size == 1
    assert int(res.sorted()[1][hit[0]]) == 10 * (300 - k + 1) + 10 * (120 - k + 1) + 10 * max(0, 40 - k + 1)


@pytest.mark.parametrize("k", [32, 64, 96])
@pytest.mark.parametrize("table", TABLES)
@pytest.mark.parametrize("mode", MODES)
def test_keys_stored_as_the_marker_take_the_emergency_area(k, table, mode):
    assert len(MARKER_32MER) == 32 and set(MARKER_32MER) <= set("ACGT")
    rng = np.random.default_rng(77 + k)
    tail = lambda n: "".join(np.array(list("ACGT"))[rng.integers(0, 4, n)].tolist())
    reads = ([MARKER_32MER + tail(150), tail(7) + MARKER_32MER + tail(120), MARKER_32MER * 3 + tail(40)] * 6
             + [tail(200) for _ in range(20)])
    a, o = reads_to_csr(reads)
    res, ref = compare_d(a, o, k, 9, 8, 1, expect_overflow=True, table=table, mode=mode)
    keys = res.sorted()[0]
    first = np.array([oracle.decode_key(kk, k)[:32] for kk in keys])
    assert (first == MARKER_32MER).sum() >= (1 if k == 32 else 3)   # at k = 32 the marker 32-mer is one key


@pytest.mark.parametrize("mode", MODES)
def test_noncanonical_counts_fold_to_the_canonical_counts(mode):
    """Every canonical count is the sum of the `-d` counts of a k-mer and its
    reverse complement (each palindrome counted once)."""
    w = synth.CONFIGS["c1_tiny"].scaled(0.02)
    a, o = w.generate()
    d = g.count_kmers(a, o, w.k, w.m, w.n_bins, 1, 256, canonical=False, mode=mode)
    c = g.count_kmers(a, o, w.k, w.m, w.n_bins, 1, 256, mode=mode)
    assert d.report.n_valid == c.report.n_valid
    folded = {}
    for key, cnt in zip(map(tuple, d.keys.tolist()), d.counts.tolist()):
        s = oracle.decode_key(np.array(key, dtype=np.uint64), w.k)
        r = s[::-1].translate(str.maketrans("ACGT", "TGCA"))
        cs = min(s, r)
        folded[cs] = folded.get(cs, 0) + cnt
    canon = {oracle.decode_key(key, w.k): int(cnt) for key, cnt in zip(c.keys, c.counts)}
    assert folded == canon


@pytest.mark.parametrize("name,scale", [("c2_k65", 0.01), ("c4_longk", 0.002)])
@pytest.mark.parametrize("mode", MODES)
def test_noncanonical_config_shapes(name, scale, mode):
    w = synth.CONFIGS[name].scaled(scale)
    a, o = w.generate()
    compare_d(a, o, w.k, w.m, w.n_bins, w.threshold, hist_len=1024, mode=mode)

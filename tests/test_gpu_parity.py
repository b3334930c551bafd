"""GPU path vs the CPU oracle, element by element, through the C ABI.

Integer work, so the bar is bit-exact: packed words and validity bitmaps,
super-mer pieces per bin, (k-mer, count) pairs and the count-of-counts
histogram. Pair order is unspecified, so pairs are compared after sorting.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import (bin_arrays, encoded_arrays, make_job, random_reads, reads_to_csr, to_device)
from conftest import read_golden
from paper_1607_06618_amd import gerbil as g

pytestmark = pytest.mark.gpu

TABLES = [pytest.param(g.GERBIL_TABLE_LDS, id="lds"), pytest.param(g.GERBIL_TABLE_HBM, id="hbm")]


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    g.load()


def run_and_compare(a, o, k, m, n_bins, t, hist_len=256, expect_overflow=None, **kw):
    res = g.count_kmers(a, o, k, m, n_bins, t, hist_len, **kw)
    ref = oracle.count(a, o, k, threshold=t)
    keys, counts = res.sorted()
    assert res.report.n_valid == ref.n_valid
    assert keys.shape == ref.keys.shape, (keys.shape, ref.keys.shape)
    assert np.array_equal(keys, ref.keys)
    assert np.array_equal(counts, ref.counts)
    assert np.array_equal(res.hist, ref.folded_hist(hist_len))
    assert res.report.max_count == (ref.hist.size - 1 if ref.hist.size > 1 else 0)
    if expect_overflow is True:
        assert res.report.n_overflow > 0
    if expect_overflow is False:
        assert res.report.n_overflow == 0
    return res, ref


# ----------------------------------------------------------------- encode

@pytest.mark.parametrize("k", [2, 3, 8, 31, 32, 33, 63, 64, 65, 99, 128, 200, 256])
def test_encode_parity(k):
    rng = np.random.default_rng(100 + k)
    reads = random_reads(rng, 300, 0, 400) + ["", "A", "ACGT" * 70, "N" * 50, "acgtn" * 20]
    a, o = reads_to_csr(reads)
    job = make_job(a, o, k, m=min(7, k - 1))
    job.encode()
    packed, ok = encoded_arrays(job)
    ref_packed, ref_ok, nv = oracle.encode(a, o, k)
    assert np.array_equal(packed, ref_packed)
    assert np.array_equal(ok, ref_ok)
    st, rep = g.gerbil_result(job.enc, None, None)
    assert st == g.GERBIL_OK and rep.n_valid == nv


def test_encode_unaligned_input_and_ragged_tail():
    import torch
    rng = np.random.default_rng(7)
    reads = random_reads(rng, 97, 1, 333)
    a, o = reads_to_csr(reads)
    for shift in (1, 3, 8, 13):
        big = torch.zeros(a.size + 64, dtype=torch.uint8, device="cuda")
        big[shift: shift + a.size] = torch.from_numpy(a).cuda()
        _, od = to_device(a, o)
        p = g.make_params(31, 7, 8, 1)
        job = g.Job(big[shift: shift + a.size], od, a.size, p)
        job.encode()
        packed, ok = encoded_arrays(job)
        ref_packed, ref_ok, nv = oracle.encode(a, o, 31)
        assert np.array_equal(packed, ref_packed) and np.array_equal(ok, ref_ok)


def test_encode_reports_inconsistent_offsets():
    a, o = reads_to_csr(["ACGTACGTAC", "GGGTTTAAAC"])
    ad, od = to_device(a, o)
    job = g.Job(ad, od, a.size - 3, g.make_params(5, 3, 4, 1))
    job.encode()
    st, rep = g.gerbil_result(job.enc, None, None)
    assert st == g.GERBIL_EINVAL and rep.status & g.ST_OFFSETS


# ------------------------------------------------------------------- bins

def gpu_pieces(job):
    desc, off, km = bin_arrays(job)
    out = []
    for b in range(job.bins.n_bins):
        for d in desc[int(off[b]): int(off[b + 1])]:
            out.append((int(d) >> 24, int(d) & 0xFFFFFF, b))
    return sorted(out), km


def oracle_pieces(a, o, k, m, nb, order, tile, bin_map=None):
    sm = oracle.supermers(a, o, k, m, nb, order, bin_map)
    out = []
    for s, n, b in zip(sm["start"].tolist(), sm["n_kmers"].tolist(), sm["bin"].tolist()):
        pos, end = s, s + n
        while pos < end:
            cut = min(end, (pos // tile + 1) * tile)
            out.append((pos, cut - pos, b))
            pos = cut
    return sorted(out)


@pytest.mark.parametrize("k,m,nb,order", [(15, 5, 7, 0), (32, 7, 64, 0), (33, 9, 17, 1), (65, 9, 512, 0),
                                          (99, 9, 33, 0), (200, 11, 2048, 0), (4, 3, 4, 1), (21, 15, 4096, 1),
                                          # windows of w = k - m + 1 = 19, 27, 256 and 257 ranks: the shortest
                                          # and a ragged window read through 9-rank block minima, the longest
                                          # window of the short-window kernel, the shortest of the long one
                                          (27, 9, 16, 1), (35, 9, 32, 0), (264, 9, 64, 0), (265, 9, 64, 0)])
def test_bin_parity(k, m, nb, order):
    rng = np.random.default_rng(k * 31 + m)
    reads = random_reads(rng, 150, 0, 600, n_rate=0.005, junk="N") + ["ACGT" * 600, "A" * 3000]
    a, o = reads_to_csr(reads)
    job = make_job(a, o, k, m=m, n_bins=nb, order=order)
    job.encode()
    job.bin()
    st, rep = g.gerbil_result(job.enc, job.bins, None)
    assert st == g.GERBIL_OK
    got, km = gpu_pieces(job)
    want = oracle_pieces(a, o, k, m, nb, order, job.bins.tile)
    assert got == want
    per_bin = np.zeros(nb, dtype=np.int64)
    for _, n, b in want:
        per_bin[b] += n
    assert np.array_equal(km.astype(np.int64), per_bin)
    assert int(km.sum()) == rep.n_valid


def test_bin_map_is_applied():
    rng = np.random.default_rng(3)
    reads = random_reads(rng, 100, 50, 300, n_rate=0.0)
    a, o = reads_to_csr(reads)
    k, m, nb = 25, 6, 13
    bmap = rng.integers(0, nb, 4 ** m).astype(np.uint32)
    import torch
    bmap_d = torch.from_numpy(bmap.view(np.int32)).cuda()
    job = make_job(a, o, k, m=m, n_bins=nb, bin_map_ptr=bmap_d.data_ptr())
    job.encode()
    job.bin()
    got, _ = gpu_pieces(job)
    assert got == oracle_pieces(a, o, k, m, nb, 0, job.bins.tile, bmap)


@pytest.mark.parametrize("order", [g.GERBIL_ORDER_LEX, g.GERBIL_ORDER_KMC2])
def test_fig1_supermers_on_gpu(order):
    lines = dict(ln.split(None, 1) for ln in read_golden("fig1_supermers.txt"))
    seq, k, m, expect = lines["sequence"], int(lines["k"]), int(lines["m"]), lines["supermers"].split()
    a, o = reads_to_csr([seq])
    job = make_job(a, o, k, m=m, n_bins=4, order=order)
    job.encode()
    job.bin()
    got, _ = gpu_pieces(job)
    assert [seq[s: s + n + k - 1] for s, n, _ in got] == expect


# ------------------------------------------------------------------ count

@pytest.mark.parametrize("k,t", [(2, 1), (5, 1), (16, 2), (31, 1), (32, 2), (33, 1), (55, 2), (63, 1), (64, 2),
                                 (65, 2), (96, 1), (99, 3), (128, 2), (160, 1), (200, 2), (256, 1)])
@pytest.mark.parametrize("table", TABLES)
def test_count_parity_random(k, t, table):
    rng = np.random.default_rng(1000 + k)
    # a small genome sampled with errors gives repeated k-mers at every k
    gen = "".join(np.array(list("ACGT"))[rng.integers(0, 4, 3000)].tolist())
    reads = []
    for _ in range(400):
        L = int(rng.integers(max(1, k - 5), k + 150))
        s = int(rng.integers(0, len(gen) - L))
        r = gen[s: s + L]
        if rng.random() < 0.5:
            r = r[::-1].translate(str.maketrans("ACGT", "TGCA"))
        r = "".join(c if rng.random() > 0.003 else "N" for c in r)
        reads.append(r)
    reads += random_reads(rng, 30, 0, 300)
    a, o = reads_to_csr(reads)
    m = min(9, k - 1)
    run_and_compare(a, o, k, m, 37, t, hist_len=64, table=table)


@pytest.mark.parametrize("table", TABLES)
def test_count_parity_c1_full(table):
    w = synth.CONFIGS["c1_tiny"]
    a, o = w.generate()
    res, ref = run_and_compare(a, o, w.k, w.m, w.n_bins, w.threshold, hist_len=512, expect_overflow=False,
                               table=table)
    assert ref.n_valid > 6_000_000


@pytest.mark.parametrize("name,scale", [("c2_k65", 0.01), ("c3_skew", 0.001), ("c4_longk", 0.002)])
@pytest.mark.parametrize("table", TABLES)
def test_count_parity_config_shapes(name, scale, table):
    w = synth.CONFIGS[name].scaled(scale)
    a, o = w.generate()
    run_and_compare(a, o, w.k, w.m, w.n_bins, w.threshold, hist_len=1024, table=table)


@pytest.mark.parametrize("k", [31, 65, 99])
@pytest.mark.parametrize("table", TABLES)
def test_overflow_path_is_exact(k, table):
    w = synth.CONFIGS["c1_tiny"].scaled(0.05)
    a, o = w.generate()
    run_and_compare(a, o, k, 9, 8, 1, max_probes=1, load_factor=0.95, expect_overflow=True, table=table)


@pytest.mark.parametrize("table", TABLES)
def test_keys_with_all_t_first_word_take_the_emergency_path(table):
    k = 65
    reads = ["T" * 32 + "A" * 40, "T" * 33 + "A" * 33 + "C", "GG" + "T" * 32 + "A" * 35] * 20
    reads += ["ACGTTGCA" * 30] * 5
    a, o = reads_to_csr(reads)
    run_and_compare(a, o, k, 9, 4, 1, expect_overflow=True, table=table)


@pytest.mark.parametrize("table", TABLES)
def test_single_key_contention(table):
    L = 260
    reads = ["A" * L] * 3000 + ["T" * L] * 3000
    a, o = reads_to_csr(reads)
    for k in (32, 65, 200):
        res, ref = run_and_compare(a, o, k, 9, 16, 2, table=table)
        assert res.counts.tolist() == [6000 * (L - k + 1)]


def test_output_capacity_error_then_retry():
    w = synth.CONFIGS["c1_tiny"].scaled(0.05)
    a, o = w.generate()
    ad, od = to_device(a, o)
    p = g.make_params(32, 7, 16, 1)
    job = g.Job(ad, od, a.size, p, cap=1000)
    job.run()
    st, rep = g.gerbil_result(job.enc, job.bins, job.state)
    assert st == g.GERBIL_ECAPACITY and rep.status & g.ST_OUT_CAP
    need = rep.n_out
    job2 = g.Job(ad, od, a.size, p, cap=need)
    job2.run()
    res = job2.result()
    ref = oracle.count(a, o, 32, threshold=1)
    keys, counts = res.sorted()
    assert np.array_equal(keys, ref.keys) and np.array_equal(counts, ref.counts)


def test_overflow_capacity_error():
    w = synth.CONFIGS["c1_tiny"].scaled(0.05)
    a, o = w.generate()
    ad, od = to_device(a, o)
    p = g.make_params(32, 7, 16, 1, max_probes=1, load_factor=0.95, overflow_cap=16)
    job = g.Job(ad, od, a.size, p)
    job.run()
    st, rep = g.gerbil_result(job.enc, job.bins, job.state)
    assert st == g.GERBIL_ECAPACITY and rep.status & g.ST_OVF_CAP and rep.n_overflow > 16


def test_superm_capacity_error():
    w = synth.CONFIGS["c1_tiny"].scaled(0.05)
    a, o = w.generate()
    ad, od = to_device(a, o)
    p = g.make_params(32, 7, 16, 1, superm_cap=100)
    job = g.Job(ad, od, a.size, p)
    job.run()
    st, rep = g.gerbil_result(job.enc, job.bins, job.state)
    assert st == g.GERBIL_ECAPACITY and rep.status & g.ST_SUPERM_CAP and rep.n_superm > 100


@pytest.mark.parametrize("load,theta,block", [(0.25, 8, 64), (0.9, 2, 1024), (0.5, 32, 512)])
@pytest.mark.parametrize("table", TABLES)
def test_results_do_not_depend_on_table_parameters(load, theta, block, table):
    w = synth.CONFIGS["c1_tiny"].scaled(0.2)
    a, o = w.generate()
    run_and_compare(a, o, 33, 7, 64, 2, load_factor=load, max_probes=theta, block=block, table=table)


def test_empty_and_short_input():
    a, o = reads_to_csr(["ACG", "", "NNNNNNNNNN"])
    res = g.count_kmers(a, o, 8, 3, 4, 1)
    assert res.keys.shape[0] == 0 and res.report.n_valid == 0 and int(res.hist.sum()) == 0


# ------------------------------------------------------- LDS sub-tables

@pytest.mark.parametrize("mode", [g.GERBIL_PLAIN, g.GERBIL_BATCHED])
def test_lds_large_bin_is_sliced(mode):
    """One bin of 6.8M k-mers with 64-key sub-tables: the bin is cut into hash
    slices (16384 sub-tables per slice at most)."""
    w = synth.CONFIGS["c1_tiny"]
    a, o = w.generate()
    run_and_compare(a, o, w.k, w.m, 1, w.threshold, hist_len=512, table=g.GERBIL_TABLE_LDS, mode=mode,
                    load_factor=0.011)


@pytest.mark.parametrize("pool", [1, 2, 5, 64])
def test_lds_key_slots(pool):
    w = synth.CONFIGS["c2_k65"].scaled(0.003)
    a, o = w.generate()
    run_and_compare(a, o, w.k, w.m, 64, w.threshold, hist_len=256, table=g.GERBIL_TABLE_LDS,
                    mode=g.GERBIL_BATCHED, pool=pool)


def test_sampled_run_sizes_spill_to_the_emergency_area_exactly():
    """LDS key runs are sized from every S-th super-mer. Homopolymer stretches
    put long clumps of one canonical key into single super-mers, so sampled
    sizes miss by more than their margin and keys spill past their run end;
    those keys take the emergency area and every count stays exact."""
    rng = np.random.default_rng(77)
    reads = []
    for _ in range(600):
        pre = "".join(np.array(list("ACGT"))[rng.integers(0, 4, int(rng.integers(20, 60)))].tolist())
        suf = "".join(np.array(list("ACGT"))[rng.integers(0, 4, int(rng.integers(20, 60)))].tolist())
        reads.append(pre + str(rng.choice(list("AC"))) * int(rng.integers(100, 400)) + suf)
    a, o = reads_to_csr(reads)
    spilled = []
    for S in (1, 2, 3, 7, 64, 1000):
        for mode in (g.GERBIL_BATCHED, g.GERBIL_PLAIN):
            res, _ = run_and_compare(a, o, 32, 7, 4, 1, hist_len=128, table=g.GERBIL_TABLE_LDS, mode=mode,
                                     size_sample=S)
            if S == 1:
                assert res.report.n_overflow == 0, "exact run sizes never spill"
            else:
                spilled.append(res.report.n_overflow)
    assert max(spilled) > 0, "no sampled run overflowed: the spill path was not exercised"


@pytest.mark.parametrize("table", [g.GERBIL_TABLE_LDS, g.GERBIL_TABLE_HBM])
def test_large_emergency_area_is_exact(table):
    """A workload of 1.7 M windows counted with a single probe per key and full
    tables, so that many of its occurrences are counted in the emergency area
    by its multi-workgroup table (hundreds of thousands with single-slot LDS
    probes; thousands with the 8-slot buckets of HBM tables)."""
    w = synth.CONFIGS["c2_k65"].scaled(0.001)
    a, o = w.generate()
    ref = oracle.count(a, o, w.k, threshold=2)
    res = g.count_kmers(a, o, w.k, w.m, 64, 2, 256, mode=g.GERBIL_BATCHED, table=table, max_probes=1,
                        load_factor=1.2 if table == g.GERBIL_TABLE_LDS else 0.95, overflow_cap=1 << 22)
    assert res.report.n_overflow > (100_000 if table == g.GERBIL_TABLE_LDS else 1_000), res.report.n_overflow
    keys, counts = res.sorted()
    assert np.array_equal(keys, ref.keys) and np.array_equal(counts, ref.counts)
    assert np.array_equal(res.hist, ref.folded_hist(256))

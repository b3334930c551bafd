"""The batched persistent counter vs the oracle and vs the plain schedule.

Same bar as the plain path: bit-exact pairs and histogram, across pool
sizes, load factors, probe limits and repeated runs on one workspace.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import random_reads, reads_to_csr, to_device
from paper_1607_06618_amd import gerbil as g

pytestmark = pytest.mark.gpu

B = g.GERBIL_BATCHED
TABLES = [pytest.param(g.GERBIL_TABLE_LDS, id="lds"), pytest.param(g.GERBIL_TABLE_HBM, id="hbm")]


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    g.load()


def same_as_oracle(res, ref, hist_len):
    keys, counts = res.sorted()
    assert res.report.n_valid == ref.n_valid
    assert keys.shape == ref.keys.shape, (keys.shape, ref.keys.shape)
    assert np.array_equal(keys, ref.keys)
    assert np.array_equal(counts, ref.counts)
    assert np.array_equal(res.hist, ref.folded_hist(hist_len))


@pytest.mark.parametrize("table", TABLES)
def test_batched_c1_full(table):
    w = synth.CONFIGS["c1_tiny"]
    a, o = w.generate()
    ref = oracle.count(a, o, w.k, threshold=w.threshold)
    res = g.count_kmers(a, o, w.k, w.m, w.n_bins, w.threshold, 512, mode=B, table=table)
    same_as_oracle(res, ref, 512)
    assert res.report.n_overflow == 0


@pytest.mark.parametrize("name,scale", [("c2_k65", 0.01), ("c3_skew", 0.001), ("c4_longk", 0.002)])
@pytest.mark.parametrize("table", TABLES)
def test_batched_config_shapes(name, scale, table):
    w = synth.CONFIGS[name].scaled(scale)
    a, o = w.generate()
    ref = oracle.count(a, o, w.k, threshold=w.threshold)
    res = g.count_kmers(a, o, w.k, w.m, w.n_bins, w.threshold, 1024, mode=B, table=table)
    same_as_oracle(res, ref, 1024)


@pytest.mark.parametrize("pool,load,theta", [(1, 0.5, 8), (2, 0.5, 8), (3, 0.7, 4), (8, 0.3, 8), (64, 0.9, 2),
                                             (1, 0.95, 1)])
@pytest.mark.parametrize("table", TABLES)
def test_batched_schedule_parameters(pool, load, theta, table):
    w = synth.CONFIGS["c2_k65"].scaled(0.003)
    a, o = w.generate()
    ref = oracle.count(a, o, w.k, threshold=w.threshold)
    res = g.count_kmers(a, o, w.k, w.m, 64, w.threshold, 256, mode=B, pool=pool, load_factor=load, max_probes=theta,
                        table=table)
    same_as_oracle(res, ref, 256)


@pytest.mark.parametrize("k", [16, 32, 33, 64, 99, 160, 256])
@pytest.mark.parametrize("table", TABLES)
def test_batched_random_k(k, table):
    rng = np.random.default_rng(77 + k)
    gen = "".join(np.array(list("ACGT"))[rng.integers(0, 4, 4000)].tolist())
    reads = []
    for _ in range(500):
        L = int(rng.integers(k, k + 200))
        s = int(rng.integers(0, len(gen) - L))
        reads.append(gen[s: s + L])
    reads += random_reads(rng, 50, 0, 400)
    a, o = reads_to_csr(reads)
    ref = oracle.count(a, o, k, threshold=2)
    res = g.count_kmers(a, o, k, min(9, k - 1), 97, 2, 128, mode=B, table=table)
    same_as_oracle(res, ref, 128)


@pytest.mark.parametrize("table", TABLES)
def test_batched_repeated_runs_reuse_workspace(table):
    w = synth.CONFIGS["c1_tiny"].scaled(0.2)
    a, o = w.generate()
    ad, od = to_device(a, o)
    p = g.make_params(w.k, w.m, w.n_bins, w.threshold, mode=B, pool=3, table=table)
    job = g.Job(ad, od, a.size, p, hist_len=128)
    ref = oracle.count(a, o, w.k, threshold=w.threshold)
    for _ in range(4):
        job.run()
        same_as_oracle(job.result(), ref, 128)


@pytest.mark.parametrize("table", TABLES)
def test_batched_and_plain_agree_on_skewed_bins(table):
    w = synth.CONFIGS["c3_skew"].scaled(0.002)
    a, o = w.generate()
    rng = np.random.default_rng(5)
    # a strongly skewed minimizer -> bin map: half of all m-mers in bin 0
    bmap = rng.integers(1, w.n_bins, 4 ** w.m).astype(np.uint32)
    bmap[rng.random(4 ** w.m) < 0.5] = 0
    import torch
    bm = torch.from_numpy(bmap.view(np.int32)).cuda()
    r1 = g.count_kmers(a, o, w.k, w.m, w.n_bins, w.threshold, 256, mode=B, bin_map_ptr=bm.data_ptr(),
                       table=table)
    r0 = g.count_kmers(a, o, w.k, w.m, w.n_bins, w.threshold, 256, mode=g.GERBIL_PLAIN,
                       bin_map_ptr=bm.data_ptr(), table=table)
    k1, c1 = r1.sorted()
    k0, c0 = r0.sorted()
    assert np.array_equal(k1, k0) and np.array_equal(c1, c0) and np.array_equal(r1.hist, r0.hist)
    ref = oracle.count(a, o, w.k, threshold=w.threshold)
    same_as_oracle(r1, ref, 256)


def test_batched_superm_capacity_error_schedules_nothing():
    w = synth.CONFIGS["c1_tiny"].scaled(0.05)
    a, o = w.generate()
    ad, od = to_device(a, o)
    p = g.make_params(32, 7, 16, 1, mode=B, superm_cap=100)
    job = g.Job(ad, od, a.size, p)
    job.run()
    st, rep = g.gerbil_result(job.enc, job.bins, job.state)
    assert st == g.GERBIL_ECAPACITY and rep.status & g.ST_SUPERM_CAP and rep.n_out == 0


def test_batched_overflow_capacity_error():
    w = synth.CONFIGS["c1_tiny"].scaled(0.05)
    a, o = w.generate()
    ad, od = to_device(a, o)
    p = g.make_params(32, 7, 16, 1, mode=B, max_probes=1, load_factor=0.95, overflow_cap=16)
    job = g.Job(ad, od, a.size, p)
    job.run()
    st, rep = g.gerbil_result(job.enc, job.bins, job.state)
    assert st == g.GERBIL_ECAPACITY and rep.status & g.ST_OVF_CAP


@pytest.mark.parametrize("mode", [g.GERBIL_PLAIN, B])
def test_sliced_bin_with_one_dominant_key(mode):
    """A bin large enough to be cut into hash slices, whose k-mers are nearly
    all one key: that key's occurrences all land in one slice, so the key
    slots must hold the whole bin (a slice is not bounded by its share)."""
    k, L, n = 65, 300, 35000
    reads = ["A" * L] * n + ["T" * L] * n   # one canonical key, A^65, in one bin
    a, o = reads_to_csr(reads)
    res = g.count_kmers(a, o, k, 9, 16, 1, 64, mode=mode, table=g.GERBIL_TABLE_LDS)
    expect = 2 * n * (L - k + 1)
    assert res.report.n_valid == expect
    keys, counts = res.sorted()
    assert keys.shape == (1, 3) and keys[0].tolist() == [0, 0, 0] and counts.tolist() == [expect]

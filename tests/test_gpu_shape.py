"""The two LDS workgroup shapes of the batched counter: one 1024-thread
workgroup per CU with 160 KB of LDS, or two 512-thread workgroups with 80 KB
each (gerbil_params.block = 512). The smaller shape has half-size LDS
tables, so ranks have twice the sub-tables and bins are cut into hash slices
sooner; results must be the oracle's, bit for bit, either way."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import reads_to_csr
from paper_1607_06618_amd import gerbil as g

pytestmark = pytest.mark.gpu

B = g.GERBIL_BATCHED
LDS = g.GERBIL_TABLE_LDS


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


@pytest.mark.parametrize("name,scale", [("c1_tiny", 1.0), ("c2_k65", 0.01), ("c3_skew", 0.001), ("c4_longk", 0.002)])
def test_half_shape_on_workload_shapes(name, scale):
    w = synth.CONFIGS[name]
    if scale != 1.0:
        w = w.scaled(scale)
    a, o = w.generate()
    ref = oracle.count(a, o, w.k, threshold=w.threshold)
    for block in (512, 1024):
        res = g.count_kmers(a, o, w.k, w.m, w.n_bins, w.threshold, 1024, mode=B, table=LDS, block=block)
        same_as_oracle(res, ref, 1024)


@pytest.mark.parametrize("k", [16, 32, 33, 55, 64, 65, 99, 160, 200, 256])
def test_half_shape_every_key_width(k):
    w = synth.CONFIGS["c2_k65"].scaled(0.002)
    a, o = w.generate()
    ref = oracle.count(a, o, k, threshold=2)
    res = g.count_kmers(a, o, k, 9, 64, 2, 256, mode=B, table=LDS, block=512)
    same_as_oracle(res, ref, 256)


@pytest.mark.parametrize("pool,load,theta,sample", [(1, 0.5, 8, 8), (3, 0.7, 4, 1), (16, 1.2, 64, 16), (2, 0.3, 1, 8)])
def test_half_shape_schedule_parameters(pool, load, theta, sample):
    w = synth.CONFIGS["c2_k65"].scaled(0.003)
    a, o = w.generate()
    ref = oracle.count(a, o, w.k, threshold=w.threshold)
    res = g.count_kmers(a, o, w.k, w.m, 64, w.threshold, 256, mode=B, pool=pool, load_factor=load, max_probes=theta,
                        size_sample=sample, table=LDS, block=512)
    same_as_oracle(res, ref, 256)


def test_half_shape_slices_a_bin_with_one_dominant_key():
    """One bin cut into hash slices (half-size tables slice sooner) whose
    k-mers are nearly all one key."""
    k, L, n = 65, 300, 35000
    reads = ["A" * L] * n + ["T" * L] * n
    a, o = reads_to_csr(reads)
    res = g.count_kmers(a, o, k, 9, 16, 1, 64, mode=B, table=LDS, block=512)
    expect = 2 * n * (L - k + 1)
    assert res.report.n_valid == expect
    keys, counts = res.sorted()
    assert keys.shape == (1, 3) and keys[0].tolist() == [0, 0, 0] and counts.tolist() == [expect]


def test_half_shape_non_canonical():
    w = synth.CONFIGS["c2_k65"].scaled(0.002)
    a, o = w.generate()
    ref = oracle.count(a, o, w.k, threshold=1, canonical=False)
    res = g.count_kmers(a, o, w.k, w.m, 64, 1, 256, mode=B, table=LDS, block=512, canonical=False)
    same_as_oracle(res, ref, 256)


@pytest.mark.parametrize("block", [256, 512, 1024])
@pytest.mark.parametrize("k", [32, 65, 200, 300])
def test_hbm_tables_every_block_size(block, k):
    """The batched counter on HBM tables with 256, 512 and 1024 threads per workgroup."""
    w = synth.CONFIGS["c2_k65"].scaled(0.002)
    a, o = w.generate()
    ref = oracle.count(a, o, k, threshold=2)
    res = g.count_kmers(a, o, k, 9, 64, 2, 256, mode=B, table=g.GERBIL_TABLE_HBM, block=block)
    same_as_oracle(res, ref, 256)


@pytest.mark.parametrize("block,theta,sample", [(1024, 0, 0), (512, 0, 0), (1024, 1, 0), (1024, 0, 64)])
def test_probe_histogram_accounts_for_every_window(block, theta, sample):
    """The optional probe histogram counts every k-mer occurrence once: by the
    probe that settled it, or in bucket 0 when it went to the emergency area
    without one (a spilled run). Counting stays exact with it enabled."""
    import torch
    w = synth.CONFIGS["c2_k65"].scaled(0.003)
    a, o = w.generate()
    ref = oracle.count(a, o, w.k, threshold=w.threshold)
    ph = torch.zeros(g.GERBIL_PROBE_HIST, dtype=torch.int64, device="cuda")
    res = g.count_kmers(a, o, w.k, w.m, 64, w.threshold, 256, mode=B, table=LDS, block=block, max_probes=theta,
                        size_sample=sample, probe_hist=ph.data_ptr())
    same_as_oracle(res, ref, 256)
    h = ph.cpu().numpy()
    assert int(h.sum()) == ref.n_valid
    if theta == 1:
        assert int(h[2:-1].sum()) == 0   # one probe, then the emergency area (last bucket)
    assert h[1] > 0

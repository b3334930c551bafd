"""The autotuner: its choice must count exactly (oracle), a second run of
the same shape must come from the cache, and a fixed placement must be kept."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import to_device
from paper_1607_06618_amd import gerbil as g

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    g.load()


def tuned_job(a, o, w, table=g.GERBIL_TABLE_AUTO):
    ad, od = to_device(a, o)
    p = g.make_params(w.k, w.m, w.n_bins, w.threshold, mode=g.GERBIL_BATCHED, table=table)
    job = g.Job(ad, od, int(o[-1]), p, hist_len=512)
    job.encode()
    job.bin()
    info = job.autotune()
    job.count()
    return job, info


def test_autotune_choice_counts_exactly_and_is_cached():
    w = synth.CONFIGS["c2_k65"].scaled(0.004)
    a, o = w.generate()
    ref = oracle.count(a, o, w.k, threshold=w.threshold)
    g.gerbil_autotune_reset()
    job, info = tuned_job(a, o, w)
    assert info.cached == 0 and info.candidates > 0 and info.best_ms > 0
    assert info.table in (g.GERBIL_TABLE_LDS, g.GERBIL_TABLE_HBM)
    assert job.p.table == info.table and job.p.pool == info.pool and job.p.block == info.block
    assert info.block in ((512, 1024) if info.table == g.GERBIL_TABLE_LDS else (256, 512, 1024))
    assert abs(job.p.load_factor - info.load_factor) < 1e-6
    res = job.result()
    keys, counts = res.sorted()
    assert np.array_equal(keys, ref.keys) and np.array_equal(counts, ref.counts)
    assert np.array_equal(res.hist, ref.folded_hist(512))
    # same shape again: the choice comes from the cache, nothing is timed
    job2, info2 = tuned_job(a, o, w)
    assert info2.cached == 1 and info2.candidates == info.candidates
    assert (info2.table, info2.pool, info2.block) == (info.table, info.pool, info.block)
    res2 = job2.result()
    k2, c2 = res2.sorted()
    assert np.array_equal(k2, ref.keys) and np.array_equal(c2, ref.counts)


@pytest.mark.parametrize("table", [g.GERBIL_TABLE_LDS, g.GERBIL_TABLE_HBM])
def test_autotune_keeps_a_fixed_placement(table):
    w = synth.CONFIGS["c1_tiny"].scaled(0.1)
    a, o = w.generate()
    ref = oracle.count(a, o, w.k, threshold=w.threshold)
    g.gerbil_autotune_reset()
    job, info = tuned_job(a, o, w, table=table)
    assert info.table == table and job.p.table == table
    res = job.result()
    keys, counts = res.sorted()
    assert np.array_equal(keys, ref.keys) and np.array_equal(counts, ref.counts)

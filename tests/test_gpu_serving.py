"""Serving loop: every job's result is the same alone and in the mix
(tolerance 0: identical pairs and histograms), and matches the oracle."""
import numpy as np
import pytest

import oracle
import synth
from paper_1607_06618_amd import gerbil as g
from paper_1607_06618_amd import serve

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    g.load()


def _requests(n_jobs, scale, arrivals):
    reqs, data = [], []
    for j in range(n_jobs):
        w = synth.serving_job(j, scale=scale)
        a, o = w.generate()
        data.append((w, a, o))
        reqs.append(serve.make_request(j, a, o, w.k, w.m, w.n_bins, w.threshold, arrival=float(arrivals[j])))
    return reqs, data


def test_alone_equals_mix_and_oracle():
    n = 6
    arrivals = synth.arrival_times(n) * 0.0   # all at once: maximal overlap
    reqs, data = _requests(n, 0.02, arrivals)
    alone = []
    for r in reqs:
        srv = serve.CountingServer(budget_bytes=64 << 30, max_inflight=1)
        alone.extend(srv.serve([r], realtime=False))
    srv = serve.CountingServer(budget_bytes=64 << 30, max_inflight=4)
    mixed = srv.serve(reqs, realtime=False)
    assert len(mixed) == n
    ks = sorted({d[0].k for d in data})
    assert len(ks) >= 2, "the mix should hold jobs of different k"
    for a_res, m_res, (w, a, o) in zip(alone, mixed, data):
        ka, ca = a_res.sorted()
        km, cm = m_res.sorted()
        assert np.array_equal(ka, km) and np.array_equal(ca, cm)
        assert np.array_equal(a_res.hist, m_res.hist)
        ref = oracle.count(a, o, w.k, threshold=w.threshold)
        assert np.array_equal(ka, ref.keys) and np.array_equal(ca, ref.counts)
        assert np.array_equal(a_res.hist, ref.folded_hist(1024))


def test_admission_respects_the_budget_and_output_retry():
    n = 4
    reqs, data = _requests(n, 0.01, np.zeros(n))
    # a budget below any single job still admits one job at a time (never zero)
    srv = serve.CountingServer(budget_bytes=1, max_inflight=4)
    res = srv.serve(reqs, realtime=False)
    assert [r.job_id for r in res] == list(range(n))
    stats = serve.summarize(res, srv.makespan)
    assert stats["jobs"] == n and stats["p99_latency_s"] >= stats["p50_latency_s"] > 0
    for r, (w, a, o) in zip(res, data):
        ref = oracle.count(a, o, w.k, threshold=w.threshold)
        k_, c_ = r.sorted()
        assert np.array_equal(k_, ref.keys) and np.array_equal(c_, ref.counts)


# The smallest seeded job of each k among the first 200 jobs of the stream,
# at their full (unscaled) sizes; their oracle results are stored as digests.
FULL_JOBS = (199, 129, 135)


def _fold(hist: np.ndarray, length: int) -> np.ndarray:
    h = np.zeros(length, dtype=np.uint64)
    h[: length - 1] = hist[: length - 1]
    h[length - 1] = hist[length - 1:].sum()
    return h


@pytest.mark.slow
def test_full_size_jobs_alone_and_mixed():
    import os
    import sys
    sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
    import fullsize
    from gpu_util import shard_digests_host

    reqs, golds = [], []
    for j in FULL_JOBS:
        gold = fullsize.read(f"job{j}")
        w = synth.serving_job(j, scale=1.0)
        a, o = w.generate()
        assert fullsize.input_fingerprint(a, o) == gold.fields["input"], "the generated reads changed"
        golds.append((w, gold))
        reqs.append(serve.make_request(j, a, o, w.k, w.m, w.n_bins, w.threshold, arrival=0.0))
    assert sorted(w.k for w, _ in golds) == [32, 55, 99]
    alone = []
    for r in reqs:
        alone.extend(serve.CountingServer(budget_bytes=64 << 30, max_inflight=1).serve([r], realtime=False))
    mixed = serve.CountingServer(budget_bytes=64 << 30, max_inflight=4).serve(reqs, realtime=False)
    alone = sorted(alone, key=lambda r: r.job_id)
    by_id = dict(zip(FULL_JOBS, golds))
    assert [r.job_id for r in mixed] == [r.job_id for r in alone] == sorted(FULL_JOBS)
    for a_res, m_res in zip(alone, mixed):
        w, gold = by_id[a_res.job_id]
        ka, ca = a_res.sorted()
        km, cm = m_res.sorted()
        assert np.array_equal(ka, km) and np.array_equal(ca, cm), f"job {a_res.job_id}: alone and mixed differ"
        assert np.array_equal(a_res.hist, m_res.hist)
        assert a_res.n_valid == gold.int("n_valid")
        assert np.array_equal(a_res.hist, _fold(gold.hist, a_res.hist.size))
        assert ka.shape[0] == gold.int("n_pairs")
        got = shard_digests_host(ka, ca, w.k, gold.int("shard_mod"))
        assert [(n, d) for n, d in got] == [(n, d) for n, _, d in gold.shards], f"job {a_res.job_id}: pairs differ"


def test_capacity_errors_are_retried_per_job():
    """A job whose emergency area is too small (forced: one probe, a tiny
    area) or whose output guess is too small is counted again with exact
    sizes; its result is still the oracle's, and no other job is affected."""
    n = 3
    reqs, data = _requests(n, 0.01, np.zeros(n))

    def tiny(p):
        p.max_probes = 1
        p.overflow_cap = 64

    srv = serve.CountingServer(budget_bytes=64 << 30, max_inflight=3, params_hook=tiny)
    res = srv.serve(reqs, realtime=False)
    assert [r.job_id for r in res] == list(range(n))
    assert all(r.retries == 1 and not r.error for r in res)
    for r, (w, a, o) in zip(res, data):
        ref = oracle.count(a, o, w.k, threshold=w.threshold)
        k_, c_ = r.sorted()
        assert np.array_equal(k_, ref.keys) and np.array_equal(c_, ref.counts)
        assert np.array_equal(r.hist, ref.folded_hist(r.hist.size))
        assert r.device_ms > 0 and r.count_kernel_ms > 0

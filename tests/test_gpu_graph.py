"""Whole-path replay: encode -> bin -> count -> histogram recorded once into a
HIP graph and replayed. Every replay must give the eager result, which must
equal the oracle's, with eager work and synchronisation between replays."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import to_device
from paper_1607_06618_amd import gerbil as g

pytestmark = pytest.mark.gpu

TABLES = [pytest.param(g.GERBIL_TABLE_LDS, id="lds"), pytest.param(g.GERBIL_TABLE_HBM, id="hbm")]


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    g.load()


def snapshot(job):
    r = job.result()
    k, c = r.sorted()
    return k.copy(), c.copy(), r.hist.copy(), r.report.n_valid, r.report.n_out


@pytest.mark.parametrize("name,scale", [("c1_tiny", 0.2), ("c2_k65", 0.005), ("c4_longk", 0.001)])
@pytest.mark.parametrize("table", TABLES)
def test_graph_replays_match_eager_and_oracle(name, scale, table):
    import torch
    w = synth.CONFIGS[name].scaled(scale)
    a, o = w.generate()
    ref = oracle.count(a, o, w.k, threshold=w.threshold)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ad, od = to_device(a, o)
    stream.synchronize()
    p = g.make_params(w.k, w.m, w.n_bins, w.threshold, mode=g.GERBIL_BATCHED, table=table)
    job = g.Job(ad, od, int(o[-1]), p, hist_len=512, stream=stream)
    job.run()
    eager = snapshot(job)
    assert np.array_equal(eager[0], ref.keys) and np.array_equal(eager[1], ref.counts)
    assert np.array_equal(eager[2], ref.folded_hist(512))
    try:
        job.capture()
        st, n_nodes, n_kernel = g.gerbil_graph_info(job.graph)
        assert st == g.GERBIL_OK and n_nodes == n_kernel and n_kernel >= 8
        for rep in range(3):
            # clobber every output, then unrelated eager work on the same stream
            with torch.cuda.stream(stream):
                job.keys_d.fill_(-1)
                job.counts_d.fill_(0)
                job.hist_d.fill_(7)
                junk = torch.ones(1 << 20, device=ad.device).cumsum(0)
            stream.synchronize()
            job.replay()
            got = snapshot(job)
            for x, y in zip(eager, got):
                assert np.array_equal(x, y), f"replay {rep} differs from the eager run"
            del junk
    finally:
        job.close()


def test_graph_replays_follow_new_input_in_place():
    """The graph reads the input buffers at replay time: new reads of the same
    size written into them give the new counts."""
    import torch
    w1 = synth.CONFIGS["c1_tiny"].scaled(0.05)
    a1, o1 = w1.generate()
    from dataclasses import replace
    w2 = replace(w1, seed=w1.seed + 17)
    a2, o2 = w2.generate()
    assert a1.size == a2.size and np.array_equal(o1, o2)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ad, od = to_device(a1, o1)
    stream.synchronize()
    p = g.make_params(w1.k, w1.m, w1.n_bins, w1.threshold, mode=g.GERBIL_BATCHED)
    job = g.Job(ad, od, int(o1[-1]), p, hist_len=256, stream=stream, cap=a1.size)
    # the tables are sized from the first input's bins: leave room for the second's
    job.encode()
    job.bin()
    need = g.gerbil_count_workspace(job.bins, job.p, g._stream_handle(stream))
    job.ws_count = torch.empty(2 * need, dtype=torch.uint8, device=ad.device)
    job.run()
    job.result()
    try:
        job.capture()
        for a, ref_in in ((a2, a2), (a1, a1)):
            with torch.cuda.stream(stream):
                ad.copy_(torch.from_numpy(a))
            stream.synchronize()
            job.replay()
            ref = oracle.count(ref_in, o1, w1.k, threshold=w1.threshold)
            keys, counts, hist, n_valid, _ = snapshot(job)
            assert n_valid == ref.n_valid
            assert np.array_equal(keys, ref.keys) and np.array_equal(counts, ref.counts)
            assert np.array_equal(hist, ref.folded_hist(256))
    finally:
        job.close()


@pytest.mark.parametrize("variant", ["noncanonical", "cgat_table", "dfp_table"])
def test_graph_replays_with_other_modes(variant):
    """The `-d` mode and the rank-table orders replay from a graph exactly as
    they run eagerly (the rank table is read at replay time)."""
    import torch
    w = synth.CONFIGS["c2_k65"].scaled(0.003)
    a, o = w.generate()
    canonical = variant != "noncanonical"
    ref = oracle.count(a, o, w.k, threshold=w.threshold, canonical=canonical)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ad, od = to_device(a, o)
    stream.synchronize()
    table_d, kw = None, {}
    if variant != "noncanonical":
        probe = g.Job(ad, od, int(o[-1]), g.make_params(w.k, w.m, w.n_bins, w.threshold), stream=stream)
        probe.encode()
        kind = g.GERBIL_RANKS_CGAT if variant == "cgat_table" else g.GERBIL_RANKS_DFP
        table_d = g.order_table(kind, w.m, pivot=0.5, enc=probe.enc, stream=stream)
        kw = dict(order=g.GERBIL_ORDER_TABLE, rank_table_ptr=table_d.data_ptr())
    p = g.make_params(w.k, w.m, w.n_bins, w.threshold, mode=g.GERBIL_BATCHED, canonical=canonical, **kw)
    job = g.Job(ad, od, int(o[-1]), p, hist_len=512, stream=stream)
    job.run()
    eager = snapshot(job)
    assert np.array_equal(eager[0], ref.keys) and np.array_equal(eager[1], ref.counts)
    try:
        job.capture()
        for rep in range(2):
            with torch.cuda.stream(stream):
                job.keys_d.fill_(-1)
                job.counts_d.fill_(0)
                job.hist_d.fill_(7)
            stream.synchronize()
            job.replay()
            got = snapshot(job)
            for x, y in zip(eager, got):
                assert np.array_equal(x, y), f"replay {rep} differs from the eager run"
    finally:
        job.close()

"""Exact parity at the full sizes of the named workloads, in the batched
launch configuration the benchmark times.

The oracle's results at these sizes are stored as digests in
``tests/golden/fullsize_<name>.txt`` (written offline by
``tests/golden/fullsize.py``, which calls only the oracle and the read
generator). The GPU result must reproduce them exactly:
  * the reads are the ones the oracle counted (input fingerprint);
  * n_valid, and every bucket of the count-of-counts histogram over all
    distinct keys;
  * the number of emitted pairs, and for every hash shard of the oracle
    (``oracle.shard_of``) the number of pairs and the SHA-256 of those pairs
    in ascending key order. Equal digests in every shard mean equal pair sets.
"""
import os
import sys

import numpy as np
import pytest

import synth
from paper_1607_06618_amd import gerbil as g

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import fullsize  # noqa: E402
from gpu_util import shard_digests_device  # noqa: E402

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    g.load()


def check_against_golden(name, job, gold, W, k):
    st, rep = g.gerbil_result(job.enc, job.bins, job.state)
    assert st == g.GERBIL_OK, (st, rep.status)
    n_out = int(rep.n_out)
    print(f"[{name}] n_valid={rep.n_valid} n_out={n_out} emergency={rep.n_overflow} max={rep.max_count}",
          flush=True)
    assert rep.n_valid == gold.int("n_valid")
    hist = job.hist_d.cpu().numpy().view(np.uint64)
    assert np.array_equal(hist, gold.hist), "count-of-counts histogram differs from the oracle's"
    assert n_out == gold.int("n_pairs")
    assert rep.max_count == gold.int("max_count")
    got = shard_digests_device(job.keys_d, job.counts_d, n_out, W, k, gold.int("shard_mod"))
    bad = [s for s, (mine, ref) in enumerate(zip(got, gold.shards)) if mine[0] != ref[0] or mine[1] != ref[2]]
    assert not bad, f"pairs differ from the oracle's in shards {bad[:10]} (of {len(got)})"


@pytest.mark.parametrize("name,tune,block", [("c2_k65", False, 0), ("c2_k65", False, 512), ("c3_skew", True, 0),
                                              ("c3_skew", False, 0), ("c4_longk", False, 0), ("c4_longk", False, 512)])
def test_full_size_workload(name, tune, block):
    import torch
    if not os.path.exists(fullsize.golden_path(name)):
        pytest.skip(f"no oracle digest for {name} yet: run tests/golden/fullsize.py {name}")
    gold = fullsize.read(name)
    w = synth.CONFIGS[name]
    a, o = w.generate(threads=16)
    assert fullsize.input_fingerprint(a, o) == gold.fields["input"], "the generated reads changed"
    k, t, W = w.k, w.threshold, g.words(w.k)
    dev = torch.device("cuda:0")
    ad = torch.from_numpy(a).to(dev)
    od = torch.from_numpy(o.view(np.int64)).to(dev)
    del a
    bm = torch.from_numpy(w.bin_map().view(np.int32)).to(dev) if w.skew_bins else None
    # the tuned run chooses among LDS-table schedules (HBM tables are an order of
    # magnitude slower on these workloads, and timing them would dominate the test)
    p = g.make_params(k, w.m, w.n_bins, t, mode=g.GERBIL_BATCHED, block=block,
                      table=g.GERBIL_TABLE_LDS if tune else g.GERBIL_TABLE_AUTO,
                      bin_map_ptr=bm.data_ptr() if bm is not None else 0)
    job = g.Job(ad, od, int(o[-1]), p, hist_len=fullsize.HIST_LEN)
    if tune:
        job.encode()
        job.bin()
        info = job.autotune()
        print(f"[{name}] tuned: table={info.table} load={info.load_factor:.2f} pool={info.pool} block={info.block} "
              f"candidates={info.candidates} best={info.best_ms:.2f} ms", flush=True)
        job.hist_d.zero_()
    job.run()
    check_against_golden(name, job, gold, W, k)

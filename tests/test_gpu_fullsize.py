"""Parity at the full sizes of the named workloads, in the batched launch
configuration the benchmark times.

The oracle cannot count billions of windows in a test, so the results are
checked by properties that hold at any size and on samples the oracle
counts one by one:
  * n_valid equals the oracle's valid-window count (read chunks in parallel);
  * sum over c of c * hist[c] equals n_valid (every occurrence is counted once);
  * the pairs emitted are exactly the histogram's keys with count >= t;
  * no key is emitted twice (hash sort on the device, full-key compare);
  * sampled output pairs carry the oracle's count of their key;
  * sampled read windows: the canonical key is emitted iff its oracle count
    is >= t, and then with that count.
"""
import concurrent.futures as cf

import numpy as np
import pytest

import oracle
import synth
from paper_1607_06618_amd import gerbil as g

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

HIST_LEN = 65536
N_SAMPLE = 256


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    g.load()


def oracle_n_valid(a, o, k, threads=16):
    """Valid windows by the oracle's encoder over read chunks."""
    n_reads = o.size - 1
    cuts = np.linspace(0, n_reads, threads + 1).astype(np.int64)

    def part(i):
        r0, r1 = int(cuts[i]), int(cuts[i + 1])
        if r1 <= r0:
            return 0
        base = int(o[r0])
        return oracle.encode(a[base: int(o[r1])], o[r0: r1 + 1] - np.uint64(base), k)[2]

    with cf.ThreadPoolExecutor(threads) as ex:
        return sum(ex.map(part, range(threads)))


def canonical_key(window: bytes, k: int) -> np.ndarray:
    """The oracle's canonical key of one window (a one-read count)."""
    a = np.frombuffer(window, dtype=np.uint8).copy()
    o = np.array([0, a.size], dtype=np.uint64)
    r = oracle.count(a, o, k, threshold=1)
    assert r.keys.shape[0] == 1
    return r.keys[0]


def find_in_output(keys_d, n_out, W, key):
    """Indexes of `key` among the emitted pairs (searched on the device)."""
    import torch
    q = torch.as_tensor(key.view(np.int64), device=keys_d.device)
    rows = keys_d[: n_out * W].view(n_out, W)
    return torch.nonzero((rows == q).all(dim=1)).flatten().cpu().numpy()


def duplicates(keys_d, n_out, W):
    """Number of keys emitted more than once (64-bit mix sorted on the device,
    candidate pairs compared word by word)."""
    import torch
    rows = keys_d[: n_out * W].view(n_out, W)
    h = torch.zeros(n_out, dtype=torch.int64, device=keys_d.device)
    for w in range(W):
        h = (h ^ rows[:, w]) * 0x1000193 + (h >> 29)
    hs, idx = torch.sort(h)
    same = torch.nonzero(hs[1:] == hs[:-1]).flatten()
    if same.numel() == 0:
        return 0
    a_rows, b_rows = rows[idx[same]], rows[idx[same + 1]]
    return int((a_rows == b_rows).all(dim=1).sum().item())


@pytest.mark.parametrize("name", ["c2_k65", "c3_skew", "c4_longk"])
def test_full_size_workload(name):
    import torch
    w = synth.CONFIGS[name]
    a, o = w.generate(threads=16)
    k, t, W = w.k, w.threshold, g.words(w.k)
    dev = torch.device("cuda:0")
    ad = torch.from_numpy(a).to(dev)
    od = torch.from_numpy(o.view(np.int64)).to(dev)
    bm = torch.from_numpy(w.bin_map().view(np.int32)).to(dev) if w.skew_bins else None
    p = g.make_params(k, w.m, w.n_bins, t, mode=g.GERBIL_BATCHED,
                      bin_map_ptr=bm.data_ptr() if bm is not None else 0)
    job = g.Job(ad, od, int(o[-1]), p, hist_len=HIST_LEN)
    job.run()
    st, rep = g.gerbil_result(job.enc, job.bins, job.state)
    assert st == g.GERBIL_OK, (st, rep.status)
    n_out = int(rep.n_out)
    hist = job.hist_d.cpu().numpy().view(np.uint64).astype(np.float64)
    print(f"[{name}] n_valid={rep.n_valid} n_out={n_out} emergency={rep.n_overflow} max={rep.max_count}", flush=True)

    # size-independent properties
    assert rep.n_valid == oracle_n_valid(a, o, k)
    assert rep.max_count < HIST_LEN - 1
    c = np.arange(HIST_LEN, dtype=np.float64)
    assert int((c * hist).sum()) == rep.n_valid
    assert int(hist[t:].sum()) == n_out
    counts_d = job.counts_d[:n_out]
    assert int(counts_d.min().item()) >= t
    assert duplicates(job.keys_d, n_out, W) == 0

    # sampled outputs, counted by the oracle
    rng = np.random.default_rng(2024)
    sel = np.unique(rng.integers(0, n_out, N_SAMPLE))
    rows = job.keys_d[: n_out * W].view(n_out, W)
    sel_d = torch.as_tensor(sel, device=dev)
    q_keys = rows[sel_d].cpu().numpy().view(np.uint64)
    q_counts = counts_d[sel_d].cpu().numpy().view(np.uint32).astype(np.uint64)

    # sampled windows of the reads
    windows = []
    while len(windows) < N_SAMPLE:
        r = int(rng.integers(0, o.size - 1))
        L = int(o[r + 1] - o[r])
        if L < k:
            continue
        s = int(o[r]) + int(rng.integers(0, L - k + 1))
        win = bytes(a[s: s + k])
        if all(ch in b"ACGTacgt" for ch in win):
            windows.append(win)
    w_keys = np.stack([canonical_key(x, k) for x in windows])

    got = oracle.count_keys_parallel(a, o, k, np.concatenate([q_keys, w_keys]), threads=16)
    assert np.array_equal(got[: sel.size], q_counts), "an emitted count differs from the oracle's"
    for key, cnt in zip(w_keys, got[sel.size:]):
        assert cnt >= 1
        where = find_in_output(job.keys_d, n_out, W, key)
        if cnt >= t:
            assert where.size == 1, "a key at or above the threshold is missing or repeated"
            assert int(job.counts_d[int(where[0])].item()) == int(cnt)
        else:
            assert where.size == 0, "a key below the threshold was emitted"

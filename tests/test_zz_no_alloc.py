"""The allocation-free entry point gerbil_records_noalloc against
gerbil_records with a caller workspace: byte-identical App. C record streams
and sizes, on calls in a row where a later input is smaller than an earlier
one (the shared scratch keeps the earlier call's contents)."""
import numpy as np
import pytest

from paper_1607_06618_amd import gerbil as g

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    g.load()


def _pairs(rng, n, k):
    W = (k + 31) // 32
    r = k - 32 * (W - 1)
    keys = rng.integers(0, 2 ** 63, size=(n, W), dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, size=(n, W),
                                                                                                 dtype=np.uint64)
    if r < 32:
        keys[:, W - 1] &= np.uint64((1 << (2 * r)) - 1)
    counts = rng.integers(1, 300, size=n, dtype=np.uint32)     # some counters take the 5-byte form
    counts[rng.random(n) < 0.001] = 0xFFFFFFFE
    return keys, counts


def _both(keys, counts, k):
    import torch
    n = counts.size
    kb = (k + 3) // 4
    keys_d = torch.from_numpy(keys.reshape(-1).view(np.int64)).cuda()
    counts_d = torch.from_numpy(counts.view(np.int32)).cuda()
    cap = max(1, n * (5 + kb))
    s = torch.cuda.current_stream()
    h = int(s.cuda_stream)
    ws = torch.empty(max(256, g.gerbil_records_workspace(n)), dtype=torch.uint8, device="cuda")
    out_a = torch.full((cap,), 0xAA, dtype=torch.uint8, device="cuda")
    out_b = torch.full((cap,), 0x55, dtype=torch.uint8, device="cuda")
    size_a = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    size_b = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    g.check("gerbil_records", g.gerbil_records(keys_d.data_ptr(), counts_d.data_ptr(), n, k, ws.data_ptr(),
                                               ws.numel(), out_a.data_ptr(), cap, size_a.data_ptr(), h))
    g.check("gerbil_records_noalloc", g.gerbil_records_noalloc(keys_d.data_ptr(), counts_d.data_ptr(), n, k,
                                                               out_b.data_ptr(), cap, size_b.data_ptr(), h))
    s.synchronize()
    na, nb = int(size_a.item()), int(size_b.item())
    return na, nb, out_a.cpu().numpy(), out_b.cpu().numpy()


def test_noalloc_equals_workspace_calls_in_a_row():
    rng = np.random.default_rng(20240607)
    # many tiles with a ragged last one, then a smaller input, then one tile
    for n, k in ((300_001, 65), (70_003, 31), (5_000, 200)):
        keys, counts = _pairs(rng, n, k)
        na, nb, a, b = _both(keys, counts, k)
        kb = (k + 3) // 4
        assert na == nb == n * (1 + kb) + 4 * int((counts >= 255).sum())
        assert np.array_equal(a[:na], b[:nb]), f"record streams differ (n={n}, k={k})"


def test_noalloc_empty_and_oversize():
    import torch
    size = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    h = int(torch.cuda.current_stream().cuda_stream)
    assert g.gerbil_records_noalloc(0, 0, 0, 65, 0, 0, size.data_ptr(), h) == g.GERBIL_OK
    torch.cuda.synchronize()
    assert int(size.item()) == 0
    # rejected before anything is enqueued
    big = g.GERBIL_RECORDS_NOALLOC_MAX + 1
    assert g.gerbil_records_noalloc(8, 8, big, 65, 8, 8, size.data_ptr(), h) == g.GERBIL_EINVAL

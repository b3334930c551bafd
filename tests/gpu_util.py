"""Helpers for the GPU tests: run the C-ABI path stage by stage and read
device arrays back. No counting arithmetic lives here."""
import numpy as np

from paper_1607_06618_amd import gerbil as g


def device_slice(ws, ptr, nbytes):
    """Bytes [ptr, ptr+nbytes) of the workspace tensor ``ws`` as a numpy array."""
    off = int(ptr) - ws.data_ptr()
    assert 0 <= off and off + nbytes <= ws.numel(), (off, nbytes, ws.numel())
    return ws[off: off + nbytes].cpu().numpy()


def to_device(ascii, offsets):
    import torch
    a = torch.from_numpy(np.ascontiguousarray(ascii, dtype=np.uint8)).cuda()
    o = torch.from_numpy(np.ascontiguousarray(offsets, dtype=np.uint64).view(np.int64)).cuda()
    return a, o


def make_job(ascii, offsets, k, m=7, n_bins=16, threshold=1, hist_len=256, **kw):
    a, o = to_device(ascii, offsets)
    p = g.make_params(k, m, n_bins, threshold, **kw)
    return g.Job(a, o, int(offsets[-1]), p, hist_len=hist_len)


def encoded_arrays(job):
    enc = job.enc
    packed = device_slice(job.ws_enc, enc.packed, 8 * enc.n_words).view(np.uint64)
    ok = device_slice(job.ws_enc, enc.kmer_ok, 8 * enc.n_mask).view(np.uint64)
    return packed, ok


def bin_arrays(job):
    """(desc uint64[n], bin_off uint64[n_bins+1], bin_kmers uint64[n_bins])."""
    b = job.bins
    off = device_slice(job.ws_bin, b.bin_off, 8 * (b.n_bins + 1)).view(np.uint64)
    km = device_slice(job.ws_bin, b.bin_kmers, 8 * b.n_bins).view(np.uint64)
    n = int(off[-1])
    desc = device_slice(job.ws_bin, b.desc, 8 * n).view(np.uint64) if n else np.zeros(0, np.uint64)
    return desc, off, km


def reads_to_csr(reads):
    data = "".join(reads).encode()
    offs = np.zeros(len(reads) + 1, dtype=np.uint64)
    offs[1:] = np.cumsum([len(r) for r in reads])
    return np.frombuffer(data, dtype=np.uint8).copy(), offs


def random_reads(rng, n, min_len, max_len, n_rate=0.02, lower_rate=0.02, junk="NnRY-"):
    reads = []
    for _ in range(n):
        L = int(rng.integers(min_len, max_len + 1))
        codes = rng.integers(0, 4, L)
        s = np.array(list("ACGT"))[codes]
        low = rng.random(L) < lower_rate
        s = np.where(low, np.char.lower(s), s)
        bad = rng.random(L) < n_rate
        s = np.where(bad, rng.choice(list(junk), L), s)
        reads.append("".join(s.tolist()))
    return reads


def shard_digests_device(keys_d, counts_d, n, W, k, shard_mod, threads=16):
    """Per-shard (pair count, SHA-256) of emitted pairs, in the layout the
    full-size golden files use: pairs of shard s (``oracle.shard_of``) in
    ascending key order. Sorting runs on the device (stable sorts, last word
    first, then by shard); shard ids and digests are computed on the host."""
    import concurrent.futures as cf
    import os
    import sys

    import torch

    import oracle
    sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
    import fullsize

    dev = keys_d.device
    rows = keys_d[: n * W].view(n, W)
    shard = oracle.shard_of(rows.cpu().numpy().view(np.uint64), k, shard_mod)
    shard_d = torch.from_numpy(shard.view(np.int64)).to(dev)
    sign = torch.iinfo(torch.int64).min   # flips the sign bit: signed order = unsigned order
    perm = torch.arange(n, device=dev)
    for w in reversed(range(W)):
        _, idx = torch.sort(rows[perm, w] ^ sign, stable=True)
        perm = perm[idx]
    _, idx = torch.sort(shard_d[perm], stable=True)
    perm = perm[idx]
    keys_s = rows[perm].cpu().numpy().view(np.uint64)
    counts_s = counts_d[:n][perm].cpu().numpy().view(np.uint32)
    per = np.bincount(shard.astype(np.int64), minlength=shard_mod)
    bounds = np.concatenate([[0], np.cumsum(per)])

    def one(s):
        lo, hi = int(bounds[s]), int(bounds[s + 1])
        return int(hi - lo), fullsize.pairs_digest(keys_s[lo:hi], counts_s[lo:hi])

    with cf.ThreadPoolExecutor(threads) as ex:
        return list(ex.map(one, range(shard_mod)))


def shard_digests_host(keys, counts, k, shard_mod):
    """The same digests for pairs already on the host (any order)."""
    import os
    import sys

    import oracle
    sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
    import fullsize

    keys = np.ascontiguousarray(keys, dtype=np.uint64).reshape(-1, (k + 31) // 32)
    shard = oracle.shard_of(keys, k, shard_mod) if keys.shape[0] else np.zeros(0, np.uint64)
    order = np.lexsort(tuple(keys.T[::-1]) + (shard,)) if keys.shape[0] else np.zeros(0, np.int64)
    keys, counts, shard = keys[order], np.asarray(counts, dtype=np.uint32)[order], shard[order]
    out = []
    for s in range(shard_mod):
        sel = shard == s
        out.append((int(sel.sum()), fullsize.pairs_digest(keys[sel], counts[sel])))
    return out

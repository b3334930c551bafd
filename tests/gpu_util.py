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

"""FASTA/FASTQ parsing on the device against the oracle's parser.

Byte and index work, so the bar is bit-exact: status bits, format, line,
read and byte counts, and -- when the status is 0 -- the read bytes and
offsets.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import random_reads, reads_to_csr
from paper_1607_06618_amd import gerbil as g

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    g.load()


def to_device(text: bytes, shift: int = 0):
    """The text on the device, starting `shift` bytes into its buffer."""
    import torch
    buf = torch.zeros(len(text) + shift + 64, dtype=torch.uint8, device="cuda")
    if text:
        buf[shift: shift + len(text)] = torch.frombuffer(bytearray(text), dtype=torch.uint8).cuda()
    return buf[shift: shift + len(text)]


def compare(text: bytes, fmt: int = 0, shift: int = 0, lines_cap=None):
    ref = oracle.parse_reads(text, fmt)
    got = g.parse(to_device(text, shift), fmt, lines_cap=lines_cap)
    info = got.info
    assert (info.status, info.format, info.n_lines, info.n_bytes) == (ref.status, ref.fmt, ref.n_lines, ref.n_bytes)
    assert info.n_reads == ref.offsets.size - 1
    if ref.status == 0:
        assert np.array_equal(got.seq.cpu().numpy(), ref.ascii)
        assert np.array_equal(got.offsets.cpu().numpy().view(np.uint64), ref.offsets)
    return got, ref


HAND = [
    b">r1 first\nACG\nTN\n>r2\n>r3\r\nGG\r\nca\r\n\n>r4\nA",
    b"@a\nACGT\n+\n@@+!\n@b x\nNN\n+b x\n>+\n@c\n\n+\n\n",
    b"", b"\n", b"@", b">", b">\n", b"@\n\n+\n\n", b">a\r\n\r\n", b">a\nAC\r", b">a\n\r",
    b"ACGT\n", b"@a\nAC\n+\nII\n@b\nAC\n", b"@a\nAC\n-\nII\n", b"@a\nAC\n+\nIII\n", b"@a\nAC\n+\nII\nb\nAC\n+\nII\n",
    b"\n@a\nAC\n+\nII\n",
]


@pytest.mark.parametrize("i", range(len(HAND)))
def test_hand_written_texts(i):
    compare(HAND[i])


def test_forced_formats():
    compare(b"AC\n>a\nAC\n", fmt=g.GERBIL_FORMAT_FASTA)     # orphan sequence
    compare(b"\n\n>a\nAC\n", fmt=g.GERBIL_FORMAT_FASTA)     # blank lines first are fine
    compare(b">a\nAC\n", fmt=g.GERBIL_FORMAT_FASTQ)          # read as FASTQ: errors
    compare(b"@a\nAC\n+\nII\n", fmt=g.GERBIL_FORMAT_FASTA)   # read as FASTA: orphans


def synthetic_reads(seed, n, max_len):
    rng = np.random.default_rng(seed)
    return reads_to_csr(random_reads(rng, n, 0, max_len) + ["", "ACGT" * 300])


@pytest.mark.parametrize("crlf", [False, True])
@pytest.mark.parametrize("shift", [0, 1, 7])
def test_fastq_many_tiles(crlf, shift):
    # about 1.3 MB of text: tens of 16 KB byte tiles, several line tiles, ragged ends
    a, o = synthetic_reads(11 + shift, 3001, 400)
    compare(synth.to_fastq(a, o, seed=4, crlf=crlf), shift=shift)


@pytest.mark.parametrize("width,crlf,blank", [(60, False, False), (1, False, True), (0, True, False),
                                              (80, True, True), (4096, False, False)])
def test_fasta_many_tiles(width, crlf, blank):
    a, o = synthetic_reads(21 + width, 1500, 2000)
    compare(synth.to_fasta(a, o, width=width, crlf=crlf, blank_lines=blank), shift=3)


def test_lines_cap_too_small_then_exact():
    a, o = synthetic_reads(5, 700, 200)
    text = synth.to_fastq(a, o)
    ref = oracle.parse_reads(text)
    import torch
    d = to_device(text)
    # the wrapper calls again with the reported line count
    got = g.parse(d, lines_cap=10)
    assert got.info.status == 0 and got.info.n_lines == ref.n_lines
    assert np.array_equal(got.seq.cpu().numpy(), ref.ascii)
    # one call with too few lines reports the count and produces no reads
    cap = 100
    ws = torch.empty(g.gerbil_parse_workspace(len(text), cap), dtype=torch.uint8, device="cuda")
    seq = torch.empty(len(text), dtype=torch.uint8, device="cuda")
    off = torch.empty(cap + 1, dtype=torch.int64, device="cuda")
    info = torch.zeros(ctypes_size(), dtype=torch.uint8, device="cuda")
    st = g.gerbil_parse(d.data_ptr(), len(text), 0, ws.data_ptr(), ws.numel(), cap, seq.data_ptr(), len(text),
                        off.data_ptr(), cap, info.data_ptr(), int(torch.cuda.current_stream().cuda_stream))
    assert st == g.GERBIL_OK
    r = g.gerbil_parsed.from_buffer_copy(info.cpu().numpy().tobytes())
    assert r.status == g.GERBIL_PARSE_ELINECAP and r.n_lines == ref.n_lines and r.n_reads == 0


def ctypes_size():
    import ctypes
    return ctypes.sizeof(g.gerbil_parsed)


def test_short_sequence_and_read_buffers():
    import torch
    a, o = synthetic_reads(8, 900, 300)
    text = synth.to_fastq(a, o)
    ref = oracle.parse_reads(text)
    d = to_device(text)
    n = len(text)
    lines = ref.n_lines
    seq_cap, reads_cap = ref.n_bytes // 2, (ref.offsets.size - 1) // 3
    ws = torch.empty(g.gerbil_parse_workspace(n, lines), dtype=torch.uint8, device="cuda")
    seq = torch.full((ref.n_bytes + 512,), 0x5A, dtype=torch.uint8, device="cuda")
    off = torch.full((reads_cap + 64,), -7, dtype=torch.int64, device="cuda")
    info = torch.zeros(ctypes_size(), dtype=torch.uint8, device="cuda")
    st = g.gerbil_parse(d.data_ptr(), n, 0, ws.data_ptr(), ws.numel(), lines, seq.data_ptr(), seq_cap,
                        off.data_ptr(), reads_cap, info.data_ptr(), int(torch.cuda.current_stream().cuda_stream))
    assert st == g.GERBIL_OK
    r = g.gerbil_parsed.from_buffer_copy(info.cpu().numpy().tobytes())
    assert r.status == g.GERBIL_PARSE_EBYTES | g.GERBIL_PARSE_EREADS
    assert r.n_bytes == ref.n_bytes and r.n_reads == ref.offsets.size - 1
    s = seq.cpu().numpy()
    assert np.array_equal(s[:seq_cap], ref.ascii[:seq_cap])
    assert (s[seq_cap:] == 0x5A).all()
    ofs = off.cpu().numpy()
    assert np.array_equal(ofs[:reads_cap].view(np.uint64), ref.offsets[:reads_cap])
    assert (ofs[reads_cap:] == -7).all()


@pytest.mark.parametrize("k", [25, 65])
def test_parse_then_count(k):
    """Parse on the device, count on the device: the oracle's count of the
    oracle's parse."""
    a, o = synthetic_reads(31 + k, 2000, 500)
    text = synth.to_fasta(a, o, width=70)
    p = g.parse(to_device(text))
    assert p.info.status == 0
    n_reads = int(p.info.n_reads)
    prm = g.make_params(k, 9, 64, 2, mode=g.GERBIL_BATCHED)
    job = g.Job(p.seq, p.offsets, int(p.info.n_bytes), prm)
    job.run()
    res = job.result()
    ref_p = oracle.parse_reads(text)
    ref = oracle.count(ref_p.ascii, ref_p.offsets, k, threshold=2)
    keys, counts = res.sorted()
    assert n_reads == ref_p.offsets.size - 1
    assert np.array_equal(keys, ref.keys) and np.array_equal(counts, ref.counts)


@pytest.mark.slow
def test_full_size_fastq_of_the_k65_workload():
    """The 100 Mbp workload rendered as FASTQ (about 220 MB of text) parses
    back to the reads it was rendered from; the oracle's parser is pinned to
    give exactly that for any rendering (round-trip pins)."""
    w = synth.CONFIGS["c2_k65"]
    a, o = w.generate(threads=16)
    text = synth.to_fastq(a, o, seed=9)
    p = g.parse(to_device(text))
    assert p.info.status == 0 and p.info.format == g.GERBIL_FORMAT_FASTQ
    assert p.info.n_reads == o.size - 1 and p.info.n_bytes == int(o[-1]) and p.info.n_lines == 4 * (o.size - 1)
    import torch
    assert torch.equal(p.seq, torch.from_numpy(a).cuda())
    assert torch.equal(p.offsets, torch.from_numpy(o.view(np.int64)).cuda())


@pytest.mark.parametrize("seq_shift", [1, 5, 12])
def test_unaligned_output_buffer(seq_shift):
    import torch
    a, o = synthetic_reads(40 + seq_shift, 600, 300)
    text = synth.to_fasta(a, o, width=33)
    ref = oracle.parse_reads(text)
    d = to_device(text, shift=seq_shift + 2)
    n = len(text)
    lines = ref.n_lines
    ws = torch.empty(g.gerbil_parse_workspace(n, lines), dtype=torch.uint8, device="cuda")
    buf = torch.full((ref.n_bytes + 64,), 0x33, dtype=torch.uint8, device="cuda")
    seq = buf[seq_shift:]
    off = torch.empty(lines + 1, dtype=torch.int64, device="cuda")
    info = torch.zeros(ctypes_size(), dtype=torch.uint8, device="cuda")
    st = g.gerbil_parse(d.data_ptr(), n, 0, ws.data_ptr(), ws.numel(), lines, seq.data_ptr(), ref.n_bytes,
                        off.data_ptr(), lines, info.data_ptr(), int(torch.cuda.current_stream().cuda_stream))
    assert st == g.GERBIL_OK
    r = g.gerbil_parsed.from_buffer_copy(info.cpu().numpy().tobytes())
    assert r.status == 0
    b = buf.cpu().numpy()
    assert (b[:seq_shift] == 0x33).all() and (b[seq_shift + ref.n_bytes:] == 0x33).all()
    assert np.array_equal(b[seq_shift: seq_shift + ref.n_bytes], ref.ascii)

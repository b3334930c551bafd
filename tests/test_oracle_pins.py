"""Pins of the CPU oracle against what the paper and plain mathematics fix.

None of these tests re-types the oracle's own formulas. They use:
  * worked examples printed in the paper (tests/golden/, each with its passage);
  * brute force in pure Python on tiny inputs (dict of substrings);
  * closed forms (de Bruijn sequences contain every k-mer exactly once);
  * invariants that hold for any input (total count = valid windows, reverse
    complement invariance, palindromes only for even k, threshold sums).
"""
import itertools
import random

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle
import synth
from conftest import read_golden

COMP = {"A": "T", "C": "G", "G": "C", "T": "A"}


def reads_to_csr(reads):
    data = "".join(reads).encode()
    offs = np.zeros(len(reads) + 1, dtype=np.uint64)
    offs[1:] = np.cumsum([len(r) for r in reads])
    return np.frombuffer(data, dtype=np.uint8).copy(), offs


def rc(s):
    return "".join(COMP[c] for c in reversed(s))


def brute_force(reads, k, canonical=True):
    """dict canonical k-mer string -> count, straight from the definition."""
    out = {}
    for r in reads:
        for i in range(len(r) - k + 1):
            w = r[i:i + k]
            if any(c not in "ACGTacgt" for c in w):
                continue
            w = w.upper()
            if canonical:
                w = min(w, rc(w))   # Python compares 'A'<'C'<'G'<'T'
            out[w] = out.get(w, 0) + 1
    return out


def oracle_dict(res):
    return {oracle.decode_key(res.keys[i], res.k): int(res.counts[i]) for i in range(res.counts.size)}


def de_bruijn(k):
    """Linearised de Bruijn sequence B(4, k) (FKM algorithm) over ACGT."""
    a = [0] * (4 * k)
    seq = []

    def db(t, p):
        if t > k:
            if k % p == 0:
                seq.extend(a[1:p + 1])
        else:
            a[t] = a[t - p]
            db(t + 1, p)
            for j in range(a[t - p] + 1, 4):
                a[t] = j
                db(t + 1, t)

    db(1, 1)
    s = "".join("ACGT"[x] for x in seq)
    return s + s[: k - 1]


# ------------------------------------------------------------ worked examples

def test_reverse_complement_worked_example():
    (line,) = read_golden("rc_pair.txt")
    kmer, rcomp, canon = line.split()
    a, o = reads_to_csr([kmer, rcomp])
    res = oracle.count(a, o, k=4, threshold=1)
    assert oracle_dict(res) == {canon: 2}
    assert res.n_valid == 2


def _fig1():
    lines = dict(ln.split(None, 1) for ln in read_golden("fig1_supermers.txt"))
    return lines["sequence"], int(lines["k"]), int(lines["m"]), lines["supermers"].split()


@pytest.mark.parametrize("order", [0, 1])
def test_fig1_supermers(order):
    seq, k, m, expect = _fig1()
    a, o = reads_to_csr([seq])
    sm = oracle.supermers(a, o, k=k, m=m, n_bins=4, order=order)
    got = [seq[int(s): int(s) + int(n) + k - 1] for s, n in zip(sm["start"], sm["n_kmers"])]
    assert got == expect


def test_fig5_layout_is_a_key_plus_counter():
    d = dict(ln.split() for ln in read_golden("fig5_layout.txt"))
    k = int(d["k"])
    # a 3-mer needs 6 bits of 2-bit code: it fits the 4-byte key of the figure
    assert 2 * k <= 8 * int(d["key_bytes"])
    assert int(d["scan_bytes"]) // (int(d["key_bytes"]) + int(d["counter_bytes"])) == int(d["entries_per_scan"])


def test_output_records_worked_examples():
    for line in read_golden("records.txt"):
        parts = line.split()
        count, kmer, bits = int(parts[0]), parts[1], "".join(parts[2:])
        got = oracle.record(kmer, count)
        assert len(got) * 8 == len(bits)
        got_bits = "".join(f"{b:08b}" for b in got)
        for g, e in zip(got_bits, bits):
            if e != "X":
                assert g == e, (kmer, got_bits, bits)


# ------------------------------------------------------------- brute force

def random_reads(rng, n, max_len, n_rate=0.1, lower_rate=0.1):
    out = []
    for _ in range(n):
        L = rng.randint(0, max_len)
        s = []
        for _ in range(L):
            u = rng.random()
            if u < n_rate:
                s.append(rng.choice("NnRY."))
            else:
                c = rng.choice("ACGT")
                s.append(c.lower() if rng.random() < lower_rate else c)
        out.append("".join(s))
    return out


@pytest.mark.parametrize("seed", range(6))
def test_count_matches_brute_force(seed):
    rng = random.Random(seed)
    reads = random_reads(rng, 40, 60)
    a, o = reads_to_csr(reads)
    for k in range(1, 13):
        for canonical in (True, False):
            res = oracle.count(a, o, k=k, threshold=1, canonical=canonical)
            assert oracle_dict(res) == brute_force(reads, k, canonical), (k, canonical)


def test_multiword_keys_match_brute_force():
    rng = random.Random(11)
    reads = random_reads(rng, 30, 260, n_rate=0.005)
    reads += ["A" * 120, "T" * 90, "ACGT" * 50]
    a, o = reads_to_csr(reads)
    for k in (31, 32, 33, 63, 64, 65, 96, 99, 128, 200):
        res = oracle.count(a, o, k=k, threshold=1)
        assert oracle_dict(res) == brute_force(reads, k), k


def test_key_layout_words():
    # a 33-mer: 32 bases in word 0 (first base in bits 63:62), 1 base right-aligned in word 1
    s = "C" + "A" * 31 + "G"
    a, o = reads_to_csr([s])
    res = oracle.count(a, o, k=33, threshold=1, canonical=False)
    assert res.keys.shape == (1, 2)
    assert int(res.keys[0, 0]) == 1 << 62
    assert int(res.keys[0, 1]) == 2


def test_threshold_is_inclusive():
    reads = ["ACGTTGCA", "ACGTTGCA", "TTTTT"]
    a, o = reads_to_csr(reads)
    bf = brute_force(reads, 4)
    for t in range(1, 6):
        res = oracle.count(a, o, k=4, threshold=t)
        assert oracle_dict(res) == {x: c for x, c in bf.items() if c >= t}


# ------------------------------------------------------------- closed forms

@pytest.mark.parametrize("k", [3, 4, 5, 6, 7])
def test_de_bruijn_histogram(k):
    s = de_bruijn(k)
    assert len(s) == 4 ** k + k - 1
    a, o = reads_to_csr([s])
    res = oracle.count(a, o, k=k, threshold=1)
    h = res.folded_hist(4)
    if k % 2 == 0:
        pal = 4 ** (k // 2)
        assert int(h[1]) == pal and int(h[2]) == (4 ** k - pal) // 2
    else:
        assert int(h[1]) == 0 and int(h[2]) == 4 ** k // 2
    if k == 4:
        assert (int(h[1]), int(h[2])) == (16, 120)
    if k == 5:
        assert (int(h[1]), int(h[2])) == (0, 512)


@pytest.mark.parametrize("L,k", [(50, 8), (40, 32), (100, 33), (130, 65)])
def test_homopolymers(L, k):
    a, o = reads_to_csr(["A" * L, "T" * L])
    res = oracle.count(a, o, k=k, threshold=1)
    assert res.counts.tolist() == [2 * (L - k + 1)]
    assert oracle.decode_key(res.keys[0], k) == "A" * k


# --------------------------------------------------------------- invariants

def n_valid_windows(reads, k):
    return sum(1 for r in reads for i in range(len(r) - k + 1) if all(c in "ACGTacgt" for c in r[i:i + k]))


read_strategy = st.lists(st.text(alphabet="ACGTACGTACGTNacgt", min_size=0, max_size=80), min_size=1, max_size=12)


@settings(max_examples=60, deadline=None)
@given(reads=read_strategy, k=st.integers(1, 40), t=st.integers(1, 4))
def test_invariants(reads, k, t):
    a, o = reads_to_csr(reads)
    res = oracle.count(a, o, k=k, threshold=t)
    hist = res.hist.astype(np.int64)
    c = np.arange(hist.size)
    # total count = number of N-free windows
    assert int((c * hist).sum()) == n_valid_windows(reads, k) == res.n_valid
    # threshold sums
    assert int(hist[t:].sum()) == res.counts.size
    assert int((c[t:] * hist[t:]).sum()) == int(res.counts.astype(np.int64).sum())
    # reverse-complementing every read changes nothing
    rcr = ["".join(COMP.get(ch.upper(), ch) for ch in reversed(r)) for r in reads]
    a2, o2 = reads_to_csr(rcr)
    res2 = oracle.count(a2, o2, k=k, threshold=t)
    assert np.array_equal(res.keys, res2.keys) and np.array_equal(res.counts, res2.counts)
    assert np.array_equal(res.hist, res2.hist)
    # palindromes (x == rc(x)) only for even k
    if k % 2 == 1:
        for i in range(res.counts.size):
            s = oracle.decode_key(res.keys[i], k)
            assert s != rc(s)


def test_palindromes_exist_for_even_k():
    a, o = reads_to_csr(["ACGT", "AATT", "GATC"])
    res = oracle.count(a, o, k=4, threshold=1)
    assert sorted(oracle_dict(res)) == ["AATT", "ACGT", "GATC"]
    assert res.counts.tolist() == [1, 1, 1]


# ------------------------------------------------------------ other entries

def test_encode_against_python():
    rng = random.Random(3)
    reads = random_reads(rng, 25, 90, n_rate=0.05)
    a, o = reads_to_csr(reads)
    for k in (1, 5, 32, 33):
        packed, ok, nv = oracle.encode(a, o, k)
        text = "".join(reads)
        for i, ch in enumerate(text):
            code = "ACGT".index(ch.upper()) if ch in "ACGTacgt" else 0
            assert (int(packed[i // 32]) >> (62 - 2 * (i % 32))) & 3 == code
        want = set()
        pos = 0
        for r in reads:
            for i in range(len(r) - k + 1):
                if all(c in "ACGTacgt" for c in r[i:i + k]):
                    want.add(pos + i)
            pos += len(r)
        got = {i for i in range(len(text)) if (int(ok[i // 64]) >> (i % 64)) & 1}
        assert got == want and nv == len(want)


def _py_rank(u, order):
    c = min(u, rc(u))
    code = 0
    for ch in c:
        code = code * 4 + "ACGT".index(ch)
    if order == 0 and len(u) >= 3 and c[:3] in ("AAA", "ACA"):
        return code + 4 ** len(u)
    return code


@pytest.mark.parametrize("order", [0, 1])
def test_supermers_against_python(order):
    rng = random.Random(5 + order)
    reads = random_reads(rng, 30, 120, n_rate=0.02, lower_rate=0.0)
    a, o = reads_to_csr(reads)
    k, m, nb = 15, 5, 7
    sm = oracle.supermers(a, o, k=k, m=m, n_bins=nb, order=order)
    # expand the oracle's super-mers to one minimizer per window
    got = {}
    for s, n, b, r in zip(sm["start"], sm["n_kmers"], sm["bin"], sm["rank"]):
        for j in range(int(n)):
            got[int(s) + j] = (int(r), int(b))
    want = {}
    pos = 0
    for read in reads:
        for i in range(len(read) - k + 1):
            w = read[i:i + k]
            if all(c in "ACGT" for c in w):
                mr = min(_py_rank(w[j:j + m], order) for j in range(k - m + 1))
                want[pos + i] = (mr, mr % nb)
        pos += len(read)
    assert got == want
    # super-mers are maximal: consecutive pieces never continue each other
    for i in range(1, len(sm["start"])):
        prev_end = int(sm["start"][i - 1]) + int(sm["n_kmers"][i - 1])
        if prev_end == int(sm["start"][i]) and sm["rank"][i - 1] == sm["rank"][i]:
            # only allowed across a read boundary
            assert int(sm["start"][i]) in set(o.tolist())


def test_count_keys_matches_count():
    rng = random.Random(9)
    reads = random_reads(rng, 50, 70, n_rate=0.02)
    a, o = reads_to_csr(reads)
    res = oracle.count(a, o, k=9, threshold=1)
    sel = np.arange(0, res.counts.size, 3)
    got = oracle.count_keys(a, o, 9, res.keys[sel])
    assert np.array_equal(got, res.counts[sel].astype(np.uint64))


def test_shards_partition_the_result():
    rng = random.Random(2)
    reads = random_reads(rng, 60, 80, n_rate=0.02)
    a, o = reads_to_csr(reads)
    full = oracle.count(a, o, k=7, threshold=1)
    parts = [oracle.count(a, o, k=7, threshold=1, shard_mod=5, shard_id=s) for s in range(5)]
    merged = {}
    for p in parts:
        d = oracle_dict(p)
        assert not (set(d) & set(merged))
        merged.update(d)
        assert p.n_valid == full.n_valid
    assert merged == oracle_dict(full)
    assert sum(p.n_valid_shard for p in parts) == full.n_valid


@pytest.mark.parametrize("k", [3, 9, 15, 16, 17, 31, 32, 33, 65, 200])
def test_parallel_prefiltered_count_keys_matches_plain_count_keys(k):
    """The prefiltered, read-split key count is the plain one: queries hold
    present keys, absent keys and absent keys sharing a present key's prefix."""
    rng = random.Random(100 + k)
    reads = random_reads(rng, 120, k + 120, n_rate=0.01)
    reads = [r.lower() if i % 7 == 0 else r for i, r in enumerate(reads)]
    a, o = reads_to_csr(reads)
    res = oracle.count(a, o, k=k, threshold=1)
    present = res.keys[:: max(1, res.keys.shape[0] // 40)]
    W = present.shape[1]
    nrng = np.random.default_rng(k)
    absent = nrng.integers(0, 2**63, size=(20, W), dtype=np.int64).view(np.uint64)
    r_last = k - 32 * (W - 1)
    if r_last < 32:
        absent[:, -1] &= np.uint64((1 << (2 * r_last)) - 1)
    near = present[:10].copy()
    near[:, -1] ^= np.uint64(1)   # same prefix, last base changed
    query = np.unique(np.concatenate([present, absent, near]), axis=0)
    want = oracle.count_keys(a, o, k, query)
    got = oracle.count_keys_parallel(a, o, k, query, threads=3)
    assert np.array_equal(got, want)
    assert (want > 0).sum() >= present.shape[0] // 2


# ------------------------------------------------------------- input parsing

def parsed_reads(p):
    return [bytes(p.ascii[int(p.offsets[i]): int(p.offsets[i + 1])]) for i in range(p.offsets.size - 1)]


def test_parse_hand_written_fasta():
    text = b">r1 first\nACG\nTN\n>r2\n>r3\r\nGG\r\nca\r\n\n>r4\nA"
    p = oracle.parse_reads(text)
    assert p.fmt == oracle.FASTA and p.status == 0
    assert parsed_reads(p) == [b"ACGTN", b"", b"GGca", b"A"]
    assert p.n_lines == 10 and p.n_bytes == 10


def test_parse_hand_written_fastq():
    # quality lines that start with '@' and '+' are still quality lines
    text = b"@a\nACGT\n+\n@@+!\n@b x\nNN\n+b x\n>+\n@c\n\n+\n\n"
    p = oracle.parse_reads(text)
    assert p.fmt == oracle.FASTQ and p.status == 0
    assert parsed_reads(p) == [b"ACGT", b"NN", b""]
    assert p.n_lines == 12


def test_parse_errors():
    assert oracle.parse_reads(b"").status == 0 and oracle.parse_reads(b"").offsets.tolist() == [0]
    assert oracle.parse_reads(b"ACGT\n").status == oracle.PARSE_EFORMAT
    assert oracle.parse_reads(b"@a\nAC\n+\nII\n@b\nAC\n").status == oracle.PARSE_ELINES
    assert oracle.parse_reads(b"@a\nAC\n-\nII\n").status == oracle.PARSE_EPLUS
    assert oracle.parse_reads(b"@a\nAC\n+\nIII\n").status == oracle.PARSE_EQUAL
    assert oracle.parse_reads(b"@a\nAC\n+\nII\nb\nAC\n+\nII\n").status == oracle.PARSE_EHEADER
    assert oracle.parse_reads(b"AC\n>a\nAC\n", fmt=oracle.FASTA).status == oracle.PARSE_EORPHAN
    # blank lines before the first header are not orphans
    assert oracle.parse_reads(b"\n\n>a\nAC\n", fmt=oracle.FASTA).status == 0


@pytest.mark.parametrize("crlf", [False, True])
def test_parse_round_trips_the_writers(crlf):
    """The writers in the input generator and the parser are independent: a
    rendering parses back to the reads it was made from."""
    rng = random.Random(5)
    reads = random_reads(rng, 300, 400) + [""]
    a = np.frombuffer("".join(reads).encode(), dtype=np.uint8)
    o = np.zeros(len(reads) + 1, dtype=np.uint64)
    o[1:] = np.cumsum([len(r) for r in reads])
    p = oracle.parse_reads(synth.to_fastq(a, o, seed=3, crlf=crlf))
    assert p.status == 0 and p.fmt == oracle.FASTQ
    assert np.array_equal(p.ascii, a) and np.array_equal(p.offsets, o)
    for width, blank in ((60, False), (1, True), (0, False), (77, True)):
        p = oracle.parse_reads(synth.to_fasta(a, o, width=width, crlf=crlf, blank_lines=blank))
        assert p.status == 0 and p.fmt == oracle.FASTA
        assert np.array_equal(p.ascii, a) and np.array_equal(p.offsets, o)


# ------------------------------------------------------------ minimizer orders

def ranked_strings(table, m):
    codes = [c for c in range(4 ** m) if table[c] != oracle.NOT_CANONICAL]
    return [oracle.mmer_string(c, m) for c in sorted(codes, key=lambda c: int(table[c]))]


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5, 6])
def test_canonical_code_count(m):
    # odd m: no m-mer is its own reverse complement; even m: 4^(m/2) are
    expect = 4 ** m // 2 if m % 2 else (4 ** m + 2 ** m) // 2
    assert len(oracle.canonical_codes(m)) == expect
    t = oracle.order_table(oracle.RANKS_LEX, m)
    assert sum(int(x) != oracle.NOT_CANONICAL for x in t) == expect


def test_cgat_order_by_hand():
    # C < G < A < T, first base first (Sec. 3.1)
    assert ranked_strings(oracle.order_table(oracle.RANKS_CGAT, 2), 2) == \
        ["CC", "CG", "CA", "GC", "GA", "AC", "AG", "AA", "AT", "TA"]


def test_roberts_order_by_hand():
    # the second base complemented, then C < A < T < G
    assert ranked_strings(oracle.order_table(oracle.RANKS_ROBERTS, 2), 2) == \
        ["CG", "CA", "CC", "AG", "AT", "AA", "AC", "TA", "GA", "GC"]
    # the paper names CGCGCG as the kind of minimizer this order prefers
    t = oracle.order_table(oracle.RANKS_ROBERTS, 6)
    assert ranked_strings(t, 6)[0] == "CGCGCG"


def test_splitmix64_published_outputs():
    # the first three outputs of SplitMix64 from state 0
    assert [oracle.splitmix64(0, i) for i in range(3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
                                                          0x06C45D188009454F]


@pytest.mark.parametrize("m", [3, 4, 7])
def test_random_order_is_a_seeded_permutation(m):
    canon = oracle.canonical_codes(m)
    t1 = oracle.order_table(oracle.RANKS_RANDOM, m, seed=1)
    t2 = oracle.order_table(oracle.RANKS_RANDOM, m, seed=2)
    assert sorted(int(t1[c]) for c in canon) == list(range(len(canon)))
    assert not np.array_equal(t1, t2)
    # ranks follow the generator's values
    keys = sorted((oracle.splitmix64(1, c) >> 34, c) for c in canon)
    assert [int(t1[c]) for _, c in keys] == list(range(len(canon)))


def test_dfp_by_hand():
    # m = 1: canonical A and C; C is the rarer
    f = {0: 5, 1: 3}
    t0 = oracle.order_table(oracle.RANKS_DFP, 1, pivot=0.0, freq=f)
    assert (int(t0[1]), int(t0[0])) == (0, 1)       # pivot 0: rare first
    t1 = oracle.order_table(oracle.RANKS_DFP, 1, pivot=1.0, freq=f)
    assert (int(t1[0]), int(t1[1])) == (0, 1)       # pivot 1: common first
    # m = 2, no samples: frequency order is code order; pivot 0.5 of M = 10 is position 5
    t = oracle.order_table(oracle.RANKS_DFP, 2, pivot=0.5, freq={})
    canon = oracle.canonical_codes(2)
    by_rank = sorted(canon, key=lambda c: int(t[c]))
    assert [canon.index(c) for c in by_rank] == [5, 4, 6, 3, 7, 2, 8, 1, 9, 0]


def test_dfp_frequency_sample_by_hand():
    a = np.frombuffer(b"ACGTACxAC", dtype=np.uint8)
    o = np.array([0, 6, 9], dtype=np.uint64)
    # 3-windows of read 0 start with AC, CG, GT, TA; read 1 has no valid window
    AC, CG, TA = 0b0001, 0b0110, 0b1100
    assert oracle.mmer_frequencies(a, o, 3, 2, 1) == {AC: 2, CG: 1, TA: 1}
    assert oracle.mmer_frequencies(a, o, 3, 2, 2) == {AC: 2}


@pytest.mark.parametrize("kind,order", [(0, 0), (1, 1)])
def test_table_order_reproduces_the_arithmetic_orders(kind, order):
    """The table path of the super-mer oracle, fed the Python tables of KMC2
    and LEX, gives the C oracle's own super-mers for those orders."""
    rng = random.Random(77)
    reads = random_reads(rng, 60, 200)
    a = np.frombuffer("".join(reads).encode(), dtype=np.uint8)
    o = np.zeros(len(reads) + 1, dtype=np.uint64)
    o[1:] = np.cumsum([len(r) for r in reads])
    for k, m in ((15, 5), (31, 7)):
        ref = oracle.supermers(a, o, k, m, 37, order=order)
        got = oracle.supermers(a, o, k, m, 37, order=2, rank_table=oracle.order_table(kind, m))
        for key in ("start", "n_kmers", "bin", "rank"):
            assert np.array_equal(ref[key], got[key]), key

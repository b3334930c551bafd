"""ctypes binding of libgerbil.so (the C ABI in include/gerbil.h).

Every function here marshals arguments and calls the library; all steps of
the counting path run in the HIP kernels behind the C ABI. PyTorch supplies
device memory and streams only. If the shared library is missing the import
of the library fails loudly: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("GERBIL_LIBRARY", os.path.join(_HERE, "libgerbil.so"))

GERBIL_OK = 0
GERBIL_EINVAL = -1
GERBIL_EUNSUPPORTED = -2
GERBIL_ECAPACITY = -3
GERBIL_EDEVICE = -4

GERBIL_PLAIN = 0
GERBIL_BATCHED = 1
GERBIL_ORDER_KMC2 = 0
GERBIL_ORDER_LEX = 1
GERBIL_ORDER_TABLE = 2
GERBIL_RANKS_KMC2 = 0
GERBIL_RANKS_LEX = 1
GERBIL_RANKS_CGAT = 2
GERBIL_RANKS_ROBERTS = 3
GERBIL_RANKS_RANDOM = 4
GERBIL_RANKS_DFP = 5
GERBIL_TABLE_AUTO = 0
GERBIL_TABLE_HBM = 1
GERBIL_TABLE_LDS = 2
GERBIL_CEIL_LDS_CAS = 0
GERBIL_CEIL_LDS_ADD = 1
GERBIL_CEIL_HBM_ADD = 2
GERBIL_CEIL_HBM_CAS = 3
GERBIL_CEIL_HBM_LOAD = 4
GERBIL_CEIL_ONE_ADDR = 5
GERBIL_PROBE_HIST = 32
GERBIL_FORMAT_DETECT = 0
GERBIL_FORMAT_FASTQ = 1
GERBIL_FORMAT_FASTA = 2
GERBIL_PARSE_EHEADER = 0x001
GERBIL_PARSE_EPLUS = 0x002
GERBIL_PARSE_EQUAL = 0x004
GERBIL_PARSE_ELINES = 0x008
GERBIL_PARSE_EORPHAN = 0x010
GERBIL_PARSE_EBYTES = 0x020
GERBIL_PARSE_EREADS = 0x040
GERBIL_PARSE_EFORMAT = 0x080
GERBIL_PARSE_ELINECAP = 0x100

# device status bits (see gerbil_report.status)
ST_OUT_CAP = 0x1
ST_OVF_CAP = 0x2
ST_SUPERM_CAP = 0x4
ST_COUNT_SAT = 0x8
ST_SPIN = 0x10
ST_OFFSETS = 0x20
ST_POOL = 0x40

u32, u64, f32, vp = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_float, ctypes.c_void_p


class gerbil_params(ctypes.Structure):
    _fields_ = [("k", u32), ("m", u32), ("n_bins", u32), ("threshold", u32), ("canonical", u32),
                ("order", u32), ("bin_map", vp), ("mode", u32), ("table", u32), ("load_factor", f32),
                ("max_probes", u32), ("block", u32), ("pool", u32), ("overflow_cap", u64),
                ("superm_cap", u64), ("table_budget", u64), ("timing_events", vp), ("stage_clocks", vp),
                ("size_sample", u32), ("reserved0", u32), ("rank_table", vp), ("probe_hist", vp)]


class gerbil_encoded(ctypes.Structure):
    _fields_ = [("n_reads", u64), ("n_bytes", u64), ("k", u32), ("reserved", u32), ("n_words", u64),
                ("n_mask", u64), ("packed", vp), ("valid", vp), ("read_start", vp), ("kmer_ok", vp),
                ("n_valid", vp), ("status", vp)]


class gerbil_bins(ctypes.Structure):
    _fields_ = [("k", u32), ("m", u32), ("n_bins", u32), ("tile", u32), ("cap_superm", u64), ("n_bytes", u64),
                ("packed", vp), ("desc", vp), ("bin_off", vp), ("bin_kmers", vp), ("n_superm", vp),
                ("status", vp)]


class gerbil_counted(ctypes.Structure):
    _fields_ = [("k", u32), ("W", u32), ("threshold", u32), ("hist_len", u32), ("cap", u64),
                ("overflow_cap", u64), ("n_out", vp), ("hist", vp), ("n_overflow", vp), ("max_count", vp),
                ("status", vp), ("n_superm", vp), ("bin_status", vp)]


class gerbil_report(ctypes.Structure):
    _fields_ = [("n_valid", u64), ("n_superm", u64), ("n_out", u64), ("n_overflow", u64), ("max_count", u64),
                ("status", u32), ("reserved", u32)]


class gerbil_pipeline(ctypes.Structure):
    _fields_ = [("ascii", vp), ("offsets", vp), ("n_reads", u64), ("n_bytes", u64), ("ws_encode", vp),
                ("ws_encode_bytes", u64), ("ws_bin", vp), ("ws_bin_bytes", u64), ("ws_count", vp),
                ("ws_count_bytes", u64), ("keys", vp), ("counts", vp), ("cap", u64), ("hist", vp),
                ("hist_len", u32), ("reserved", u32)]


class gerbil_tune_result(ctypes.Structure):
    _fields_ = [("table", u32), ("load_factor", f32), ("pool", u32), ("candidates", u32), ("cached", u32),
                ("best_ms", f32), ("block", u32)]


class gerbil_parsed(ctypes.Structure):
    _fields_ = [("n_reads", u64), ("n_bytes", u64), ("n_lines", u64), ("status", u32), ("format", u32)]


class GerbilError(RuntimeError):
    def __init__(self, fn: str, status: int, report: Optional[gerbil_report] = None):
        self.status = status
        self.report = report
        msg = f"{fn} failed: {status_string(status)} ({status})"
        if report is not None:
            msg += (f"; device status 0x{report.status:x}, n_out={report.n_out}, n_superm={report.n_superm}, "
                    f"n_overflow={report.n_overflow}")
        super().__init__(msg)


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libgerbil.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path} is missing: build the HIP library first "
                                f"(python -m paper_1607_06618_amd.build)")
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    lib.gerbil_version.restype = u32
    lib.gerbil_version.argtypes = []
    lib.gerbil_status_string.restype = ctypes.c_char_p
    lib.gerbil_status_string.argtypes = [ctypes.c_int32]
    lib.gerbil_encode_workspace.argtypes = [u64, u64, u32, P(u64)]
    lib.gerbil_encode.argtypes = [vp, vp, u64, u64, u32, vp, u64, P(gerbil_encoded), vp]
    lib.gerbil_bin_workspace.argtypes = [P(gerbil_encoded), P(gerbil_params), P(u64)]
    lib.gerbil_bin.argtypes = [P(gerbil_encoded), P(gerbil_params), vp, u64, P(gerbil_bins), vp]
    lib.gerbil_count_workspace.argtypes = [P(gerbil_bins), P(gerbil_params), P(u64), vp]
    lib.gerbil_count.argtypes = [P(gerbil_bins), P(gerbil_params), vp, u64, vp, vp, u64, P(gerbil_counted), vp]
    lib.gerbil_histogram.argtypes = [P(gerbil_counted), vp, u32, vp]
    lib.gerbil_result.argtypes = [P(gerbil_encoded), P(gerbil_bins), P(gerbil_counted), P(gerbil_report), vp]
    lib.gerbil_graph_capture.argtypes = [P(gerbil_pipeline), P(gerbil_params), P(gerbil_encoded), P(gerbil_bins),
                                         P(gerbil_counted), vp, P(vp)]
    lib.gerbil_graph_launch.argtypes = [vp, vp]
    lib.gerbil_graph_info.argtypes = [vp, P(u32), P(u32)]
    lib.gerbil_graph_destroy.argtypes = [vp]
    lib.gerbil_autotune_workspace.argtypes = [P(gerbil_bins), P(gerbil_params), P(u64), vp]
    lib.gerbil_autotune.argtypes = [P(gerbil_bins), P(gerbil_params), vp, u64, vp, vp, u64, P(gerbil_params),
                                    P(gerbil_tune_result), vp]
    lib.gerbil_autotune_reset.argtypes = []
    lib.gerbil_records_workspace.argtypes = [u64, P(u64)]
    lib.gerbil_records.argtypes = [vp, vp, u64, u32, vp, u64, vp, u64, vp, vp]
    lib.gerbil_records_noalloc.argtypes = [vp, vp, u64, u32, vp, u64, vp, vp]
    lib.gerbil_parse_workspace.argtypes = [u64, u64, P(u64)]
    lib.gerbil_order_table_workspace.argtypes = [u32, u32, P(u64)]
    lib.gerbil_key_bins.argtypes = [vp, u64, P(gerbil_params), vp, vp]
    lib.gerbil_hll_bins.argtypes = [P(gerbil_bins), P(gerbil_params), u32, vp, vp]
    lib.gerbil_order_table.argtypes = [u32, u32, u64, f32, u32, P(gerbil_encoded), vp, u64, vp, vp]
    lib.gerbil_parse.argtypes = [vp, u64, u32, vp, u64, u64, vp, u64, vp, u64, vp, vp]
    lib.gerbil_ceiling.argtypes = [u32, vp, u64, u32, u32, vp, vp]
    for name in ("gerbil_encode_workspace", "gerbil_encode", "gerbil_bin_workspace", "gerbil_bin",
                 "gerbil_count_workspace", "gerbil_count", "gerbil_histogram", "gerbil_result",
                 "gerbil_graph_capture", "gerbil_graph_launch", "gerbil_graph_info", "gerbil_graph_destroy",
                 "gerbil_autotune_workspace", "gerbil_autotune", "gerbil_autotune_reset",
                 "gerbil_records_workspace", "gerbil_records", "gerbil_records_noalloc", "gerbil_parse_workspace", "gerbil_parse",
                 "gerbil_order_table_workspace", "gerbil_order_table", "gerbil_key_bins",
                 "gerbil_hll_bins", "gerbil_ceiling"):
        getattr(lib, name).restype = ctypes.c_int32
    _lib = lib
    return lib


# ------------------------------------------------------------ C-ABI names

def gerbil_version() -> int:
    return int(load().gerbil_version())


def status_string(status: int) -> str:
    return load().gerbil_status_string(status).decode()


gerbil_status_string = status_string


def gerbil_encode_workspace(n_reads: int, n_bytes: int, k: int) -> int:
    out = u64(0)
    st = load().gerbil_encode_workspace(n_reads, n_bytes, k, ctypes.byref(out))
    if st:
        raise GerbilError("gerbil_encode_workspace", st)
    return out.value


def gerbil_encode(ascii_ptr: int, offsets_ptr: int, n_reads: int, n_bytes: int, k: int, ws_ptr: int,
                  ws_bytes: int, out: gerbil_encoded, stream: int = 0) -> int:
    return load().gerbil_encode(ascii_ptr, offsets_ptr, n_reads, n_bytes, k, ws_ptr, ws_bytes, ctypes.byref(out),
                                stream)


def gerbil_bin_workspace(enc: gerbil_encoded, p: gerbil_params) -> int:
    out = u64(0)
    st = load().gerbil_bin_workspace(ctypes.byref(enc), ctypes.byref(p), ctypes.byref(out))
    if st:
        raise GerbilError("gerbil_bin_workspace", st)
    return out.value


def gerbil_bin(enc: gerbil_encoded, p: gerbil_params, ws_ptr: int, ws_bytes: int, out: gerbil_bins,
               stream: int = 0) -> int:
    return load().gerbil_bin(ctypes.byref(enc), ctypes.byref(p), ws_ptr, ws_bytes, ctypes.byref(out), stream)


def gerbil_count_workspace(bins: gerbil_bins, p: gerbil_params, stream: int = 0) -> int:
    out = u64(0)
    st = load().gerbil_count_workspace(ctypes.byref(bins), ctypes.byref(p), ctypes.byref(out), stream)
    if st:
        raise GerbilError("gerbil_count_workspace", st)
    return out.value


def gerbil_count(bins: gerbil_bins, p: gerbil_params, ws_ptr: int, ws_bytes: int, keys_ptr: int, counts_ptr: int,
                 cap: int, state: gerbil_counted, stream: int = 0) -> int:
    return load().gerbil_count(ctypes.byref(bins), ctypes.byref(p), ws_ptr, ws_bytes, keys_ptr, counts_ptr, cap,
                               ctypes.byref(state), stream)


def gerbil_histogram(state: gerbil_counted, hist_ptr: int, length: int, stream: int = 0) -> int:
    return load().gerbil_histogram(ctypes.byref(state), hist_ptr, length, stream)


def gerbil_result(enc: Optional[gerbil_encoded], bins: Optional[gerbil_bins], state: Optional[gerbil_counted],
                  stream: int = 0):
    rep = gerbil_report()
    st = load().gerbil_result(ctypes.byref(enc) if enc is not None else None,
                              ctypes.byref(bins) if bins is not None else None,
                              ctypes.byref(state) if state is not None else None, ctypes.byref(rep), stream)
    return st, rep


def gerbil_graph_capture(pl: gerbil_pipeline, p: gerbil_params, enc: gerbil_encoded, bins: gerbil_bins,
                         state: gerbil_counted, stream: int):
    """Returns (status, graph handle or None)."""
    h = vp(0)
    st = load().gerbil_graph_capture(ctypes.byref(pl), ctypes.byref(p), ctypes.byref(enc), ctypes.byref(bins),
                                     ctypes.byref(state), stream, ctypes.byref(h))
    return st, (h.value if st == GERBIL_OK else None)


def gerbil_graph_launch(graph: int, stream: int) -> int:
    return load().gerbil_graph_launch(graph, stream)


def gerbil_graph_info(graph: int):
    n, nk = u32(0), u32(0)
    st = load().gerbil_graph_info(graph, ctypes.byref(n), ctypes.byref(nk))
    return st, n.value, nk.value


def gerbil_graph_destroy(graph: Optional[int]) -> int:
    return load().gerbil_graph_destroy(graph)


def gerbil_autotune_workspace(bins: gerbil_bins, p: gerbil_params, stream: int = 0) -> int:
    out = u64(0)
    st = load().gerbil_autotune_workspace(ctypes.byref(bins), ctypes.byref(p), ctypes.byref(out), stream)
    if st:
        raise GerbilError("gerbil_autotune_workspace", st)
    return out.value


def gerbil_autotune(bins: gerbil_bins, p: gerbil_params, ws_ptr: int, ws_bytes: int, keys_ptr: int,
                    counts_ptr: int, cap: int, stream: int = 0):
    """Returns (status, best params, tune result)."""
    best = gerbil_params()
    info = gerbil_tune_result()
    st = load().gerbil_autotune(ctypes.byref(bins), ctypes.byref(p), ws_ptr, ws_bytes, keys_ptr, counts_ptr, cap,
                                ctypes.byref(best), ctypes.byref(info), stream)
    return st, best, info


def gerbil_autotune_reset() -> int:
    return load().gerbil_autotune_reset()


def gerbil_records_workspace(n: int) -> int:
    out = u64(0)
    st = load().gerbil_records_workspace(n, ctypes.byref(out))
    if st:
        raise GerbilError("gerbil_records_workspace", st)
    return out.value


def gerbil_records(keys_ptr: int, counts_ptr: int, n: int, k: int, ws_ptr: int, ws_bytes: int, out_ptr: int,
                   out_cap: int, out_bytes_ptr: int, stream: int = 0) -> int:
    return load().gerbil_records(keys_ptr or None, counts_ptr or None, n, k, ws_ptr or None, ws_bytes,
                                 out_ptr or None, out_cap, out_bytes_ptr, stream)


GERBIL_RECORDS_NOALLOC_MAX = 1 << 29


def gerbil_records_noalloc(keys_ptr: int, counts_ptr: int, n: int, k: int, out_ptr: int, out_cap: int,
                           out_bytes_ptr: int, stream: int = 0) -> int:
    return load().gerbil_records_noalloc(keys_ptr or None, counts_ptr or None, n, k, out_ptr or None, out_cap,
                                         out_bytes_ptr or None, stream)


def records(keys_d, counts_d, n: int, k: int, stream=None):
    """The App. C record stream of n device pairs, as a device uint8 tensor."""
    import torch
    dev = counts_d.device
    s = _stream_handle(stream)
    ws = torch.empty(max(256, gerbil_records_workspace(n)), dtype=torch.uint8, device=dev)
    size_d = torch.zeros(1, dtype=torch.int64, device=dev)
    kb = (k + 3) // 4
    cap = n * (5 + kb)   # every record at its largest
    out = torch.empty(max(1, cap), dtype=torch.uint8, device=dev)
    check("gerbil_records", gerbil_records(keys_d.data_ptr(), counts_d.data_ptr(), n, k, ws.data_ptr(), ws.numel(),
                                           out.data_ptr(), cap, size_d.data_ptr(), s))
    if stream is not None:
        stream.synchronize()
    size = int(size_d.item())
    return out[:size]


def gerbil_key_bins(keys_ptr: int, n: int, params: gerbil_params, bins_ptr: int, stream: int = 0) -> int:
    return load().gerbil_key_bins(keys_ptr or None, n, ctypes.byref(params), bins_ptr or None, stream)


def gerbil_hll_bins(bins: gerbil_bins, params: gerbil_params, log2_regs: int, regs_ptr: int, stream: int = 0) -> int:
    return load().gerbil_hll_bins(ctypes.byref(bins), ctypes.byref(params), log2_regs, regs_ptr or None, stream)


def hll_registers(job, log2_regs: int = 12, stream=None):
    """HyperLogLog registers [n_bins, 2^log2_regs] of a binned job (device int32 tensor)."""
    import torch
    regs = torch.empty((job.bins.n_bins, 1 << log2_regs), dtype=torch.int32, device=job.ascii_d.device)
    check("gerbil_hll_bins", gerbil_hll_bins(job.bins, job.p, log2_regs, regs.data_ptr(), _stream_handle(stream)))
    return regs


def key_bins(keys_d, n: int, params: gerbil_params, stream=None):
    """Bin of each of the first n device keys under `params`' binning (device int32 tensor)."""
    import torch
    bins = torch.empty(max(1, n), dtype=torch.int32, device=keys_d.device)
    check("gerbil_key_bins", gerbil_key_bins(keys_d.data_ptr(), n, params, bins.data_ptr(), _stream_handle(stream)))
    return bins[:n]


def gerbil_ceiling(kind: int, buf_ptr: int, buf_bytes: int, grid: int, iters: int, sink_ptr: int,
                   stream: int = 0) -> int:
    return load().gerbil_ceiling(kind, buf_ptr or None, buf_bytes, grid, iters, sink_ptr or None, stream)


def ceiling(kind: int, grid: int, iters: int, buf_bytes: int = 0, repeats: int = 3, device="cuda"):
    """Operations per second of one access kind (GERBIL_CEIL_*): the best of
    `repeats` timed launches after one warm-up, timed with HIP events on the
    current stream. Returns (ops_per_s, ops_per_launch, ms_per_launch)."""
    import torch
    s = torch.cuda.current_stream()
    h = _stream_handle(s)
    sink = torch.empty(grid * 1024, dtype=torch.int64, device=device)
    buf = torch.zeros(max(64, buf_bytes) // 8, dtype=torch.int64, device=device) if buf_bytes else None
    bp, bb = (buf.data_ptr(), buf.numel() * 8) if buf is not None else (0, 0)
    ops = grid * (16 if kind == GERBIL_CEIL_ONE_ADDR else 1024) * iters
    check("gerbil_ceiling", gerbil_ceiling(kind, bp, bb, grid, iters, sink.data_ptr(), h))
    best = None
    for _ in range(repeats):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        check("gerbil_ceiling", gerbil_ceiling(kind, bp, bb, grid, iters, sink.data_ptr(), h))
        e1.record(s)
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    return ops / (best * 1e-3), ops, best


def gerbil_order_table_workspace(kind: int, m: int) -> int:
    out = u64(0)
    st = load().gerbil_order_table_workspace(kind, m, ctypes.byref(out))
    if st:
        raise GerbilError("gerbil_order_table_workspace", st)
    return out.value


def gerbil_order_table(kind: int, m: int, seed: int, pivot: float, stride: int, enc, ws_ptr: int, ws_bytes: int,
                       table_ptr: int, stream: int = 0) -> int:
    return load().gerbil_order_table(kind, m, seed, pivot, stride, ctypes.byref(enc) if enc is not None else None,
                                     ws_ptr or None, ws_bytes, table_ptr or None, stream)


def order_table(kind: int, m: int, seed: int = 0, pivot: float = 0.0, stride: int = 0, enc=None, device="cuda",
                stream=None):
    """Device rank table (uint32 [4^m], as an int32 tensor) of a minimizer order of Sec. 3.1."""
    import torch
    s = _stream_handle(stream)
    table = torch.empty(4 ** m, dtype=torch.int32, device=device)
    wsb = gerbil_order_table_workspace(kind, m)
    ws = torch.empty(max(256, wsb), dtype=torch.uint8, device=device)
    check("gerbil_order_table", gerbil_order_table(kind, m, seed, pivot, stride, enc, ws.data_ptr(), wsb,
                                                   table.data_ptr(), s))
    if stream is not None:
        stream.synchronize()
    else:
        torch.cuda.current_stream().synchronize()
    return table


def gerbil_parse_workspace(n: int, lines_cap: int) -> int:
    out = u64(0)
    st = load().gerbil_parse_workspace(n, lines_cap, ctypes.byref(out))
    if st:
        raise GerbilError("gerbil_parse_workspace", st)
    return out.value


def gerbil_parse(text_ptr: int, n: int, fmt: int, ws_ptr: int, ws_bytes: int, lines_cap: int, seq_ptr: int,
                 seq_cap: int, offsets_ptr: int, reads_cap: int, out_ptr: int, stream: int = 0) -> int:
    return load().gerbil_parse(text_ptr or None, n, fmt, ws_ptr or None, ws_bytes, lines_cap, seq_ptr or None,
                               seq_cap, offsets_ptr or None, reads_cap, out_ptr or None, stream)


@dataclass
class Parsed:
    seq: "object"        # device uint8 [n_bytes]: the reads back to back
    offsets: "object"    # device int64 [n_reads + 1]
    info: gerbil_parsed  # counts, status, format


def parse(text_d, fmt: int = GERBIL_FORMAT_DETECT, lines_cap: Optional[int] = None, stream=None) -> Parsed:
    """FASTA/FASTQ text in a device uint8 tensor -> CSR reads on the device.

    Starts from a guess of the line count and calls again with the exact
    count when the guess was too small."""
    import torch
    n = int(text_d.numel())
    dev = text_d.device
    s = _stream_handle(stream)
    cap = min(n + 1, lines_cap if lines_cap is not None else n // 32 + 1024)
    info_d = torch.zeros(ctypes.sizeof(gerbil_parsed), dtype=torch.uint8, device=dev)
    seq = torch.empty(max(1, n), dtype=torch.uint8, device=dev)
    for _ in range(2):
        ws = torch.empty(max(256, gerbil_parse_workspace(n, cap)), dtype=torch.uint8, device=dev)
        offsets = torch.empty(cap + 1, dtype=torch.int64, device=dev)
        check("gerbil_parse", gerbil_parse(text_d.data_ptr() if n else 0, n, fmt, ws.data_ptr(), ws.numel(), cap,
                                           seq.data_ptr(), n, offsets.data_ptr(), cap, info_d.data_ptr(), s))
        if stream is not None:
            stream.synchronize()
        info = gerbil_parsed.from_buffer_copy(info_d.cpu().numpy().tobytes())
        if not (info.status & GERBIL_PARSE_ELINECAP):
            break
        cap = int(info.n_lines)
    return Parsed(seq[: info.n_bytes], offsets[: info.n_reads + 1], info)


def check(fn: str, status: int):
    if status != GERBIL_OK:
        raise GerbilError(fn, status)


# ------------------------------------------------------- torch-side driver

def words(k: int) -> int:
    return (k + 31) // 32


def make_params(k: int, m: int, n_bins: int, threshold: int, mode: int = GERBIL_PLAIN, order: int = 0,
                bin_map_ptr: int = 0, load_factor: float = 0.0, max_probes: int = 0, block: int = 0,
                table: int = GERBIL_TABLE_AUTO, pool: int = 0, overflow_cap: int = 0, superm_cap: int = 0,
                table_budget: int = 0, timing_events: int = 0, stage_clocks: int = 0,
                size_sample: int = 0, canonical: bool = True, rank_table_ptr: int = 0,
                probe_hist: int = 0) -> gerbil_params:
    return gerbil_params(k=k, m=m, n_bins=n_bins, threshold=threshold, canonical=int(canonical), order=order,
                         bin_map=bin_map_ptr or None, mode=mode, table=table, load_factor=load_factor,
                         max_probes=max_probes, block=block, pool=pool, overflow_cap=overflow_cap,
                         superm_cap=superm_cap, table_budget=table_budget, timing_events=timing_events or None,
                         stage_clocks=stage_clocks or None, size_sample=size_sample,
                         rank_table=rank_table_ptr or None, probe_hist=probe_hist or None)


@dataclass
class CountResult:
    keys: np.ndarray      # uint64 [n, W], unspecified order
    counts: np.ndarray    # uint32 [n]
    hist: np.ndarray      # uint64 [hist_len]
    report: gerbil_report

    def sorted(self):
        """Pairs sorted by key (for comparisons)."""
        if self.keys.shape[0] == 0:
            return self.keys, self.counts
        order = np.lexsort(self.keys.T[::-1])
        return self.keys[order], self.counts[order]


def _stream_handle(stream) -> int:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


class Job:
    """Device buffers and C-ABI state of one counting run (encode -> bin -> count -> histogram).

    Workspaces are torch tensors on the current device; the library itself
    never allocates. ``run`` enqueues the whole path on ``stream``.
    """

    def __init__(self, ascii_d, offsets_d, n_bytes: int, params: gerbil_params, hist_len: int = 256,
                 cap: Optional[int] = None, stream=None):
        import torch
        self.torch = torch
        self.ascii_d, self.offsets_d = ascii_d, offsets_d
        self.n_reads = offsets_d.numel() - 1
        self.n_bytes = n_bytes
        self.p = params
        self.hist_len = hist_len
        self.W = words(params.k)
        self.stream = stream
        dev = ascii_d.device
        self.enc = gerbil_encoded()
        self.bins = gerbil_bins()
        self.state = gerbil_counted()
        self.ws_enc = torch.empty(gerbil_encode_workspace(self.n_reads, n_bytes, params.k), dtype=torch.uint8,
                                  device=dev)
        self.cap = cap
        self.ws_bin = None
        self.ws_count = None
        self.keys_d = None
        self.counts_d = None
        self.hist_d = torch.zeros(hist_len, dtype=torch.int64, device=dev)
        self.graph = None

    def encode(self):
        s = _stream_handle(self.stream)
        check("gerbil_encode", gerbil_encode(self.ascii_d.data_ptr(), self.offsets_d.data_ptr(), self.n_reads,
                                             self.n_bytes, self.p.k, self.ws_enc.data_ptr(), self.ws_enc.numel(),
                                             self.enc, s))

    def bin(self):
        torch = self.torch
        s = _stream_handle(self.stream)
        if self.ws_bin is None:
            self.ws_bin = torch.empty(gerbil_bin_workspace(self.enc, self.p), dtype=torch.uint8,
                                      device=self.ascii_d.device)
        check("gerbil_bin", gerbil_bin(self.enc, self.p, self.ws_bin.data_ptr(), self.ws_bin.numel(), self.bins, s))

    def prepare_count(self, n_valid: Optional[int] = None):
        """Size the count workspace and output arrays (synchronises once)."""
        torch = self.torch
        if self.ws_count is None:
            self.ws_count = torch.empty(gerbil_count_workspace(self.bins, self.p, _stream_handle(self.stream)),
                                        dtype=torch.uint8, device=self.ascii_d.device)
        if self.keys_d is None:
            if self.cap is None:
                if n_valid is None:
                    st, rep = gerbil_result(self.enc, None, None, _stream_handle(self.stream))
                    n_valid = rep.n_valid
                self.cap = max(1, n_valid // max(1, self.p.threshold) + 1)
            self.keys_d = torch.empty(self.cap * self.W, dtype=torch.int64, device=self.ascii_d.device)
            self.counts_d = torch.empty(self.cap, dtype=torch.int32, device=self.ascii_d.device)

    def count(self):
        s = _stream_handle(self.stream)
        check("gerbil_count", gerbil_count(self.bins, self.p, self.ws_count.data_ptr(), self.ws_count.numel(),
                                           self.keys_d.data_ptr(), self.counts_d.data_ptr(), self.cap, self.state, s))
        check("gerbil_histogram", gerbil_histogram(self.state, self.hist_d.data_ptr(), self.hist_len, s))

    def run(self):
        """Enqueue encode -> bin -> count -> histogram (sizes taken on the first call)."""
        self.encode()
        self.bin()
        if self.ws_count is None or self.keys_d is None:
            self.prepare_count()
        self.count()

    def autotune(self) -> gerbil_tune_result:
        """Choose table placement, fill, pool and workgroup shape by timing them on this job's bins
        (after encode and bin); the job then counts with the choice."""
        torch = self.torch
        s = _stream_handle(self.stream)
        need = gerbil_autotune_workspace(self.bins, self.p, s)
        if self.ws_count is None or self.ws_count.numel() < need:
            self.ws_count = torch.empty(need, dtype=torch.uint8, device=self.ascii_d.device)
        self.prepare_count()
        st, best, info = gerbil_autotune(self.bins, self.p, self.ws_count.data_ptr(), self.ws_count.numel(),
                                         self.keys_d.data_ptr(), self.counts_d.data_ptr(), self.cap, s)
        check("gerbil_autotune", st)
        self.p = best
        return info

    def pipeline(self) -> gerbil_pipeline:
        """Buffers of the whole path (sizes must have been taken by a first run)."""
        if self.ws_bin is None or self.ws_count is None or self.keys_d is None:
            raise RuntimeError("run the job once before capturing it: the count workspace is sized from the bins")
        return gerbil_pipeline(ascii=self.ascii_d.data_ptr(), offsets=self.offsets_d.data_ptr(),
                               n_reads=self.n_reads, n_bytes=self.n_bytes, ws_encode=self.ws_enc.data_ptr(),
                               ws_encode_bytes=self.ws_enc.numel(), ws_bin=self.ws_bin.data_ptr(),
                               ws_bin_bytes=self.ws_bin.numel(), ws_count=self.ws_count.data_ptr(),
                               ws_count_bytes=self.ws_count.numel(), keys=self.keys_d.data_ptr(),
                               counts=self.counts_d.data_ptr(), cap=self.cap, hist=self.hist_d.data_ptr(),
                               hist_len=self.hist_len)

    def capture(self):
        """Record encode -> bin -> count -> histogram into a HIP graph (batched mode, non-default stream)."""
        if self.graph is not None:
            gerbil_graph_destroy(self.graph)
            self.graph = None
        self._pl = self.pipeline()
        st, h = gerbil_graph_capture(self._pl, self.p, self.enc, self.bins, self.state, _stream_handle(self.stream))
        check("gerbil_graph_capture", st)
        self.graph = h
        return h

    def replay(self):
        check("gerbil_graph_launch", gerbil_graph_launch(self.graph, _stream_handle(self.stream)))

    def close(self):
        if self.graph is not None:
            gerbil_graph_destroy(self.graph)
            self.graph = None

    def result(self, raise_on_error: bool = True) -> CountResult:
        st, rep = gerbil_result(self.enc, self.bins, self.state, _stream_handle(self.stream))
        if st != GERBIL_OK and raise_on_error:
            raise GerbilError("gerbil_result", st, rep)
        n = min(rep.n_out, self.cap or 0)
        keys = self.keys_d[: n * self.W].cpu().numpy().view(np.uint64).reshape(n, self.W)
        counts = self.counts_d[:n].cpu().numpy().view(np.uint32)
        hist = self.hist_d.cpu().numpy().view(np.uint64)
        return CountResult(keys, counts, hist, rep)


def count_kmers(ascii: np.ndarray, offsets: np.ndarray, k: int, m: int, n_bins: int, threshold: int,
                hist_len: int = 256, device: str = "cuda", **kw) -> CountResult:
    """Convenience: copy host reads to the device and run the whole path once."""
    import torch
    a = torch.from_numpy(np.ascontiguousarray(ascii, dtype=np.uint8)).to(device)
    o = torch.from_numpy(np.ascontiguousarray(offsets, dtype=np.uint64).view(np.int64)).to(device)
    p = make_params(k, m, n_bins, threshold, **kw)
    job = Job(a, o, int(offsets[-1]), p, hist_len=hist_len)
    job.run()
    return job.result()

"""C-ABI checks that need no GPU: the library loads, exports every declared
symbol, validates arguments before any launch, and the Python structs match
the C layout."""
import ctypes
import os
import re
import subprocess

import pytest

from conftest import ROOT
from paper_1607_06618_amd import gerbil as g

HEADER = os.path.join(ROOT, "include", "gerbil.h")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const char\*|uint32_t|int32_t)\s+(gerbil_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    lib = g.load()
    names = declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", g.LIB_PATH], capture_output=True, text=True, check=True)
    exported = set(re.findall(r" T (gerbil_\w+)", out.stdout))
    assert set(names) <= exported
    # nothing else with the gerbil_ prefix leaks out
    assert exported == set(names)


def test_version_and_status_strings():
    assert g.gerbil_version() == 0x000100
    assert g.status_string(g.GERBIL_OK) == "ok"
    assert "capacity" in g.status_string(g.GERBIL_ECAPACITY)


def test_encode_workspace_validation():
    assert g.gerbil_encode_workspace(10, 1000, 32) > 1000 // 4
    with pytest.raises(g.GerbilError):
        g.gerbil_encode_workspace(10, 1000, 1)
    assert g.gerbil_encode_workspace(10, 1000, 480) > 1000 // 4   # keys of up to 15 words
    with pytest.raises(g.GerbilError):
        g.gerbil_encode_workspace(10, 1000, 481)


def test_param_validation_before_launch():
    enc = g.gerbil_encoded(n_reads=1, n_bytes=100, k=32)
    good = g.make_params(32, 7, 64, 2)
    assert g.gerbil_bin_workspace(enc, good) > 0
    # LDS sub-tables are sized in k-mer occurrences: more than one per slot is allowed
    assert g.gerbil_bin_workspace(enc, g.make_params(32, 7, 64, 2, load_factor=1.2)) > 0
    for bad in (g.make_params(32, 32, 64, 2), g.make_params(32, 0, 64, 2), g.make_params(32, 16, 64, 2),
                g.make_params(32, 7, 0, 2), g.make_params(32, 7, 5000, 2), g.make_params(32, 7, 64, 0),
                g.make_params(32, 7, 64, 2, block=100),
                g.make_params(32, 7, 64, 2, load_factor=0.99, table=g.GERBIL_TABLE_HBM),
                g.make_params(32, 7, 64, 2, load_factor=4.5),
                g.make_params(32, 7, 64, 2, overflow_cap=(1 << 31) + 1)):
        with pytest.raises(g.GerbilError) as e:
            g.gerbil_bin_workspace(enc, bad)
        assert e.value.status == g.GERBIL_EINVAL
    # `-d` (no reverse-complement normalisation) is accepted; other values are not
    assert g.gerbil_bin_workspace(enc, g.make_params(32, 7, 64, 2, canonical=False)) > 0
    p = g.make_params(32, 7, 64, 2)
    p.canonical = 2
    with pytest.raises(g.GerbilError) as e:
        g.gerbil_bin_workspace(enc, p)
    assert e.value.status == g.GERBIL_EINVAL
    # k above 256 takes HBM tables: AUTO picks them, LDS is refused
    e300 = g.gerbil_encoded(n_reads=1, n_bytes=1000, k=300)
    assert g.gerbil_bin_workspace(e300, g.make_params(300, 11, 64, 2)) > 0
    with pytest.raises(g.GerbilError) as e:
        g.gerbil_bin_workspace(e300, g.make_params(300, 11, 64, 2, table=g.GERBIL_TABLE_LDS))
    assert e.value.status == g.GERBIL_EUNSUPPORTED
    with pytest.raises(g.GerbilError) as e:
        g.gerbil_bin_workspace(g.gerbil_encoded(n_reads=1, n_bytes=1000, k=481), g.make_params(481, 11, 64, 2))
    # k must match the encoding
    with pytest.raises(g.GerbilError):
        g.gerbil_bin_workspace(enc, g.make_params(33, 7, 64, 2))
    # null workspace / output pointers are rejected without touching the device
    assert g.gerbil_encode(0, 0, 1, 100, 32, 0, 0, g.gerbil_encoded()) == g.GERBIL_EINVAL


def test_struct_layout_matches_header(tmp_path):
    structs = {
        "gerbil_params": g.gerbil_params, "gerbil_encoded": g.gerbil_encoded, "gerbil_bins": g.gerbil_bins,
        "gerbil_counted": g.gerbil_counted, "gerbil_report": g.gerbil_report,
        "gerbil_pipeline": g.gerbil_pipeline, "gerbil_tune_result": g.gerbil_tune_result,
    }
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "gerbil.h"', "int main(void) {"]
    for sname, cls in structs.items():
        lines.append(f'  printf("{sname} %zu\\n", sizeof({sname}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{sname}.{fname} %zu\\n", offsetof({sname}, {fname}));')
    lines.append("  return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"), "-I", "/opt/rocm/include",
                    str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = dict(ln.split() for ln in out if ln)
    for sname, cls in structs.items():
        assert int(got[sname]) == ctypes.sizeof(cls), sname
        for fname, _ in cls._fields_:
            assert int(got[f"{sname}.{fname}"]) == getattr(cls, fname).offset, (sname, fname)


def test_graph_capture_validation():
    """Argument errors of the graph entry points come back before any device call."""
    pl = g.gerbil_pipeline()
    plain = g.make_params(32, 7, 64, 2, mode=g.GERBIL_PLAIN)
    batched = g.make_params(32, 7, 64, 2, mode=g.GERBIL_BATCHED)
    enc, bins, state = g.gerbil_encoded(), g.gerbil_bins(), g.gerbil_counted()
    # the NULL stream cannot be recorded
    st, h = g.gerbil_graph_capture(pl, batched, enc, bins, state, 0)
    assert st == g.GERBIL_EINVAL and h is None
    # only the batched path is free of host synchronisation
    st, h = g.gerbil_graph_capture(pl, plain, enc, bins, state, 1)
    assert st == g.GERBIL_EUNSUPPORTED and h is None
    assert g.gerbil_graph_launch(None, 1) == g.GERBIL_EINVAL
    assert g.gerbil_graph_info(None)[0] == g.GERBIL_EINVAL
    assert g.gerbil_graph_destroy(None) == g.GERBIL_OK


def test_autotune_validation():
    p = g.make_params(32, 7, 64, 2, mode=g.GERBIL_BATCHED)
    st, _, _ = g.gerbil_autotune(g.gerbil_bins(), p, 0, 0, 0, 0, 0, 1)
    assert st == g.GERBIL_EINVAL
    assert g.gerbil_autotune_reset() == g.GERBIL_OK


def test_records_validation():
    """Argument errors of the record codec come back before any device call."""
    assert g.gerbil_records_workspace(0) == 256
    assert g.gerbil_records_workspace(8192 * 3 + 1) >= 256 + 4 * 4 + 8 * 4
    fake, ws_need = 4096, g.gerbil_records_workspace(100)
    size = ctypes.c_uint64(0)
    ok_args = dict(keys_ptr=fake, counts_ptr=fake, n=100, k=31, ws_ptr=4096, ws_bytes=ws_need, out_ptr=fake,
                   out_cap=1000, out_bytes_ptr=ctypes.addressof(size))
    for bad in (dict(out_bytes_ptr=None), dict(k=0), dict(k=481), dict(keys_ptr=0), dict(counts_ptr=0),
                dict(ws_ptr=0), dict(ws_bytes=ws_need - 1), dict(ws_ptr=4096 + 8), dict(out_ptr=0)):
        args = dict(ok_args, **bad)
        assert g.gerbil_records(**args) == g.GERBIL_EINVAL, bad


def test_parse_validation():
    """Argument errors of the parser come back before any device call."""
    ws = g.gerbil_parse_workspace(1000, 100)
    assert ws >= 256
    with pytest.raises(g.GerbilError):
        g.gerbil_parse_workspace(1000, 1002)       # more lines than bytes + 1
    fake = 4096
    ok = dict(text_ptr=fake, n=1000, fmt=0, ws_ptr=fake, ws_bytes=ws, lines_cap=100, seq_ptr=fake, seq_cap=1000,
              offsets_ptr=fake, reads_cap=100, out_ptr=fake)
    for bad in (dict(text_ptr=0), dict(ws_ptr=0), dict(offsets_ptr=0), dict(out_ptr=0), dict(seq_ptr=0),
                dict(fmt=3), dict(ws_bytes=ws - 1), dict(ws_ptr=fake + 16), dict(lines_cap=1002),
                dict(n=1 << 40)):
        assert g.gerbil_parse(**dict(ok, **bad)) == g.GERBIL_EINVAL, bad


def test_order_table_validation():
    assert g.gerbil_order_table_workspace(g.GERBIL_RANKS_CGAT, 15) == 0
    assert g.gerbil_order_table_workspace(g.GERBIL_RANKS_RANDOM, 9) == 8 * 4 ** 9
    assert g.gerbil_order_table_workspace(g.GERBIL_RANKS_DFP, 9) == 12 * 4 ** 9
    for kind, m in ((6, 5), (0, 0), (0, 16), (g.GERBIL_RANKS_RANDOM, 13)):
        with pytest.raises(g.GerbilError):
            g.gerbil_order_table_workspace(kind, m)
    fake = 4096
    ws = g.gerbil_order_table_workspace(g.GERBIL_RANKS_DFP, 5)
    enc = g.gerbil_encoded(n_reads=1, n_bytes=100, k=21, packed=fake, kmer_ok=fake)
    ok = dict(kind=g.GERBIL_RANKS_DFP, m=5, seed=0, pivot=0.5, stride=0, enc=enc, ws_ptr=fake, ws_bytes=ws,
              table_ptr=fake)
    for bad in (dict(table_ptr=0), dict(ws_ptr=0), dict(ws_bytes=ws - 1), dict(pivot=1.5), dict(pivot=-0.1),
                dict(enc=None), dict(m=21), dict(ws_ptr=fake + 8)):
        assert g.gerbil_order_table(**dict(ok, **bad)) == g.GERBIL_EINVAL, bad
    # the table order needs a table and no bin map
    e = g.gerbil_encoded(n_reads=1, n_bytes=100, k=32)
    with pytest.raises(g.GerbilError):
        g.gerbil_bin_workspace(e, g.make_params(32, 7, 64, 2, order=g.GERBIL_ORDER_TABLE))
    with pytest.raises(g.GerbilError):
        g.gerbil_bin_workspace(e, g.make_params(32, 7, 64, 2, order=g.GERBIL_ORDER_TABLE, rank_table_ptr=fake,
                                                bin_map_ptr=fake))
    assert g.gerbil_bin_workspace(e, g.make_params(32, 7, 64, 2, order=g.GERBIL_ORDER_TABLE,
                                                   rank_table_ptr=fake)) > 0


def test_key_bins_and_hll_validation():
    fake = 4096
    p = g.make_params(65, 9, 64, 1)
    assert g.gerbil_key_bins(0, 10, p, fake) == g.GERBIL_EINVAL       # keys missing
    assert g.gerbil_key_bins(fake, 10, p, 0) == g.GERBIL_EINVAL       # output missing
    assert g.gerbil_key_bins(fake, 10, g.make_params(65, 0, 64, 1), fake) == g.GERBIL_EINVAL
    bins = g.gerbil_bins(k=65, n_bins=64, packed=fake, desc=fake, bin_off=fake)
    assert g.gerbil_hll_bins(bins, p, 3, fake) == g.GERBIL_EINVAL      # too few registers
    assert g.gerbil_hll_bins(bins, p, 16, fake) == g.GERBIL_EINVAL     # too many
    assert g.gerbil_hll_bins(bins, p, 12, 0) == g.GERBIL_EINVAL
    assert g.gerbil_hll_bins(bins, g.make_params(33, 9, 64, 1), 12, fake) == g.GERBIL_EINVAL   # k differs
    assert g.gerbil_hll_bins(g.gerbil_bins(k=65, n_bins=64), p, 12, fake) == g.GERBIL_EINVAL  # no bins


def test_ceiling_validation_before_launch():
    # every argument error is returned before anything is enqueued (no GPU needed)
    sink = 4096
    assert g.gerbil_ceiling(g.GERBIL_CEIL_LDS_CAS, 0, 0, 1, 1, 0) == g.GERBIL_EINVAL          # no sink
    assert g.gerbil_ceiling(g.GERBIL_CEIL_LDS_CAS, 0, 0, 0, 1, sink) == g.GERBIL_EINVAL       # empty grid
    assert g.gerbil_ceiling(g.GERBIL_CEIL_LDS_CAS, 0, 0, 1, 0, sink) == g.GERBIL_EINVAL       # no iterations
    assert g.gerbil_ceiling(6, 0, 0, 1, 1, sink) == g.GERBIL_EINVAL                          # unknown kind
    for kind in (g.GERBIL_CEIL_HBM_ADD, g.GERBIL_CEIL_HBM_CAS, g.GERBIL_CEIL_HBM_LOAD, g.GERBIL_CEIL_ONE_ADDR):
        assert g.gerbil_ceiling(kind, 0, 4096, 1, 1, sink) == g.GERBIL_EINVAL                # no buffer
        assert g.gerbil_ceiling(kind, 4096, 32, 1, 1, sink) == g.GERBIL_EINVAL               # under one line
        assert g.gerbil_ceiling(kind, 4096, 100, 1, 1, sink) == g.GERBIL_EINVAL              # not whole lines
        assert g.gerbil_ceiling(kind, 4100, 4096, 1, 1, sink) == g.GERBIL_EINVAL             # misaligned


def test_records_noalloc_validation_before_launch():
    # argument errors come back before the scratch is looked up or anything is enqueued
    size = 4096
    assert g.gerbil_records_noalloc(8, 8, 1, 65, 8, 8, 0) == g.GERBIL_EINVAL                  # no out_bytes
    assert g.gerbil_records_noalloc(8, 8, 1, 0, 8, 8, size) == g.GERBIL_EINVAL                # k = 0
    assert g.gerbil_records_noalloc(8, 8, 1, 481, 8, 8, size) == g.GERBIL_EINVAL              # k too long
    assert g.gerbil_records_noalloc(0, 8, 1, 65, 8, 8, size) == g.GERBIL_EINVAL               # no keys
    assert g.gerbil_records_noalloc(8, 8, 1, 65, 0, 8, size) == g.GERBIL_EINVAL               # no output
    assert g.gerbil_records_noalloc(8, 8, g.GERBIL_RECORDS_NOALLOC_MAX + 1, 65, 8, 8, size) == g.GERBIL_EINVAL

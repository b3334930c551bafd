#!/usr/bin/env python3
"""Benchmark of the counting path on one MI355X.

A step is one pass of the whole path over the workload's reads, already
resident in HBM: encode -> bin -> count -> histogram. The headline is the
BATCHED schedule (all bins in one persistent launch); the PLAIN schedule (one
launch sequence per bin) is timed beside it on the same inputs. The unit of
work is a valid (N-free) k-mer window.

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "canonical k-mers counted/s at k=65 (batched vs per-bin); HBM GB/s; p50/p99"
HBM_PEAK_GBS = 8000.0


def parse_args(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c2_k65")
    ap.add_argument("--scale", type=float, default=1.0, help="genome scale factor (1.0 = the named workload)")
    ap.add_argument("--modes", default="batched,plain,graph",
                    help="batched: persistent counter; plain: one launch sequence per bin; "
                         "graph: the batched path replayed from one HIP graph")
    ap.add_argument("--pool", type=int, default=0)
    ap.add_argument("--load", type=float, default=0.0)
    ap.add_argument("--table", default="lds", choices=["lds", "hbm"])
    ap.add_argument("--theta", type=int, default=0, help="probes per key before the emergency area (0: default)")
    ap.add_argument("--overflow-cap", type=int, default=0, help="emergency-area capacity in keys (0: default)")
    ap.add_argument("--block", type=int, default=0,
                    help="threads per counting workgroup (LDS tables: 512 = two workgroups per CU)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target length of the CPU-oracle sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--tune", action="store_true", help="autotune the batched schedule before timing it")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES bytes three times (calibrates HBM byte counters)")
    ap.add_argument("--stage-clocks", action="store_true", help="report busy time per LDS stage (batched)")
    ap.add_argument("--probes", action="store_true",
                    help="report how many probes LDS-table inserts took (batched; the statistic of Sec. 3.3.1)")
    ap.add_argument("--serving", type=int, default=0, help="also serve this many jobs of the Poisson job stream")
    ap.add_argument("--serving-scale", type=float, default=1.0, help="genome-size scale of the served jobs")
    ap.add_argument("--serving-inflight", type=int, default=4)
    ap.add_argument("--serving-distinct", type=int, default=24,
                    help="distinct job payloads the serving stream cycles through")
    ap.add_argument("--size-sample", type=int, default=0,
                    help="LDS run sizing: every n-th segment is counted (0 = library default, 1 = exact)")
    ap.add_argument("--k", type=int, default=0, help="override the workload's k (keys above 256 bases use HBM tables)")
    ap.add_argument("--non-canonical", action="store_true",
                    help="count k-mers as read, without reverse-complement normalisation (-d)")
    ap.add_argument("--records", action="store_true",
                    help="also time the binary output records (App. C) of the step's pairs")
    ap.add_argument("--estimator", action="store_true",
                    help="also evaluate the distinct-k-mer estimate of the paper's table sizing on the workload's bins")
    ap.add_argument("--orders", action="store_true",
                    help="also compare the minimizer orders of Sec. 3.1 on the workload (super-mers, bins, step time)")
    ap.add_argument("--no-ceiling", action="store_true",
                    help="skip the random-access and atomic ceilings of the device")
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="threads of the all-core oracle leg (0: the usable cores, at most 16)")
    ap.add_argument("--parse", action="store_true",
                    help="also time FASTQ/FASTA parsing of the workload's reads on the device")
    return ap.parse_args(argv)


class HipEvents:
    """hipEvent_t pairs through the HIP runtime (the library records them on its stream)."""

    def __init__(self):
        self.hip = ctypes.CDLL("libamdhip64.so")
        self.hip.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
        self.hip.hipEventSynchronize.argtypes = [ctypes.c_void_p]
        self.hip.hipEventDestroy.argtypes = [ctypes.c_void_p]

    def pair(self):
        arr = (ctypes.c_void_p * 2)()
        for i in range(2):
            ev = ctypes.c_void_p()
            rc = self.hip.hipEventCreate(ctypes.byref(ev))
            if rc != 0:
                raise RuntimeError(f"hipEventCreate failed ({rc})")
            arr[i] = ev
        return arr

    def elapsed_ms(self, arr) -> float:
        self.hip.hipEventSynchronize(arr[1])
        ms = ctypes.c_float()
        rc = self.hip.hipEventElapsedTime(ctypes.byref(ms), arr[0], arr[1])
        if rc != 0:
            raise RuntimeError(f"hipEventElapsedTime failed ({rc})")
        return float(ms.value)


# Kernel sources whose change invalidates the measured HBM traffic of the counting kernel.
TRAFFIC_SOURCES = ["paper_1607_06618_amd/csrc/lds.hip", "paper_1607_06618_amd/csrc/common.h",
                   "paper_1607_06618_amd/csrc/internal.h", "paper_1607_06618_amd/csrc/table.h",
                   "paper_1607_06618_amd/csrc/api.hip"]


def sources_digest(paths) -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in paths:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(rel.encode() + b"\0" + f.read())
    return h.hexdigest()


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed counter summary of `kernel` on
    `workload`, or None if there is none or the kernel changed since."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_pmc.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for ln in f:
            if ":" in ln and not ln.startswith("#"):
                key, _, v = ln.partition(":")
                vals[key.strip()] = v.strip()
    if vals.get("source_sha256") != sources_digest(TRAFFIC_SOURCES):
        return None
    try:
        return int(float(vals["traffic_bytes"]))
    except (KeyError, ValueError):
        return None


def measure_h2d(ascii_, offsets, dev, repeats: int = 3) -> dict:
    """Upload of the reads (ASCII and offsets) from pinned host memory, timed
    with events on the current stream: the best of `repeats` copies. Outside
    every timed step."""
    import numpy as np
    import torch
    a_pin = torch.empty(ascii_.size, dtype=torch.uint8, pin_memory=True)
    a_pin.numpy()[:] = ascii_
    o_pin = torch.empty(offsets.size, dtype=torch.int64, pin_memory=True)
    o_pin.numpy()[:] = offsets.view(np.int64)
    a_d = torch.empty(ascii_.size, dtype=torch.uint8, device=dev)
    o_d = torch.empty(offsets.size, dtype=torch.int64, device=dev)
    best = None
    for _ in range(repeats):
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record()
        a_d.copy_(a_pin, non_blocking=True)
        o_d.copy_(o_pin, non_blocking=True)
        t1.record()
        t1.synchronize()
        ms = t0.elapsed_time(t1)
        best = ms if best is None else min(best, ms)
    nbytes = int(ascii_.size + 8 * offsets.size)
    del a_d, o_d, a_pin, o_pin
    return {"ms": round(best, 3), "bytes": nbytes, "gb_per_s": round(nbytes / best / 1e6, 1)}


def hll_cardinality(regs):
    """HyperLogLog estimate of each row of registers (Flajolet et al. 2007),
    with linear counting while an estimate is small."""
    import numpy as np
    m = regs.shape[1]
    alpha = 0.7213 / (1.0 + 1.079 / m)
    est = alpha * m * m / np.exp2(-regs.astype(np.float64)).sum(axis=1)
    zeros = (regs == 0).sum(axis=1)
    small = (est <= 2.5 * m) & (zeros > 0)
    est[small] = m * np.log(m / zeros[small])
    return est


def bin_diagnostics(job, stream) -> dict:
    """The realised bins of a counted job: k-mer occurrences per bin (quantiles,
    largest over median) and each bin's distinct fraction rho = distinct keys /
    occurrences, its distinct keys estimated from a HyperLogLog sketch of the
    bin (2^12 registers, about 1.6% standard error)."""
    import numpy as np
    import torch
    from paper_1607_06618_amd import gerbil as g
    nb = int(job.bins.n_bins)
    off = int(job.bins.bin_kmers) - job.ws_bin.data_ptr()
    km = job.ws_bin[off: off + 8 * nb].cpu().numpy().view(np.uint64).astype(np.float64)
    with torch.cuda.stream(stream):
        regs = g.hll_registers(job, 12, stream).cpu().numpy()
    torch.cuda.synchronize()
    used = km > 0
    rho = hll_cardinality(regs)[used] / km[used]

    def quant(x):
        return {f"p{q}": float(f"{np.percentile(x, q):.6g}") for q in (0, 10, 50, 90, 99, 100)} if x.size else {}
    med = float(np.median(km[used])) if used.any() else 0.0
    return {"n_bins": nb, "empty_bins": int((~used).sum()), "kmers_per_bin": quant(km[used]),
            "largest_over_median": round(float(km.max()) / med, 3) if med else None,
            "rho_per_bin": quant(rho), "rho_from": "HyperLogLog per bin, 2^12 registers"}


def calibrate_copy(nbytes: int) -> int:
    import torch
    src = torch.ones(nbytes // 8, dtype=torch.int64, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "copy", "bytes_read": src.numel() * 8, "bytes_written": dst.numel() * 8,
                      "launches": 3}), flush=True)
    return 0


def percentile(xs, q):
    s = sorted(xs)
    if not s:
        return None
    i = min(len(s) - 1, max(0, int(math.ceil(q / 100.0 * len(s))) - 1))
    return s[i]


def host_description():
    """Cores usable by this process, the CPU model and the RAM of the host."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    ram = None
    try:
        with open("/proc/meminfo") as f:
            for ln in f:
                if ln.startswith("MemTotal:"):
                    ram = round(int(ln.split()[1]) * 1024 / 2 ** 30, 1)
                    break
    except OSError:
        pass
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"nproc": usable, "cpu_count": os.cpu_count(), "cpu_model": model, "ram_gib": ram}


def cpu_baseline(ascii_, offsets, k, threshold, target_s, canonical=True, threads=0):
    """The oracle as it stands on a leading sample of reads: single-threaded
    (oracle.count), then the same sample split into hash shards over every
    usable core (oracle.count_sharded, one collecting thread per read range
    and one sorting thread per shard). The all-core rate is the headline."""
    import oracle
    n_reads = offsets.size - 1
    # calibrate on a small sample, then size the timed sample to ~target_s of one core
    n0 = min(n_reads, 2000)
    t = time.perf_counter()
    r0 = oracle.count(ascii_, offsets[: n0 + 1], k, threshold=threshold, canonical=canonical)
    dt0 = max(1e-3, time.perf_counter() - t)
    per_window = dt0 / max(1, r0.n_valid)
    want_windows = target_s / per_window
    avg_windows = max(1.0, r0.n_valid / n0)
    n = int(min(n_reads, max(n0, want_windows / avg_windows)))
    t = time.perf_counter()
    r = oracle.count(ascii_, offsets[: n + 1], k, threshold=threshold, canonical=canonical)
    dt1 = time.perf_counter() - t
    one = {"value": r.n_valid / dt1, "cores": 1, "seconds": round(dt1, 2)}
    host = host_description()
    T = threads or max(1, min(16, host["nproc"] or 1))
    pairs = [0]

    def on_shard(s, res):
        pairs[0] += res.keys.shape[0]

    t = time.perf_counter()
    nv = oracle.count_sharded(ascii_, offsets[: n + 1], k, threshold, T, on_shard, canonical=canonical, group=0,
                              threads=T, sort_workers=T)
    dtT = time.perf_counter() - t
    assert nv == r.n_valid and pairs[0] == r.keys.shape[0], "sharded oracle disagrees with the single-threaded one"
    return {"value": nv / dtT, "unit": "k-mers/s", "cores": T, "kind": "oracle",
            "sample": f"first {n} of {n_reads} reads ({r.n_valid} valid windows): {dtT:.1f} s on {T} threads "
                      f"(hash shards, one per thread), {dt1:.1f} s single-threaded sort-and-count",
            "single_core": one, "host": host}


def device_ceilings():
    """Random-access and atomic rates of the device (GERBIL_CEIL_*), in
    operations per second, each the best of three timed launches."""
    import torch

    from paper_1607_06618_amd import gerbil as g
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    out = {}
    for name, kind, grid, iters, buf in (
            ("lds_cas64_per_s", g.GERBIL_CEIL_LDS_CAS, cus * 4, 256, 0),
            ("lds_add32_per_s", g.GERBIL_CEIL_LDS_ADD, cus * 4, 256, 0),
            ("hbm_add32_random_line_per_s", g.GERBIL_CEIL_HBM_ADD, cus * 8, 64, 4 << 30),
            ("hbm_cas64_random_line_per_s", g.GERBIL_CEIL_HBM_CAS, cus * 8, 64, 4 << 30),
            ("hbm_load64_random_line_per_s", g.GERBIL_CEIL_HBM_LOAD, cus * 8, 64, 4 << 30),
            ("one_address_add_return_per_s", g.GERBIL_CEIL_ONE_ADDR, cus * 2, 256, 64)):
        rate, ops, ms = g.ceiling(kind, grid, iters, buf_bytes=buf)
        out[name] = float(f"{rate:.4g}")
    torch.cuda.empty_cache()
    print(f"[bench] device ceilings: {out}", file=sys.stderr, flush=True)
    return out


def main(argv=None):
    args = parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py: the counting path runs on one GPU; --gpus {args.gpus} is not supported "
              f"(sharding over several GPUs is described, not built)", file=sys.stderr, flush=True)
        return 2

    if args.calibrate_copy:
        return calibrate_copy(args.calibrate_copy)

    import numpy as np
    import torch

    import synth
    from paper_1607_06618_amd import gerbil as g

    g.load()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    w = synth.CONFIGS[args.config]
    if args.scale != 1.0:
        w = w.scaled(args.scale)
    if args.k:
        import dataclasses
        w = dataclasses.replace(w, k=args.k, name=f"{w.name}_k{args.k}",
                                note=f"{w.note}; k overridden to {args.k}")
    t0 = time.perf_counter()
    ascii_, offsets = w.generate(threads=16)
    gen_s = time.perf_counter() - t0
    print(f"[bench] generated {w.name}: {ascii_.size / 1e9:.2f} GB ASCII, {offsets.size - 1} reads in {gen_s:.1f} s",
          file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ascii_d = torch.from_numpy(ascii_).to(dev)
    offsets_d = torch.from_numpy(offsets.view(np.int64)).to(dev)
    torch.cuda.synchronize()
    bin_map_d = None
    if w.skew_bins:
        bin_map_d = torch.from_numpy(w.bin_map().view(np.int32)).to(dev)

    evs = HipEvents()
    modes = [m.strip() for m in args.modes.split(",") if m.strip()]
    if not any(m in ("batched", "plain") for m in modes):
        modes.insert(0, "batched")   # the roofline needs an eager run with kernel events
    results = {}
    shared_out = {}
    stream = torch.cuda.Stream(device=dev)   # default priority; graph capture needs a non-NULL stream
    for mode_name in modes:
        graph = mode_name == "graph"   # the batched path replayed from a HIP graph
        mode = g.GERBIL_PLAIN if mode_name == "plain" else g.GERBIL_BATCHED
        ev = evs.pair()
        table = g.GERBIL_TABLE_LDS if args.table == "lds" else g.GERBIL_TABLE_HBM
        if w.k > 256 and args.table == "lds":
            table = g.GERBIL_TABLE_HBM   # LDS tables hold keys of up to 256 bases
        p = g.make_params(w.k, w.m, w.n_bins, w.threshold, mode=mode, pool=args.pool, load_factor=args.load, table=table,
                          block=args.block, max_probes=args.theta, overflow_cap=args.overflow_cap,
                          canonical=not args.non_canonical, size_sample=args.size_sample,
                          bin_map_ptr=bin_map_d.data_ptr() if bin_map_d is not None else 0,
                          timing_events=ctypes.addressof(ev))
        clocks_d = None
        if args.stage_clocks and mode == g.GERBIL_BATCHED and not graph:
            clocks_d = torch.zeros(8, dtype=torch.int64, device=dev)
            p.stage_clocks = clocks_d.data_ptr()
        probes_d = None
        if args.probes and mode == g.GERBIL_BATCHED and not graph:
            probes_d = torch.zeros(g.GERBIL_PROBE_HIST, dtype=torch.int64, device=dev)
            p.probe_hist = probes_d.data_ptr()
        with torch.cuda.stream(stream):
            job = g.Job(ascii_d, offsets_d, int(offsets[-1]), p, hist_len=65536, stream=stream)
            # first pass sizes the workspaces (synchronises); outputs are shared between schedules
            job.encode()
            job.bin()
            st, rep = g.gerbil_result(job.enc, job.bins, None, g._stream_handle(stream))
            if "keys" in shared_out:
                job.cap, job.keys_d, job.counts_d = shared_out["cap"], shared_out["keys"], shared_out["counts"]
            tune = None
            if args.tune and mode == g.GERBIL_BATCHED:
                info = job.autotune()
                tune = {"table": {g.GERBIL_TABLE_LDS: "lds", g.GERBIL_TABLE_HBM: "hbm"}[info.table],
                        "load_factor": round(info.load_factor, 3), "pool": info.pool, "block": info.block,
                        "candidates": info.candidates, "cached": bool(info.cached),
                        "best_count_ms": round(info.best_ms, 3)}
                print(f"[bench] {mode_name} autotune: {tune}", file=sys.stderr, flush=True)
            job.prepare_count(n_valid=rep.n_valid)
            shared_out.update(cap=job.cap, keys=job.keys_d, counts=job.counts_d)
            for _ in range(args.warmup):
                job.run()
            if args.warmup:
                job.result()   # raises if a warm-up run hit a capacity or device error
            if graph:
                job.capture()
                job.replay()
                job.result()
            torch.cuda.synchronize()
            step_ms = []
            starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
            kev = [evs.pair() for _ in range(args.steps)]   # counting-kernel events, one pair per step
            torch.cuda.synchronize()
            wall0 = time.perf_counter()
            starts[0].record(stream)
            for s in range(args.steps):
                if graph:
                    job.replay()
                else:
                    job.p.timing_events = ctypes.cast(kev[s], ctypes.c_void_p)
                    job.run()
                starts[s + 1].record(stream)
            torch.cuda.synchronize()
            wall = time.perf_counter() - wall0
            res_t = job.result()
            if not graph and "bins" not in shared_out:
                shared_out["bins"] = bin_diagnostics(job, stream)   # after the timed steps
            job.close()
        for s in range(args.steps):
            step_ms.append(starts[s].elapsed_time(starts[s + 1]))
        kms = None
        if not graph:
            kms_all = [evs.elapsed_ms(e) for e in kev]
            kms = sum(kms_all) / len(kms_all)
        results[mode_name] = dict(job=job, res=res_t, wall=wall, step_ms=step_ms, kernel_ms=kms, ev=ev, tune=tune,
                                  table=job.p.table)
        if probes_d is not None:
            ph = probes_d.cpu().numpy().astype(np.float64) / (args.warmup + args.steps)
            tot = ph.sum()
            used = np.nonzero(ph)[0]
            results[mode_name]["probes"] = {
                "inserts_per_step": int(round(tot)),
                "first_probe_frac": round(float(ph[1] / tot), 6) if tot else None,
                "mean_probes": round(float((np.arange(ph.size) * ph)[1:].sum() / max(1.0, ph[1:].sum())), 4),
                "max_probe_bucket": int(used.max()) if used.size else 0,
                "emergency_without_probe": int(round(ph[0])),
                "by_probe": {int(t): int(round(ph[t])) for t in used}}
            print(f"[bench] {mode_name} probes: {results[mode_name]['probes']}", file=sys.stderr, flush=True)
        if clocks_d is not None:
            c = clocks_d.cpu().numpy()
            runs = args.warmup + args.steps
            names = ["count", "scan", "scatter", "table"]
            results[mode_name]["stage_ms"] = {names[i]: float(c[i]) / 1e5 / runs for i in range(4)}
            results[mode_name]["stage_items"] = {names[i]: int(c[4 + i]) // runs for i in range(4)}
            print(f"[bench] {mode_name} stage busy ms (summed over workgroups, per step): "
                  f"{results[mode_name]['stage_ms']} items {results[mode_name]['stage_items']}",
                  file=sys.stderr, flush=True)
        kdesc = f", counting kernel {kms:.2f} ms" if kms is not None else ""
        print(f"[bench] {mode_name}: {args.steps} steps in {wall:.3f} s, step p50 {percentile(step_ms, 50):.2f} ms"
              f"{kdesc}", file=sys.stderr, flush=True)

    head = "batched" if "batched" in results else [m for m in modes if m != "graph"][0]
    R = results[head]
    head_table = "hbm" if R["table"] == g.GERBIL_TABLE_HBM else "lds"
    rep = R["res"].report
    n_valid = rep.n_valid
    value = n_valid * args.steps / R["wall"]
    ms_per_step = 1000.0 * R["wall"] / args.steps
    hist = R["res"].hist.astype(np.float64)
    n_distinct = int(hist[1:].sum())
    c = np.arange(hist.size, dtype=np.float64)
    checks = {"sum_c_h_equals_valid": bool(rep.max_count < hist.size - 1 and int((c * hist).sum()) == n_valid)}
    if len(results) > 1:
        checks["modes_agree"] = all(
            bool(results[m]["res"].report.n_out == rep.n_out and np.array_equal(results[m]["res"].hist, R["res"].hist))
            for m in results if m != head)

    # Algorithmic bytes of one counting launch: the super-mer bases read
    # (2 bits per base, n_kmers + k - 1 bases per super-mer), every distinct
    # entry (key + 32-bit counter, E = 8W + 4 bytes) written once and read
    # once, and every output pair written once.
    W = (w.k + 31) // 32
    E = 8 * W + 4
    b_in = 0.25 * (n_valid + rep.n_superm * (w.k - 1))
    alg_bytes = b_in + 2.0 * E * n_distinct + E * rep.n_out
    achieved = alg_bytes / (R["kernel_ms"] / 1000.0) / 1e9
    kname = {("batched", "lds"): "k_lds_persistent", ("plain", "lds"): "k_lds_stage",
             ("batched", "hbm"): "k_count_persistent", ("plain", "hbm"): "k_count_bin+k_compact"}[(head, head_table)]
    traffic = None
    default_schedule = (not args.tune and args.load == 0.0 and args.pool == 0 and args.scale == 1.0 and args.block == 0
                        and args.theta == 0 and args.overflow_cap == 0
                        and not args.non_canonical and args.size_sample == 0)
    if default_schedule and "+" not in kname:
        traffic = measured_traffic(kname, w.name)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": kname,
                "kernel_ms": round(R["kernel_ms"], 3), "alg_bytes": int(alg_bytes),
                "alg_bytes_per_window": round(alg_bytes / max(1, n_valid), 2)}

    h2d = measure_h2d(ascii_, offsets, dev)
    print(f"[bench] upload of the reads from pinned host memory: {h2d}", file=sys.stderr, flush=True)
    h2d["end_to_end_with_h2d_kmers_per_s"] = float(f"{n_valid / ((ms_per_step + h2d['ms']) / 1000.0):.4g}")

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(ascii_, offsets, w.k, w.threshold, args.cpu_seconds, canonical=not args.non_canonical,
                           threads=args.cpu_threads)
    if not args.no_ceiling:
        ceil = device_ceilings()
        # every valid window is one insert of Alg. 1 into an LDS (or HBM) table
        roofline["inserts_per_s"] = float(f"{n_valid / (R['kernel_ms'] / 1000.0):.4g}")
        roofline["ceilings"] = ceil
        key = "lds_cas64_per_s" if head_table == "lds" else "hbm_cas64_random_line_per_s"
        roofline["inserts_frac_of_ceiling"] = round(roofline["inserts_per_s"] / ceil[key], 4)
        roofline["ceiling_kind"] = key

    out = {
        "metric": METRIC, "value": value, "unit": "k-mers/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": w.name, "description": w.note, "k": w.k, "m": w.m, "n_bins": w.n_bins,
                   "threshold": w.threshold, "reads": int(offsets.size - 1), "bytes": int(ascii_.size),
                   "valid_windows": int(n_valid), "super_mers": int(rep.n_superm), "distinct": n_distinct,
                   "pairs_out": int(rep.n_out), "emergency_keys": int(rep.n_overflow), "schedule": head,
                   "table": head_table, "canonical": not args.non_canonical},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "p50_ms": percentile(R["step_ms"], 50), "p99_ms": percentile(R["step_ms"], 99),
        "checks": checks,
        "count_kernel_kmers_per_s": float(f"{n_valid / (R['kernel_ms'] / 1000.0):.4g}"),
        "h2d": h2d,
        "bins": shared_out.get("bins"),
    }
    for m, r in results.items():
        out[f"{m}_kmers_per_s"] = n_valid * args.steps / r["wall"]
        out[f"{m}_ms_per_step"] = 1000.0 * r["wall"] / args.steps
        if r["kernel_ms"] is not None:
            out[f"{m}_count_kernel_ms"] = r["kernel_ms"]
        if r.get("tune"):
            out[f"{m}_autotune"] = r["tune"]
        if "probes" in r:
            out[f"{m}_probes"] = r["probes"]
        if "stage_ms" in r:
            out[f"{m}_stage_busy_ms"] = r["stage_ms"]
            out[f"{m}_stage_items"] = r["stage_items"]
    if "batched" in results and "plain" in results:
        out["batched_over_plain"] = results["plain"]["wall"] / results["batched"]["wall"]
    if args.serving:
        out["serving"] = run_serving(args)
    if args.records:
        out["records"] = run_records(R["job"], int(rep.n_out), w.k, stream)
    if args.orders:
        out["orders"] = run_orders(args, w, ascii_d, offsets_d, int(offsets[-1]), stream)
    if args.estimator:
        # the step's buffers are no longer needed: the threshold-1 count holds every distinct key
        for r in results.values():
            r["job"] = None
        shared_out.clear()
        R = job = None   # the timing loop's last job holds its workspaces and outputs
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        out["estimator"] = run_estimator(args, w, ascii_d, offsets_d, int(offsets[-1]), stream, cap=n_distinct + 1)
    if args.parse:
        out["parse"] = run_parse(args, ascii_, offsets)
    print(json.dumps(out), flush=True)
    return 0


def run_serving(args):
    """Poisson stream of independent counting jobs through the serving loop
    (arrival -> results on the host), at the jobs' stated sizes. The payloads
    are the first D distinct seeded jobs of the stream, generated before
    serving (the generator is not timed); the stream of N requests cycles
    through them with its own Poisson arrival times, so host memory holds D
    payloads, not N."""
    import concurrent.futures as cf
    import dataclasses

    import synth
    from paper_1607_06618_amd import serve

    n = args.serving
    d = max(1, min(n, args.serving_distinct))
    arrivals = synth.arrival_times(n)

    def make(j):
        w = synth.serving_job(j, scale=args.serving_scale)
        a, o = w.generate(threads=4)
        return serve.make_request(j, a, o, w.k, w.m, w.n_bins, w.threshold, arrival=0.0)

    t = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=4) as ex:
        payloads = list(ex.map(make, range(d)))
    gen_s = time.perf_counter() - t
    reqs = [dataclasses.replace(payloads[j % d], job_id=j, arrival=float(arrivals[j])) for j in range(n)]
    import torch
    free, total = torch.cuda.mem_get_info()
    # one warm-up pass over the distinct payloads (allocator, pinned pool, kernels), not timed
    warm = serve.CountingServer(budget_bytes=int(free * 0.6), max_inflight=args.serving_inflight)
    warm.serve([dataclasses.replace(r, arrival=0.0) for r in payloads[: min(d, 4)]], realtime=False)
    srv = serve.CountingServer(budget_bytes=int(free * 0.6), max_inflight=args.serving_inflight)
    srv.pool = warm.pool
    res = []

    def keep(r):   # the caller's side: take the timings, hand the pinned buffers back
        r.release()
        res.append(r)

    srv.serve(reqs, realtime=True, on_result=keep)
    stats = serve.summarize(res, srv.makespan)
    stats["count_kernel_busy_frac"] = sum(r.count_kernel_ms for r in res) / 1000.0 / srv.makespan
    stats.update({"offered_jobs_per_s": synth.SERVING_RATE, "requests": n, "distinct_payloads": d,
                  "scale": args.serving_scale, "inflight": args.serving_inflight,
                  "generation_s": round(gen_s, 1), "k_mix": sorted({r.k for r in payloads}),
                  "mean_job_valid_windows": sum(r.n_valid for r in res) / max(1, len(res))})
    print(f"[bench] serving: {stats}", file=sys.stderr, flush=True)
    return stats


def run_records(job, n: int, k: int, stream):
    """The App. C record stream of the step's output pairs, timed with events
    on the stream it runs on (pairs already in HBM; records written to HBM)."""
    import torch

    from paper_1607_06618_amd import gerbil as g

    W, kb = (k + 31) // 32, (k + 3) // 4
    with torch.cuda.stream(stream):
        ws = torch.empty(max(256, g.gerbil_records_workspace(n)), dtype=torch.uint8, device="cuda")
        cap = n * (5 + kb)
        out = torch.empty(max(1, cap), dtype=torch.uint8, device="cuda")
        size = torch.zeros(1, dtype=torch.int64, device="cuda")
        call = lambda: g.check("gerbil_records", g.gerbil_records(
            job.keys_d.data_ptr(), job.counts_d.data_ptr(), n, k, ws.data_ptr(), ws.numel(), out.data_ptr(), cap,
            size.data_ptr(), int(stream.cuda_stream)))
        call()
        reps = 10
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            call()
        e1.record(stream)
        e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    nbytes = int(size.item())
    alg = n * (8 * W + 4) + nbytes   # pairs read once, records written once
    res = {"pairs": n, "record_bytes": nbytes, "ms": round(ms, 4), "alg_GBps": round(alg / ms / 1e6, 1),
           "alg_frac_of_hbm_peak": round(alg / ms / 1e6 / HBM_PEAK_GBS, 4)}
    print(f"[bench] records: {res}", file=sys.stderr, flush=True)
    return res


def run_estimator(args, w, ascii_d, offsets_d, n_bytes, stream, cap=None):
    """The table-size estimate of Sec. 3.4.1 on this workload's bins: the
    distinct k-mers of a bin predicted as its k-mers times the ratio of
    distinct to all k-mers over the bins counted before it (bins in index
    order, the first predicted with ratio 1), against the true distinct
    k-mers per bin (a count with threshold 1, every key mapped to its bin)."""
    import numpy as np
    import torch

    from paper_1607_06618_amd import gerbil as g

    with torch.cuda.stream(stream):
        # threshold 1 keeps every distinct key (131 GB of keys on the skewed k = 99 reads); this
        # count is not timed, so it takes 8 key slots, each sized for the largest bin, not 16
        p = g.make_params(w.k, w.m, w.n_bins, 1, mode=g.GERBIL_BATCHED, canonical=not args.non_canonical, pool=8)
        job = g.Job(ascii_d, offsets_d, n_bytes, p, hist_len=65536, stream=stream, cap=cap)
        job.run()
        st, rep = g.gerbil_result(job.enc, job.bins, job.state, g._stream_handle(stream))
        if st != g.GERBIL_OK:
            raise g.GerbilError("gerbil_result", st, rep)
        n = int(rep.n_out)
        bins = g.key_bins(job.keys_d, n, job.p, stream=stream)
        distinct = torch.bincount(bins, minlength=w.n_bins).cpu().numpy().astype(np.float64)
        koff = int(job.bins.bin_kmers) - job.ws_bin.data_ptr()
        kmers = job.ws_bin[koff: koff + 8 * w.n_bins].view(torch.int64).cpu().numpy().astype(np.float64)
        # HyperLogLog sketches of the same bins, from the k-mer occurrences (no counting)
        log2_regs = 12
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        regs = g.hll_registers(job, log2_regs, stream=stream)
        e1.record(stream)
        e1.synchronize()
        hll_ms = e0.elapsed_time(e1)
        regs = regs.cpu().numpy()
    del job, bins
    torch.cuda.empty_cache()
    assert int(distinct.sum()) == n
    used = kmers > 0
    ratio = distinct[used] / kmers[used]
    cum_d = np.concatenate([[0.0], np.cumsum(distinct)[:-1]])
    cum_k = np.concatenate([[0.0], np.cumsum(kmers)[:-1]])
    run_ratio = np.where(cum_k > 0, cum_d / np.maximum(cum_k, 1.0), 1.0)
    pred = kmers * run_ratio
    sel = used & (np.arange(w.n_bins) > 0) & (distinct > 0)
    rel = (pred[sel] - distinct[sel]) / distinct[sel]
    glob = float(distinct.sum() / kmers.sum())
    rel_static = (kmers[sel] * glob - distinct[sel]) / distinct[sel]
    mreg = regs.shape[1]
    alpha = 0.7213 / (1.0 + 1.079 / mreg)
    hll = alpha * mreg * mreg / (2.0 ** -regs.astype(np.float64)).sum(axis=1)
    zeros = (regs == 0).sum(axis=1)
    small = (hll <= 2.5 * mreg) & (zeros > 0)
    hll[small] = mreg * np.log(mreg / zeros[small])   # linear counting
    rel_hll = (hll[sel] - distinct[sel]) / distinct[sel]
    res = {"distinct": n, "kmers": int(kmers.sum()), "global_ratio": round(glob, 4),
           "bin_ratio_min_median_max": [round(float(x), 4) for x in (ratio.min(), np.median(ratio), ratio.max())],
           "running_estimate_abs_rel_err_median_p95_max": [round(float(x), 4) for x in
                                                           (np.median(np.abs(rel)), np.percentile(np.abs(rel), 95),
                                                            np.abs(rel).max())],
           "running_estimate_under_5pct_bins": int((rel < -0.05).sum()),
           "running_estimate_under_10pct_bins": int((rel < -0.10).sum()),
           "global_ratio_abs_rel_err_median_max": [round(float(np.median(np.abs(rel_static))), 4),
                                                   round(float(np.abs(rel_static).max()), 4)],
           "hll_registers_per_bin": mreg,
           "hll_abs_rel_err_median_p95_max": [round(float(x), 4) for x in
                                              (np.median(np.abs(rel_hll)), np.percentile(np.abs(rel_hll), 95),
                                               np.abs(rel_hll).max())],
           "hll_under_5pct_bins": int((rel_hll < -0.05).sum()),
           "hll_ms": round(hll_ms, 2),
           "bins": int(sel.sum())}
    print(f"[bench] estimator: {res}", file=sys.stderr, flush=True)
    return res


def run_orders(args, w, ascii_d, offsets_d, n_bytes, stream):
    """The analogue of the paper's Fig. 4 on this workload: for each minimizer
    order, the super-mers (count and bases, the temporary data of the paper),
    the largest bin in k-mers (what bounds a bin's table), and the batched
    step time with that order."""
    import torch

    from paper_1607_06618_amd import gerbil as g

    orders = [("kmc2", g.GERBIL_ORDER_KMC2, None), ("lex", g.GERBIL_ORDER_LEX, None),
              ("cgat", g.GERBIL_ORDER_TABLE, (g.GERBIL_RANKS_CGAT, 0.0)),
              ("roberts", g.GERBIL_ORDER_TABLE, (g.GERBIL_RANKS_ROBERTS, 0.0)),
              ("random", g.GERBIL_ORDER_TABLE, (g.GERBIL_RANKS_RANDOM, 0.0))]
    orders += [(f"dfp{p}", g.GERBIL_ORDER_TABLE, (g.GERBIL_RANKS_DFP, p)) for p in (0.0, 0.5, 0.8, 1.0)]
    res = {}
    with torch.cuda.stream(stream):
        probe = g.Job(ascii_d, offsets_d, n_bytes, g.make_params(w.k, w.m, w.n_bins, w.threshold), stream=stream)
        probe.encode()   # the dfp frequency sample is taken from this encoding
        for name, order, spec in orders:
            table_d, table_ms = None, 0.0
            if spec is not None:
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                table_d = g.order_table(spec[0], w.m, seed=1, pivot=spec[1], enc=probe.enc, stream=stream)
                e1.record(stream)
                e1.synchronize()
                table_ms = e0.elapsed_time(e1)
            p = g.make_params(w.k, w.m, w.n_bins, w.threshold, mode=g.GERBIL_BATCHED, order=order,
                              rank_table_ptr=table_d.data_ptr() if table_d is not None else 0)
            job = g.Job(ascii_d, offsets_d, n_bytes, p, hist_len=65536, stream=stream)
            job.encode()
            job.bin()
            st, rep = g.gerbil_result(job.enc, job.bins, None, g._stream_handle(stream))
            n_sm = int(rep.n_superm)
            off = int(job.bins.desc) - job.ws_bin.data_ptr()
            desc = job.ws_bin[off: off + 8 * n_sm].view(torch.int64)
            kmers = int((desc & 0xFFFFFF).sum().item())
            koff = int(job.bins.bin_kmers) - job.ws_bin.data_ptr()
            bin_kmers = job.ws_bin[koff: koff + 8 * w.n_bins].view(torch.int64)
            job.prepare_count(n_valid=rep.n_valid)
            job.run()
            job.result()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(args.steps):
                job.run()
            e1.record(stream)
            e1.synchronize()
            r = job.result()
            res[name] = {"superm": n_sm, "superm_bases": kmers + n_sm * (w.k - 1),
                         "max_bin_kmers": int(bin_kmers.max().item()), "mean_bin_kmers": kmers / w.n_bins,
                         "step_ms": round(e0.elapsed_time(e1) / args.steps, 3), "table_ms": round(table_ms, 3),
                         "n_out": int(r.report.n_out)}
            print(f"[bench] order {name}: {res[name]}", file=sys.stderr, flush=True)
            job.close()
            del job, table_d
        probe.close()
    torch.cuda.empty_cache()
    return res


def run_parse(args, ascii_, offsets):
    """Device parsing of the workload's reads rendered as FASTQ and as 60-column
    FASTA: text in HBM -> CSR reads in HBM, timed with events on the stream
    the parser runs on."""
    import numpy as np
    import torch

    import synth
    from paper_1607_06618_amd import gerbil as g

    res = {}
    renders = (("fastq", lambda: synth.to_fastq(ascii_, offsets, seed=9)),
               ("fasta60", lambda: synth.to_fasta(ascii_, offsets, width=60)))
    for name, render in renders:
        text = render()
        n = len(text)
        text_d = torch.frombuffer(bytearray(text), dtype=torch.uint8).cuda()
        del text
        first = g.parse(text_d)   # sizes the line capacity
        info = first.info
        assert info.status == 0 and info.n_reads == offsets.size - 1 and info.n_bytes == int(offsets[-1])
        cap = int(info.n_lines)
        ws = torch.empty(g.gerbil_parse_workspace(n, cap), dtype=torch.uint8, device="cuda")
        seq = torch.empty(n, dtype=torch.uint8, device="cuda")
        offs = torch.empty(cap + 1, dtype=torch.int64, device="cuda")
        info_d = torch.zeros(ctypes.sizeof(g.gerbil_parsed), dtype=torch.uint8, device="cuda")
        s = torch.cuda.current_stream()
        call = lambda: g.check("gerbil_parse", g.gerbil_parse(
            text_d.data_ptr(), n, 0, ws.data_ptr(), ws.numel(), cap, seq.data_ptr(), n, offs.data_ptr(), cap,
            info_d.data_ptr(), int(s.cuda_stream)))
        for _ in range(2):
            call()
        reps = 20
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(s)
        for _ in range(reps):
            call()
        e1.record(s)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / reps
        alg = n + int(info.n_bytes) + 8 * (int(info.n_reads) + 1)   # text read, reads written, offsets written
        res[name] = {"text_bytes": n, "reads": int(info.n_reads), "lines": int(info.n_lines), "ms": round(ms, 4),
                     "text_GBps": round(n / ms / 1e6, 1), "alg_GBps": round(alg / ms / 1e6, 1),
                     "alg_frac_of_hbm_peak": round(alg / ms / 1e6 / HBM_PEAK_GBS, 4)}
        print(f"[bench] parse {name}: {res[name]}", file=sys.stderr, flush=True)
        del text_d, ws, seq, offs, first
        torch.cuda.empty_cache()
    return res


if __name__ == "__main__":
    sys.exit(main())

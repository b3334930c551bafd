"""Serving loop: continuous batching of independent counting jobs on one GPU.

A request is a set of reads (host memory) plus counting parameters. The
loop admits requests in arrival order while their estimated device
footprint fits the HBM budget and an in-flight slot is free, so requests
that arrive while others run are admitted as soon as memory and slots free
up. Every admitted job runs on its own HIP stream and advances through an
event-driven state machine, so the copies and kernels of different jobs
overlap on the device:

  ADMITTED   host->device copy, gerbil_encode, gerbil_bin enqueued; when the
             bins are done: workspace sized, gerbil_count + gerbil_histogram
  COUNTED    when the count is done: capacities checked (the count is
             repeated once with the exact output capacity if the first
             guess was too small, or with exact run sizing and a larger
             emergency area if a sampled run or the emergency area ran
             out), results copied to pinned host memory
  COPIED     when the copies are done: finished, memory released

Pinned host buffers for the results are taken from a pool: a Result's arrays
are views of them (no host copy) until Result.release() hands them back, so
once the pool has warmed up jobs allocate no pinned memory. Device memory comes from torch's caching allocator. A job
whose retry fails again is reported with its error instead of stopping the
other jobs.

All counting runs in the library's kernels; this module only schedules.
Latency is measured from arrival to results on the host and split into
queueing delay (arrival -> admission) and service time.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass
from typing import List

import numpy as np

from . import gerbil as g


@dataclass
class Request:
    job_id: int
    ascii: "object"            # pinned host uint8 tensor (or numpy array)
    offsets: "object"          # pinned host int64 tensor holding uint64 offsets (or numpy array)
    k: int
    m: int
    n_bins: int
    threshold: int
    arrival: float = 0.0       # seconds after the start of serving
    hist_len: int = 1024


@dataclass
class Result:
    job_id: int
    keys: np.ndarray
    counts: np.ndarray
    hist: np.ndarray
    n_valid: int
    arrival: float
    admitted: float
    done: float
    retries: int = 0
    error: str = ""            # set when the job could not be counted (its arrays are then empty)
    device_ms: float = 0.0     # stream time from the host-to-device copy to the results on the host
    count_kernel_ms: float = 0.0  # the counting kernel(s) alone
    _release: object = None

    def release(self):
        """Give the pinned buffers behind keys, counts and hist back to the
        server's pool; the arrays must not be used afterwards."""
        if self._release is not None:
            self._release()
            self._release = None
        self.keys = self.counts = self.hist = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival

    @property
    def queue_delay(self) -> float:
        return self.admitted - self.arrival

    def sorted(self):
        if self.keys.shape[0] == 0:
            return self.keys, self.counts
        order = np.lexsort(self.keys.T[::-1])
        return self.keys[order], self.counts[order]


SERVING_KEY_SLOTS = 8


def footprint(n_bytes: int, n_reads: int, k: int, m: int, n_bins: int, threshold: int) -> int:
    """Estimated device bytes of one job (admission control)."""
    W = (k + 31) // 32
    w = k - m + 1
    ascii_b = n_bytes + 8 * (n_reads + 1)
    enc = n_bytes // 4 + 3 * (n_bytes // 8) + 4096
    superm = min(n_bytes, n_bytes * 4 // (w + 1) + n_bytes // 2048 + 4096)
    bins = superm * 20 + n_bins * 32
    keys = SERVING_KEY_SLOTS * 2 * n_bytes * 8 * W // max(1, n_bins) + (1 << 24)   # key slots, bins up to 2x the mean
    out = (n_bytes // (2 * threshold) + 1) * (8 * W + 4)               # first output guess
    return ascii_b + enc + bins + keys + out + (1 << 22)


class _HipEventPair:
    """Two hipEvent_t for gerbil_params.timing_events (the library records
    them around its counting kernels on the job's stream)."""
    _hip = None

    def __init__(self):
        import ctypes
        if _HipEventPair._hip is None:
            hip = ctypes.CDLL("libamdhip64.so")
            hip.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
            hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
            hip.hipEventDestroy.argtypes = [ctypes.c_void_p]
            _HipEventPair._hip = hip
        self.arr = (ctypes.c_void_p * 2)()
        for i in range(2):
            ev = ctypes.c_void_p()
            if _HipEventPair._hip.hipEventCreate(ctypes.byref(ev)) != 0:
                raise RuntimeError("hipEventCreate failed")
            self.arr[i] = ev

    def ms(self) -> float:
        import ctypes
        out = ctypes.c_float()
        if self._hip.hipEventElapsedTime(ctypes.byref(out), self.arr[0], self.arr[1]) != 0:
            return 0.0
        return float(out.value)

    def close(self):
        for i in range(2):
            if self.arr[i]:
                self._hip.hipEventDestroy(self.arr[i])
                self.arr[i] = None


class _PinnedPool:
    """Pinned host buffers reused across jobs (pinning memory costs far more
    than a copy). Buffers come in power-of-two sizes of at least 1 MiB."""

    def __init__(self, torch):
        self.torch = torch
        self.free = collections.defaultdict(list)

    def take(self, nbytes: int):
        size = 1 << 20
        while size < nbytes:
            size <<= 1
        if self.free[size]:
            return self.free[size].pop()
        return self.torch.empty(size, dtype=self.torch.uint8, pin_memory=True)

    def give(self, buf):
        self.free[int(buf.numel())].append(buf)


class _Job:
    def __init__(self, req: Request, t_admit: float, device, torch, pool: "_PinnedPool", params_hook=None):
        self.req = req
        self.t_admit = t_admit
        self.torch = torch
        self.pool = pool
        self.stream = torch.cuda.Stream(device=device)   # default priority
        self.state = "ADMITTED"
        self.retries = 0
        self.error = ""
        self.ev = torch.cuda.Event()
        self.ev_start = torch.cuda.Event(enable_timing=True)
        self.ev_end = torch.cuda.Event(enable_timing=True)
        self.kev = _HipEventPair()
        self.host_bufs = []
        with torch.cuda.stream(self.stream):
            self.ev_start.record(self.stream)
            self.ascii_d = torch.as_tensor(req.ascii).to(device, non_blocking=True)
            self.offsets_d = torch.as_tensor(req.offsets).to(device, non_blocking=True)
            n_bytes = int(self.ascii_d.numel())
            # 8 key slots (one per XCD queue) instead of the library's 16: the jobs in
            # flight already overlap on the GPU, and a smaller count workspace per job
            # keeps the allocator's cache of freed workspaces small
            p = g.make_params(req.k, req.m, req.n_bins, req.threshold, mode=g.GERBIL_BATCHED, pool=SERVING_KEY_SLOTS)
            if params_hook is not None:
                params_hook(p)
            import ctypes
            p.timing_events = ctypes.cast(self.kev.arr, ctypes.c_void_p)
            self.p = p
            self.job = g.Job(self.ascii_d, self.offsets_d, n_bytes, p, hist_len=req.hist_len, stream=self.stream)
            self.job.encode()
            self.job.bin()
        self.ev.record(self.stream)

    def advance(self) -> bool:
        """Move forward if the device work of the current state is done; True when finished."""
        if not self.ev.query():
            return False
        with self.torch.cuda.stream(self.stream):
            return self._advance()

    def _advance(self) -> bool:
        torch = self.torch
        s = g._stream_handle(self.stream)
        if self.state == "ADMITTED":
            st, rep = g.gerbil_result(self.job.enc, self.job.bins, None, s)
            if st != g.GERBIL_OK:
                raise g.GerbilError("gerbil_result", st, rep)
            self.n_valid = rep.n_valid
            # first output guess: at most n_valid / t keys reach the threshold; with
            # coverage above ~7x the distinct keys that do are below n_valid / (2t)
            self.job.cap = max(1024, rep.n_valid // (2 * self.req.threshold) + 1)
            self.job.prepare_count(n_valid=rep.n_valid)
            self.job.count()
            self.ev.record(self.stream)
            self.state = "COUNTED"
            return False
        if self.state == "COUNTED":
            st, rep = g.gerbil_result(self.job.enc, self.job.bins, self.job.state, s)
            if st == g.GERBIL_ECAPACITY and self.retries == 0 and \
                    not rep.status & ~(g.ST_OUT_CAP | g.ST_POOL | g.ST_OVF_CAP):
                # Repeat only the count (the bins stay on the device): with the
                # exact output capacity, and, if a run sized from the sample or
                # the emergency area ran out, with exact run sizing and an
                # emergency area large enough for what was pushed.
                self.retries += 1
                if rep.status & ~g.ST_OUT_CAP:
                    self.p.size_sample = 1
                    self.p.overflow_cap = max(4 * int(self.job.state.overflow_cap), int(rep.n_overflow) + (1 << 16))
                    self.job.ws_count = None
                self.job.cap = max(int(self.job.cap), int(rep.n_out))
                self.job.keys_d = None
                self.job.hist_d.zero_()
                self.job.prepare_count(n_valid=self.n_valid)
                self.job.count()
                self.ev.record(self.stream)
                return False
            if st != g.GERBIL_OK:
                self.error = f"gerbil_result: status {st} ({g.status_string(st)}), device bits {rep.status:#x}"
                self.n_out = 0
                self.ev_end.record(self.stream)
                self.state = "COPIED"
                return True
            n = int(rep.n_out)
            W = self.job.W
            kb, cb, hb = self.pool.take(8 * n * W), self.pool.take(4 * n), self.pool.take(8 * self.req.hist_len)
            self.host_bufs = [kb, cb, hb]
            self.keys_h = kb[: 8 * n * W].view(torch.int64)
            self.counts_h = cb[: 4 * n].view(torch.int32)
            self.hist_h = hb[: 8 * self.req.hist_len].view(torch.int64)
            self.keys_h.copy_(self.job.keys_d[: n * W], non_blocking=True)
            self.counts_h.copy_(self.job.counts_d[:n], non_blocking=True)
            self.hist_h.copy_(self.job.hist_d, non_blocking=True)
            self.n_out = n
            self.ev_end.record(self.stream)
            self.ev.record(self.stream)
            self.state = "COPIED"
            return False
        return True   # COPIED and complete

    def result(self, t_done: float) -> Result:
        n, W = self.n_out, self.job.W
        if self.error:
            keys = np.zeros((0, W), dtype=np.uint64)
            counts = np.zeros(0, dtype=np.uint32)
            hist = np.zeros(self.req.hist_len, dtype=np.uint64)
        else:
            # views of the pinned buffers: no host copy
            keys = self.keys_h.numpy().view(np.uint64).reshape(n, W)
            counts = self.counts_h.numpy().view(np.uint32)
            hist = self.hist_h.numpy().view(np.uint64)
        bufs, pool = self.host_bufs, self.pool
        self.host_bufs = []

        def release():
            for b in bufs:
                pool.give(b)

        self.ev_end.synchronize()
        dev_ms = self.ev_start.elapsed_time(self.ev_end)
        k_ms = self.kev.ms()
        self.kev.close()
        return Result(self.req.job_id, keys, counts, hist, getattr(self, "n_valid", 0), self.req.arrival,
                      self.t_admit, t_done, self.retries, self.error, dev_ms, k_ms, release)


def _numel(x) -> int:
    return int(x.numel()) if hasattr(x, "numel") and callable(x.numel) else int(np.asarray(x).size)


def make_request(job_id: int, ascii: np.ndarray, offsets: np.ndarray, k: int, m: int, n_bins: int, threshold: int,
                 arrival: float = 0.0, hist_len: int = 1024) -> Request:
    """Request with its reads in pinned host memory (so the copy to the device is asynchronous)."""
    import torch
    a = torch.from_numpy(np.ascontiguousarray(ascii, dtype=np.uint8)).pin_memory()
    o = torch.from_numpy(np.ascontiguousarray(offsets, dtype=np.uint64).view(np.int64)).pin_memory()
    return Request(job_id, a, o, k, m, n_bins, threshold, arrival, hist_len)


class CountingServer:
    """Admission by HBM footprint, continuous batching over HIP streams."""

    def __init__(self, budget_bytes: int, max_inflight: int = 4, device: str = "cuda:0", params_hook=None):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.budget = int(budget_bytes)
        self.max_inflight = int(max_inflight)
        self.params_hook = params_hook   # optional: adjusts each job's gerbil_params (tests force capacities)
        self.pool = _PinnedPool(torch)
        g.load()

    def serve(self, requests: List[Request], realtime: bool = True, poll_s: float = 2e-4,
              on_result=None) -> List[Result]:
        """Serve `requests` (sorted by arrival). With realtime=False every request arrives at t=0.
        Results are returned sorted by job id; with `on_result`, each is instead
        handed to on_result(result) as it completes (the callback owns it and
        should release() it) and the returned list is empty."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        pending: collections.deque = collections.deque()
        inflight: List = []
        used = 0
        done: List[Result] = []
        t0 = time.perf_counter()
        i = 0
        while i < len(reqs) or pending or inflight:
            now = time.perf_counter() - t0
            while i < len(reqs) and (not realtime or reqs[i].arrival <= now):
                pending.append(reqs[i])
                i += 1
            # admission in arrival order while memory and slots allow
            while pending and len(inflight) < self.max_inflight:
                r = pending[0]
                fp = footprint(_numel(r.ascii), _numel(r.offsets) - 1, r.k, r.m, r.n_bins, r.threshold)
                if inflight and used + fp > self.budget:
                    break
                pending.popleft()
                inflight.append((_Job(r, time.perf_counter() - t0, self.device, self.torch, self.pool,
                                      self.params_hook), fp))
                used += fp
            progressed = False
            still = []
            for job, fp in inflight:
                if job.advance():
                    res = job.result(time.perf_counter() - t0)
                    if on_result is not None:
                        on_result(res)
                    else:
                        done.append(res)
                    used -= fp
                    progressed = True
                else:
                    still.append((job, fp))
            inflight = still
            if not progressed and inflight:
                time.sleep(poll_s)
            elif not inflight and not pending and i < len(reqs):
                time.sleep(max(0.0, min(poll_s * 10, reqs[i].arrival - (time.perf_counter() - t0))))
        self.makespan = time.perf_counter() - t0
        return sorted(done, key=lambda r: r.job_id)


def summarize(results: List[Result], makespan: float) -> dict:
    lat = sorted(r.latency for r in results)
    q = sorted(r.queue_delay for r in results)

    def pct(xs, p):
        if not xs:
            return None
        return xs[min(len(xs) - 1, max(0, int(np.ceil(p / 100.0 * len(xs))) - 1))]

    windows = sum(r.n_valid for r in results)
    dev = sum(r.device_ms for r in results)
    kern = sum(r.count_kernel_ms for r in results)
    svc = sorted(r.done - r.admitted for r in results)
    return {"jobs": len(results), "makespan_s": makespan, "jobs_per_s": len(results) / makespan,
            "kmers_per_s": windows / makespan, "p50_latency_s": pct(lat, 50), "p99_latency_s": pct(lat, 99),
            "p50_queue_s": pct(q, 50), "p99_queue_s": pct(q, 99),
            "p50_service_s": pct(svc, 50), "p99_service_s": pct(svc, 99),
            "mean_device_ms_per_job": dev / max(1, len(results)),
            "mean_count_kernel_ms_per_job": kern / max(1, len(results)),
            "count_kernel_share_of_device_time": (kern / dev) if dev > 0 else None,
            "retries": sum(r.retries for r in results), "errors": sum(1 for r in results if r.error)}

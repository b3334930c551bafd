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
  COUNTED    when the count is done: output capacity checked (the count is
             repeated with the exact capacity if the first guess was too
             small), results copied to pinned host memory
  COPIED     when the copies are done: finished, memory released

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


def footprint(n_bytes: int, n_reads: int, k: int, m: int, n_bins: int, threshold: int) -> int:
    """Estimated device bytes of one job (admission control)."""
    W = (k + 31) // 32
    w = k - m + 1
    ascii_b = n_bytes + 8 * (n_reads + 1)
    enc = n_bytes // 4 + 3 * (n_bytes // 8) + 4096
    superm = min(n_bytes, n_bytes * 4 // (w + 1) + n_bytes // 2048 + 4096)
    bins = superm * 20 + n_bins * 32
    keys = 8 * 2 * n_bytes * 8 * W // max(1, n_bins) + (1 << 24)      # key slots, bins up to 2x the mean
    out = (n_bytes // (2 * threshold) + 1) * (8 * W + 4)               # first output guess
    return ascii_b + enc + bins + keys + out + (1 << 22)


class _Job:
    def __init__(self, req: Request, t_admit: float, device, torch):
        self.req = req
        self.t_admit = t_admit
        self.torch = torch
        self.stream = torch.cuda.Stream(device=device)   # default priority
        self.state = "ADMITTED"
        self.retries = 0
        self.ev = torch.cuda.Event()
        with torch.cuda.stream(self.stream):
            self.ascii_d = torch.as_tensor(req.ascii).to(device, non_blocking=True)
            self.offsets_d = torch.as_tensor(req.offsets).to(device, non_blocking=True)
            n_bytes = int(self.ascii_d.numel())
            p = g.make_params(req.k, req.m, req.n_bins, req.threshold, mode=g.GERBIL_BATCHED)
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
            if st == g.GERBIL_ECAPACITY and rep.status == g.ST_OUT_CAP:
                # repeat only the count, with the exact capacity (the bins stay on the device)
                self.retries += 1
                self.job.cap = int(rep.n_out)
                self.job.keys_d = None
                self.job.prepare_count(n_valid=self.n_valid)
                self.job.count()
                self.ev.record(self.stream)
                return False
            if st != g.GERBIL_OK:
                raise g.GerbilError("gerbil_result", st, rep)
            n = int(rep.n_out)
            W = self.job.W
            self.keys_h = torch.empty(n * W, dtype=torch.int64, pin_memory=True)
            self.counts_h = torch.empty(n, dtype=torch.int32, pin_memory=True)
            self.hist_h = torch.empty(self.req.hist_len, dtype=torch.int64, pin_memory=True)
            self.keys_h.copy_(self.job.keys_d[: n * W], non_blocking=True)
            self.counts_h.copy_(self.job.counts_d[:n], non_blocking=True)
            self.hist_h.copy_(self.job.hist_d, non_blocking=True)
            self.n_out = n
            self.ev.record(self.stream)
            self.state = "COPIED"
            return False
        return True   # COPIED and complete

    def result(self, t_done: float) -> Result:
        n, W = self.n_out, self.job.W
        keys = self.keys_h.numpy().view(np.uint64).reshape(n, W).copy()
        counts = self.counts_h.numpy().view(np.uint32).copy()
        hist = self.hist_h.numpy().view(np.uint64).copy()
        return Result(self.req.job_id, keys, counts, hist, self.n_valid, self.req.arrival, self.t_admit, t_done,
                      self.retries)


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

    def __init__(self, budget_bytes: int, max_inflight: int = 4, device: str = "cuda:0"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.budget = int(budget_bytes)
        self.max_inflight = int(max_inflight)
        g.load()

    def serve(self, requests: List[Request], realtime: bool = True, poll_s: float = 2e-4) -> List[Result]:
        """Serve `requests` (sorted by arrival). With realtime=False every request arrives at t=0."""
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
                inflight.append((_Job(r, time.perf_counter() - t0, self.device, self.torch), fp))
                used += fp
            progressed = False
            still = []
            for job, fp in inflight:
                if job.advance():
                    done.append(job.result(time.perf_counter() - t0))
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
    return {"jobs": len(results), "makespan_s": makespan, "jobs_per_s": len(results) / makespan,
            "kmers_per_s": windows / makespan, "p50_latency_s": pct(lat, 50), "p99_latency_s": pct(lat, 99),
            "p50_queue_s": pct(q, 50), "p99_queue_s": pct(q, 99),
            "retries": sum(r.retries for r in results)}

"""Serving loop: continuous admission of time-frame chunks on one GPU.

Chunks arrive over time with their zero-suppressed input already resident in
HBM (the paper's synchronous processing receives collision-complete time
frames over the network into the processing nodes, section "Hardware and data
flow").  Each admitted chunk runs on one of a fixed set of slots -- a library
context with its own HIP stream -- so the launch sequences of several chunks
overlap on the device.  A chunk is admitted, in arrival order, when a slot is
free and its output buffers fit in the HBM budget beside the chunks in flight.
Completion is seen from an event recorded after the chunk's launch sequence;
the status and counts are read then.  A chunk whose output estimate was too
small (the device reports the size it needed) is run again with that size.

The scheduling logic (`Scheduler`) is plain host code with an executor
interface, so it is exercised without a GPU; `GpuExecutor` binds it to the
library.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional

import numpy as np

from . import tpc

# bytes of the output buffers per cluster and per tracklet slot (see _outputs)
BYTES_PER_CLUSTER = 33 + 16 + 4 + 4
BYTES_PER_TRACKLET = 6 + 4 + 20 + 60 + 4 + 2 + 1 + 1 + 4 + 4


@dataclass
class Job:
    """One chunk: its resident input and the bookkeeping of its run."""
    id: int
    zs: dict
    n_units: int
    n_time_bins: int
    n_samples: int
    cl_cap: int = 0
    tl_cap: int = 0
    arrival: float = 0.0
    start: float = -1.0
    done: float = -1.0
    retries: int = 0
    nbytes: int = 0
    counts: Optional[dict] = None
    outputs: Optional[dict] = None
    error: Optional[str] = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def estimate_caps(n_samples: int, cl_ratio: float = 6.0, tl_ratio: float = 12.0):
    """Output capacities from the input size: clusters <= samples / cl_ratio,
    tracklets <= clusters / tl_ratio (generous for the synthetic workloads;
    an overflow is detected on the device and the chunk rerun)."""
    cl = max(1024, int(n_samples / cl_ratio) + 1024)
    tl = max(256, int(cl / tl_ratio) + 256)
    return cl, tl


def job_bytes(job: Job) -> int:
    return job.cl_cap * BYTES_PER_CLUSTER + job.tl_cap * BYTES_PER_TRACKLET


class Scheduler:
    """FIFO admission by free slot and HBM budget; executor-agnostic.

    executor.launch(slot, job) enqueues the chunk; executor.done(slot) says
    whether the slot's chunk has finished on the device; executor.finish(slot,
    job) reads its status and returns True when the chunk must run again (its
    capacities were updated)."""

    def __init__(self, executor, n_slots: int, budget_bytes: int):
        if n_slots < 1:
            raise ValueError("need at least one slot")
        self.ex = executor
        self.budget = int(budget_bytes)
        self.queue: collections.deque = collections.deque()
        self.free: List[int] = list(range(n_slots))[::-1]
        self.busy: Dict[int, Job] = {}
        self.in_use = 0
        self.peak_in_use = 0
        self.max_concurrent = 0

    def arrive(self, job: Job, now: float):
        job.arrival = now
        self.queue.append(job)

    @property
    def idle(self) -> bool:
        return not self.queue and not self.busy

    def step(self, now: float) -> List[Job]:
        """Retire finished chunks, then admit waiting ones; returns the
        chunks completed in this step."""
        completed = []
        for slot, job in list(self.busy.items()):
            if not self.ex.done(slot):
                continue
            again = self.ex.finish(slot, job)
            del self.busy[slot]
            self.in_use -= job.nbytes
            self.free.append(slot)
            if again:
                job.retries += 1
                self.queue.appendleft(job)
            else:
                job.done = now
                completed.append(job)
        while self.queue and self.free:
            job = self.queue[0]
            nb = job_bytes(job)
            if nb > self.budget:
                self.queue.popleft()
                job.error = f"needs {nb} bytes, budget {self.budget}"
                job.done = now
                completed.append(job)
                continue
            if self.in_use + nb > self.budget:
                break  # head of line waits for memory
            self.queue.popleft()
            slot = self.free.pop()
            job.nbytes = nb
            job.start = now if job.start < 0 else job.start
            self.in_use += nb
            self.peak_in_use = max(self.peak_in_use, self.in_use)
            self.ex.launch(slot, job)
            self.busy[slot] = job
            self.max_concurrent = max(self.max_concurrent, len(self.busy))
        return completed


def run_stream(sched: Scheduler, jobs: List[Job], arrivals: np.ndarray,
               clock: Callable[[], float] = time.perf_counter, poll_s: float = 2e-4,
               on_complete: Optional[Callable[[Job], None]] = None,
               sleep: Callable[[float], None] = time.sleep) -> List[Job]:
    """Feed jobs at their arrival times (seconds from the start) and run until
    every one has completed.  Returns the jobs in completion order."""
    order = np.argsort(arrivals, kind="stable")
    t0 = clock()
    nxt = 0
    done: List[Job] = []
    while len(done) < len(jobs):
        now = clock() - t0
        while nxt < len(jobs) and arrivals[order[nxt]] <= now:
            j = jobs[order[nxt]]
            sched.arrive(j, float(arrivals[order[nxt]]))
            nxt += 1
        fin = sched.step(now)
        for j in fin:
            if on_complete:
                on_complete(j)
        done.extend(fin)
        if not fin:
            sleep(poll_s)
    return done


def latency_stats(jobs: List[Job]) -> dict:
    lat = np.array([j.latency for j in jobs if j.error is None]) * 1e3
    if len(lat) == 0:
        return dict(p50_ms=None, p99_ms=None, mean_ms=None)
    return dict(p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                mean_ms=float(lat.mean()), max_ms=float(lat.max()))


class GpuExecutor:
    """Slots = library contexts, one torch stream each, sized for the largest
    chunk; output buffers are allocated per chunk on the slot's stream."""

    def __init__(self, n_slots: int, max_units: int, max_time_bins: int, max_clusters: int,
                 max_tracklets: int, param_overrides: Optional[dict] = None,
                 noise_sigma: float = 1.0, keep_outputs: bool = False, tuning: Optional[dict] = None,
                 max_samples: Optional[int] = None):
        import torch

        self.torch = torch
        self.keep = keep_outputs
        self.max_clusters = max_clusters
        self.max_tracklets = max_tracklets
        self.streams = [torch.cuda.Stream() for _ in range(n_slots)]
        self.recos = [tpc.Reco(max_units, max_time_bins, max_clusters, max_tracklets,
                               param_overrides=param_overrides, noise_sigma=noise_sigma,
                               stream=s, max_samples=max_samples) for s in self.streams]
        if tuning:
            for r in self.recos:
                r.set_tuning(**tuning)
        self.events = [torch.cuda.Event() for _ in range(n_slots)]
        self.live: Dict[int, tuple] = {}

    def close(self):
        for r in self.recos:
            r.close()

    def _outputs(self, reco: tpc.Reco, job: Job):
        cl = reco.alloc_clusters(job.n_units, job.n_time_bins, job.cl_cap)
        links = reco.alloc_links(job.cl_cap)
        tl = reco.alloc_tracklets(job.tl_cap)
        tr = reco.alloc_tracks(job.tl_cap, job.cl_cap, job.cl_cap)
        return cl, links, tl, tr

    def launch(self, slot: int, job: Job):
        torch = self.torch
        reco = self.recos[slot]
        job.cl_cap = min(job.cl_cap, self.max_clusters)
        job.tl_cap = min(job.tl_cap, self.max_tracklets)
        with torch.cuda.stream(self.streams[slot]):
            bufs = self._outputs(reco, job)
            reco.process(job.zs, *bufs, zs_s=job.zs.get("_struct"))
            self.events[slot].record(self.streams[slot])
        self.live[slot] = bufs

    def done(self, slot: int) -> bool:
        return self.events[slot].query()

    def finish(self, slot: int, job: Job) -> bool:
        bufs = self.live.pop(slot)
        c = self.recos[slot].sync(raise_on_error=False)
        job.counts = c
        if c["status"] == -2:  # capacity: rerun with what the device needed
            req = c["required_by"]
            # track hits are bounded by the cluster capacity, tracks by the
            # tracklet capacity (see _outputs)
            need_cl = max(req.get("clusters", 0), req.get("hits", 0))
            need_tl = max(req.get("tracklets", 0), req.get("tracks", 0))
            if need_cl > self.max_clusters:
                job.error = f"chunk needs {need_cl} clusters, slots hold {self.max_clusters}"
                return False
            if need_tl > self.max_tracklets:
                job.error = f"chunk needs {need_tl} tracklets, slots hold {self.max_tracklets}"
                return False
            if need_cl:
                job.cl_cap = need_cl + need_cl // 16
                job.tl_cap = max(job.tl_cap, job.cl_cap // 8)
            if need_tl:
                job.tl_cap = max(job.tl_cap, need_tl + need_tl // 16)
            return True
        if c["status"] != 0:
            job.error = tpc.load().tpc_status_string(c["status"]).decode()
        elif self.keep:
            job.outputs = dict(clusters=bufs[0], links=bufs[1], tracklets=bufs[2], tracks=bufs[3])
        return False


def make_job(i: int, ev, device="cuda", **cap_kw) -> Job:
    """A job with its input copied into HBM (done before the stream starts)."""
    zs = tpc.to_device_zs(ev.pad, ev.time, ev.adc, ev.row_start, ev.n_units, ev.n_time_bins,
                          device=device)
    zs["_struct"] = tpc.zs_struct(zs)
    cl, tl = estimate_caps(ev.n_samples, **cap_kw)
    return Job(i, zs, ev.n_units, ev.n_time_bins, ev.n_samples, cl_cap=cl, tl_cap=tl)


def poisson_arrivals(n: int, rate_hz: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_hz, n))

"""Batched form over slices of a frame's units, run concurrently.

A unit (one sector of one frame) is reconstructed independently of every
other unit, so a frame can be cut into slices of consecutive units and each
slice reconstructed by its own library context on its own HIP stream.  By
default slice i starts when slice i-1 has finished clustering (other start
points are a choice), so the slices run about one stage apart: the stages
whose end is bound by latency (the longest tracks of the refit and of the
FP64 refit, the longest chains of the tracklet building, the longest
tracklets of the following) overlap with throughput-bound stages of the next
slice.  Each slice writes its own outputs, equal to those of one
call over its units.  The launch sequence of all slices can be captured into
one HIP graph (the slice streams fork from and join the capturing stream).
"""
from __future__ import annotations

from typing import List, Optional

import numpy as np

from . import tpc

NROW = tpc.NROW


def split_units(row_start: np.ndarray, n_units: int, n_parts: int) -> List[int]:
    """Unit boundaries u_0 = 0 < u_1 < ... < u_n = n_units that balance the
    samples of the slices (row_start: per (unit, row) first sample)."""
    n_parts = max(1, min(int(n_parts), int(n_units)))
    cum = np.asarray(row_start, np.int64)[np.arange(n_units + 1) * NROW]
    total = cum[-1] - cum[0]
    bounds = [0]
    for k in range(1, n_parts):
        target = cum[0] + total * k / n_parts
        u = int(np.argmin(np.abs(cum - target)))
        u = min(max(u, bounds[-1] + 1), n_units - (n_parts - k))
        bounds.append(u)
    bounds.append(int(n_units))
    return bounds


class Slice:
    """One slice: its input views, library context, stream and outputs."""

    def __init__(self, zs: dict, row_start_host: np.ndarray, u0: int, u1: int, device,
                 cl_ratio: int, tl_ratio: int, noise_sigma: float,
                 param_overrides: Optional[dict], tuning: Optional[dict]):
        torch = tpc._torch()
        s0 = int(row_start_host[u0 * NROW])
        s1 = int(row_start_host[u1 * NROW])
        rs = (row_start_host[u0 * NROW:u1 * NROW + 1].astype(np.int64) - s0).astype(np.uint32)
        self.u0, self.u1, self.s0, self.s1 = u0, u1, s0, s1
        self.zs = dict(pad=zs["pad"][s0:s1], time=zs["time"][s0:s1], adc=zs["adc"][s0:s1],
                       row_start=torch.from_numpy(rs.view(np.int32)).to(device),
                       n_samples=s1 - s0, n_units=u1 - u0, n_time_bins=zs["n_time_bins"])
        ns = max(s1 - s0, 1)
        self.max_clusters = max(ns // cl_ratio, 1 << 16)
        self.max_tracklets = max(self.max_clusters // tl_ratio, 1 << 14)
        self.stream = torch.cuda.Stream(device)
        nu = u1 - u0
        self.reco = tpc.Reco(nu, zs["n_time_bins"], self.max_clusters, self.max_tracklets,
                             param_overrides=param_overrides, noise_sigma=noise_sigma,
                             device=str(device), stream=self.stream, max_samples=ns)
        if tuning:
            self.reco.set_tuning(**tuning)
        r = self.reco
        self.cl = r.alloc_clusters(nu, zs["n_time_bins"], self.max_clusters)
        self.links = r.alloc_links(self.max_clusters)
        self.tl = r.alloc_tracklets(self.max_tracklets)
        self.tr = r.alloc_tracks(self.max_tracklets, self.max_clusters, self.max_clusters)
        self.mark = torch.cuda.Event()  # where the next slice may start
        self.done = torch.cuda.Event()

    def enqueue(self, start, after, stagger: str):
        """Enqueue the slice on its stream behind the events start and after
        (the previous slice's stagger point, or None)."""
        torch = tpc._torch()
        self.stream.wait_event(start)
        if after is not None:
            self.stream.wait_event(after)
        with torch.cuda.stream(self.stream):
            self.reco.cluster(self.zs, self.cl)
            if stagger == "cluster":
                self.mark.record(self.stream)
            self.reco.find_neighbours(self.cl, self.links)
            self.reco.build_tracklets(self.cl, self.links, self.tl)
            if stagger == "tracklets":
                self.mark.record(self.stream)
            self.reco.fit_tracks(self.cl, self.links, self.tl, self.tr)
            self.done.record(self.stream)


class Pipeline:
    """A frame's units in n_parts slices, each slice one stage behind the
    previous one.  enqueue() forks the slices from the current stream and
    joins them back into it."""

    STAGGERS = ("cluster", "tracklets", "none")

    def __init__(self, zs: dict, n_parts: int, device="cuda", cl_ratio: int = 8,
                 tl_ratio: int = 8, noise_sigma: float = 1.0,
                 param_overrides: Optional[dict] = None, tuning: Optional[dict] = None,
                 stagger: str = "cluster"):
        """stagger: the point of slice i-1 after which slice i starts (the end
        of its clustering, of its tracklet building, or no wait)."""
        torch = tpc._torch()
        if stagger not in self.STAGGERS:
            raise ValueError(f"stagger must be one of {self.STAGGERS}")
        self.stagger = stagger
        self.device = torch.device(device)
        rs = zs["row_start"].cpu().numpy().view(np.uint32)
        self.bounds = split_units(rs, zs["n_units"], n_parts)
        self.slices = [Slice(zs, rs, a, b, self.device, cl_ratio, tl_ratio, noise_sigma,
                             param_overrides, tuning)
                       for a, b in zip(self.bounds[:-1], self.bounds[1:])]
        self.start = torch.cuda.Event()

    @property
    def n_parts(self) -> int:
        return len(self.slices)

    def enqueue(self):
        torch = tpc._torch()
        main = torch.cuda.current_stream(self.device)
        self.start.record(main)
        prev = None
        for sl in self.slices:
            after = prev.mark if prev is not None and self.stagger != "none" else None
            sl.enqueue(self.start, after, self.stagger)
            prev = sl
        for sl in self.slices:
            main.wait_event(sl.done)

    def sync(self) -> dict:
        """Counts summed over the slices (raises on a device error)."""
        tot = {}
        for sl in self.slices:
            c = sl.reco.sync()
            for k, v in c.items():
                if isinstance(v, (int, np.integer)) and k != "status":
                    tot[k] = tot.get(k, 0) + int(v)
        return tot

    def close(self):
        for sl in self.slices:
            sl.reco.close()

#!/usr/bin/env python3
"""Benchmark: TPC clusters reconstructed per second on one MI355X.

Workload (headline): a 2 ms slice of 50 kHz minimum-bias Pb-Pb, 100
collisions overlapping in 10,500 time bins, 36 sectors x 152 pad rows,
seed 303, reconstructed in one graph-captured launch sequence (the batched
form).  Inputs are resident in HBM before the timed region starts.

Beside it: the plain form (one central collision per synchronous call, seed
202) with its per-call latency, per-stage timing of the library's kernels
(HIP events on the library's stream) for the roofline, and the CPU oracle
timed on a bounded sample of the same workload.

Prints one JSON line.  ``--gpus N`` with N > 1 is not supported: the path
runs on one GPU.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "TPC clusters reconstructed/sec on 1 MI355X (batched vs plain); p50/p99 chunk latency"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Algorithmic bytes each stage must move, per unit of work:
# samples are (pad, time, adc) u16; a cluster record is y_fx, z_fx (i32),
# pad, time, s2pad, s2time (f32), qtot, qmax, ppad, ptime (u16), flags (u8).
def stage_bytes(ns, nc, n_ur, nblk):
    rec = 4 * 2 + 4 * 4 + 2 * 4 + 1
    return {
        "sample_index": 2 * ns + 4 * n_ur * (nblk + 1),
        "cluster_count": 6 * ns,
        "cluster_emit": 6 * ns + rec * nc,
        "cluster_grid": 2 * nc + 4 * n_ur * (nblk + 1),
        "neighbours": 8 * nc + 8 * nc,
    }


def make_reco(tpc, ev, stream, max_clusters, max_tracklets, noise):
    return tpc.Reco(ev.n_units, ev.n_time_bins, max_clusters, max_tracklets,
                    noise_sigma=noise, stream=stream)


def buffers(reco, ev, max_clusters, max_tracklets):
    cl = reco.alloc_clusters(ev.n_units, ev.n_time_bins, max_clusters)
    links = reco.alloc_links(max_clusters)
    tl = reco.alloc_tracklets(max_tracklets)
    tr = reco.alloc_tracks(max_tracklets, max_clusters, max_clusters)
    return cl, links, tl, tr


def cpu_baseline(ev, target_s=12.0):
    """The oracle (full chain) on the whole slice, repeated until about
    target_s seconds of host work, on the host's cores."""
    import oracle

    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count() or 1
    threads = max(1, min(16, ncpu))
    total_t, total_c, reps = 0.0, 0, 0
    while total_t < target_s and reps < 50:
        t0 = time.perf_counter()
        res = oracle.process(ev.pad, ev.time, ev.adc, ev.row_start, ev.n_units, ev.n_time_bins,
                             n_threads=threads)
        total_t += time.perf_counter() - t0
        total_c += len(res["clusters"]["y_fx"])
        reps += 1
    return dict(value=total_c / total_t, unit="clusters/s", cores=threads, kind="oracle",
                sample=f"full chain on the whole 2 ms slice (seed 303), {reps} repetition(s): "
                       f"{total_c} clusters in {total_t:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain-form leg")
    ap.add_argument("--no-graph", action="store_true", help="time eager launches instead")
    ap.add_argument("--collisions", type=int, default=100)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} not supported; the reconstruction path runs on one "
              "GPU (frames shard across GPUs with no exchange; see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch

    import tpcsynth
    from paper_2208_07412_amd import tpc

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t0 = time.perf_counter()
    cfg = tpcsynth.config_c3(303, args.collisions)
    ev = tpcsynth.generate(cfg, 303)
    log(f"[bench] generated slice: {ev.n_samples} samples, {ev.n_time_bins} bins "
        f"in {time.perf_counter() - t0:.1f}s")
    ns = ev.n_samples
    max_cl = max(ns // 8, 1 << 20)
    max_tl = max(max_cl // 8, 1 << 16)
    stream = torch.cuda.Stream(dev)
    reco = make_reco(tpc, ev, stream, max_cl, max_tl, 1.0)
    zs = tpc.to_device_zs(ev.pad, ev.time, ev.adc, ev.row_start, ev.n_units, ev.n_time_bins, dev)
    zs_s = tpc.zs_struct(zs)
    cl, links, tl, tr = buffers(reco, ev, max_cl, max_tl)
    torch.cuda.synchronize()

    # warm-up and counts
    with torch.cuda.stream(stream):
        for _ in range(max(args.warmup, 1)):
            reco.process(zs, cl, links, tl, tr, zs_s)
    counts = reco.sync()
    nc = counts["n_clusters"]
    log(f"[bench] clusters {nc} tracklets {counts['n_tracklets']} tracks {counts['n_tracks']} "
        f"fallback {counts['n_fallback']}")

    # per-stage timing (eager launches, events on the library's stream)
    reco.profile(True)
    with torch.cuda.stream(stream):
        for _ in range(3):
            reco.process(zs, cl, links, tl, tr, zs_s)
    prof = reco.profile_read()
    reco.profile(False)
    reco.sync()
    stages = {k: v[0] / max(v[1], 1) for k, v in prof.items()}
    log("[bench] stage ms: " + ", ".join(f"{k} {v:.3f}" for k, v in stages.items()))

    # timed region: the batched form, one graph replay per step
    graph = None
    if not args.no_graph:
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=stream):
            reco.process(zs, cl, links, tl, tr, zs_s)
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            graph.replay()
        reco.sync()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    with torch.cuda.stream(stream):
        e0.record(stream)
        for _ in range(args.steps):
            if graph is not None:
                graph.replay()
            else:
                reco.process(zs, cl, links, tl, tr, zs_s)
        e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms_step = e0.elapsed_time(e1) / args.steps
    c2 = reco.sync()
    assert c2["n_clusters"] == nc, "graph replay changed the result"
    value = nc / (ms_step / 1e3)
    log(f"[bench] batched: {ms_step:.3f} ms/step ({wall / args.steps * 1e3:.3f} wall), "
        f"{value:.4g} clusters/s")

    # roofline of the dominant HBM-bound stage
    n_ur = ev.n_units * 152
    nblk = (ev.n_time_bins + 7) // 8
    sb = stage_bytes(ns, nc, n_ur, nblk)
    dom = max(stages, key=lambda k: stages[k])
    hbm_dom = max(sb, key=lambda k: stages.get(k, 0.0))
    ach = sb[hbm_dom] / (stages[hbm_dom] / 1e3) / 1e9
    roofline = dict(bound="hbm", kernel=hbm_dom, achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=ach / HBM_PEAK_GBS, traffic=None, bytes_per_launch=sb[hbm_dom],
                    ms_per_launch=stages[hbm_dom], dominant_stage=dom,
                    dominant_stage_ms=stages[dom])

    out = dict(metric=METRIC, value=value, unit="clusters/s", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=ms_step, higher_is_better=True, scaling="weak",
               vs_baseline=None, dtype="f32+int", data="synthetic",
               config=dict(workload="2 ms Pb-Pb slice at 50 kHz: 100 minimum-bias collisions, "
                           "36 sectors x 152 rows, 10500 time bins, seed 303",
                           form="batched (graph replay)" if graph is not None else "eager",
                           samples=ns, clusters=nc, tracks=counts["n_tracks"]),
               roofline=roofline, stages_ms=stages)
    del graph

    # plain form: one central collision per synchronous call
    if not args.no_plain:
        ev2 = tpcsynth.generate(tpcsynth.config_c2(), 202)
        mc2 = max(ev2.n_samples // 4, 1 << 16)
        mt2 = max(mc2 // 4, 1 << 14)
        reco2 = make_reco(tpc, ev2, stream, mc2, mt2, 1.0)
        zs2 = tpc.to_device_zs(ev2.pad, ev2.time, ev2.adc, ev2.row_start, ev2.n_units,
                               ev2.n_time_bins, dev)
        b2 = buffers(reco2, ev2, mc2, mt2)
        lat = []
        with torch.cuda.stream(stream):
            for i in range(args.warmup + max(args.steps, 20)):
                t = time.perf_counter()
                reco2.process(zs2, *b2)
                c = reco2.sync()
                if i >= args.warmup:
                    lat.append(time.perf_counter() - t)
        lat = np.array(lat)
        n2 = c["n_clusters"]
        out["plain"] = dict(workload="one central Pb-Pb collision (3000 + 600 tracks), seed 202",
                            clusters=n2, value=n2 / lat.mean(), unit="clusters/s",
                            p50_ms=float(np.percentile(lat, 50) * 1e3),
                            p99_ms=float(np.percentile(lat, 99) * 1e3))
        out["batched_over_plain"] = value / out["plain"]["value"]
        reco2.close()
        log(f"[bench] plain: {out['plain']}")
    reco.close()

    if not args.no_cpu:
        t = time.perf_counter()
        out["cpu_baseline"] = cpu_baseline(ev)
        log(f"[bench] cpu baseline in {time.perf_counter() - t:.1f}s: {out['cpu_baseline']}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

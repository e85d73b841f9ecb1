#!/usr/bin/env python3
"""Benchmark: TPC clusters reconstructed per second on one MI355X.

Workload (headline): a 2 ms slice of 50 kHz minimum-bias Pb-Pb, 100
collisions overlapping in 10,500 time bins, 36 sectors x 152 pad rows,
seed 303, reconstructed as one graph replay per step (the batched form: one
library context over the whole slice, or the units cut into slices on
concurrent streams, whichever is faster).  Inputs are resident in HBM before
the timed region starts.

Beside it: the plain form (one central collision per synchronous call, seed
202, default launch shapes, no graph) with its per-call latency; the serving
form (a Poisson stream of chunks of 10-200 collisions, seed 404, at 80% of
the measured capacity, admitted continuously over several streams) with its
p50/p99 chunk latency; per-stage timing of the library's kernels (HIP events
on the library's stream) for the roofline; and the CPU oracle timed on a
bounded sample of the same workload.  Launch shapes of the batched and
serving forms are picked by the autotuner on the workload itself.

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
FP32_PEAK_TFLOPS = 157.3  # MI355X vector FP32 (published)
# FP32 operations of one unit of following work (FMA = 2), from the formulas:
# helix step with analytic Jacobian (8-point quadrature) and covariance
# transport; chi2 of one candidate against the inverted residual covariance;
# one Kalman update (gain, state, covariance).
FLOPS_STEP, FLOPS_CAND, FLOPS_UPDATE = 220, 12, 122
METRIC = "TPC clusters reconstructed/sec on 1 MI355X (batched vs plain); p50/p99 chunk latency"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Algorithmic bytes each stage must move, per unit of work:
# samples are (pad, time, adc) u16; a cluster record is y_fx, z_fx (i32),
# pad, time, s2pad, s2time (f32), qtot, qmax, ppad, ptime (u16), flags (u8).
def stage_bytes(ns, nc, n_ur, T, W=24):
    rec = 4 * 2 + 4 * 4 + 2 * 4 + 1
    raw = 24                 # raw record per cluster between the two clusterizer passes
    nblk_s = (T + 3) // 4   # sample index: one entry per 4 time bins
    nblk_c = (T + 1) // 2   # cluster grid: one entry per 2 time bins
    nwin = n_ur * ((T + W - 1) // W)
    return {
        "sample_index": 2 * ns + 4 * n_ur * (nblk_s + 1),
        "cluster_peaks": 6 * ns + raw * nc + 4 * nwin,
        "cluster_output": raw * nc + rec * nc + 4 * nwin,
        "cluster_grid": 2 * nc + 4 * n_ur * (nblk_c + 1),
        "neighbours": 8 * nc + 8 * nc,
    }


def source_hash(files):
    """sha256 over the given source files (repository-relative), in order."""
    import hashlib

    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()


def pmc_traffic(files, stage, kernel_name):
    """HBM bytes per launch of a stage's kernel(s) from the committed rocprofv3
    counter summary (FETCH_SIZE + WRITE_SIZE scaled by a plain copy of known
    size), or None when the kernel sources changed since the counters were
    taken, the summary is for another launch shape, or none exists."""
    path = os.path.join(ROOT, "profiles", f"pmc_{stage}_c3_slice.md")
    if not os.path.exists(path):
        return None
    rec = None
    for line in open(path):
        if line.startswith("traffic_json: "):
            rec = json.loads(line[len("traffic_json: "):])
    if rec is None or not rec.get("kernel", "").startswith(kernel_name):
        return None
    return rec["bytes_per_launch"] if rec.get("source_sha256") == source_hash(files) else None


KERNEL_SOURCES = {
    "cluster_peaks": ("paper_2208_07412_amd/csrc/common.hpp", "paper_2208_07412_amd/csrc/k_cluster.hpp"),
    "following": ("paper_2208_07412_amd/csrc/common.hpp", "paper_2208_07412_amd/csrc/k_cluster.hpp",
                  "paper_2208_07412_amd/csrc/k_links.hpp", "paper_2208_07412_amd/csrc/k_track.hpp"),
}


def make_reco(tpc, ev, stream, max_clusters, max_tracklets, noise):
    return tpc.Reco(ev.n_units, ev.n_time_bins, max_clusters, max_tracklets,
                    noise_sigma=noise, stream=stream, max_samples=max(ev.n_samples, 1))


def buffers(reco, ev, max_clusters, max_tracklets):
    cl = reco.alloc_clusters(ev.n_units, ev.n_time_bins, max_clusters)
    links = reco.alloc_links(max_clusters)
    tl = reco.alloc_tracklets(max_tracklets)
    tr = reco.alloc_tracks(max_tracklets, max_clusters, max_clusters)
    return cl, links, tl, tr


def host_threads():
    """Threads the oracle may use: the host's CPU share for one GPU.  The GPU
    boxes give one GPU a share of 16 CPUs (whatever os.cpu_count() shows
    there); a smaller affinity mask is honoured."""
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count() or 1
    return max(1, min(16, ncpu)), ncpu


def _time_oracle(ev, threads, target_s, max_reps=50, noise=1.0):
    """The oracle's full chain on ev, repeated until about target_s seconds."""
    import oracle

    params = oracle.default_params(noise)
    total_t, total_c, reps = 0.0, 0, 0
    while (total_t < target_s or reps == 0) and reps < max_reps:
        t0 = time.perf_counter()
        res = oracle.process(ev.pad, ev.time, ev.adc, ev.row_start, ev.n_units, ev.n_time_bins,
                             params=params, n_threads=threads)
        total_t += time.perf_counter() - t0
        total_c += len(res["clusters"]["y_fx"])
        reps += 1
    return total_c / total_t, total_c, total_t, reps, res


def stress_errors(gpu, res, floors=(1.0, 1.0, 1e-2, 1e-2, 0.1)):
    """Per-parameter deviation of the GPU tracks from the FP64 oracle's, over
    tracks of the same tracklet with the same kept hits: |gpu - oracle| /
    max(|oracle|, floor), as median / p99 / max per parameter."""
    fit = res["fit"]
    kept = np.nonzero(fit["kept"])[0]
    okept = set(kept.tolist())
    owner = fit["cluster_owner"]
    rels = []
    same = 0
    for j, t in enumerate(gpu["tracklet"]):
        t = int(t)
        if t not in okept:
            continue
        h = fit["hits"][t]
        oh = h[h >= 0]
        oh = np.sort(oh[owner[oh] == t])
        gh = np.sort(gpu["hits"][gpu["hit_start"][j]:gpu["hit_start"][j + 1]])
        if not np.array_equal(gh, oh):
            continue
        same += 1
        op = fit["par"][t]
        rels.append(np.abs(gpu["par"][j].astype(np.float64) - op) /
                    np.maximum(np.abs(op), np.array(floors)))
    out = dict(tracks_compared=same, gpu_tracks=len(gpu["tracklet"]), oracle_tracks=len(kept),
               floors=list(floors))
    if rels:
        R = np.array(rels)
        q = np.percentile(R, [50, 99, 100], axis=0)
        for i, name in enumerate(("y", "z", "snp", "tgl", "qpt")):
            out[name] = dict(median=float(q[0][i]), p99=float(q[1][i]), max=float(q[2][i]))
    return out


def cpu_baseline(ev, stress=None, target_s=10.0):
    """The oracle as it stands, on this machine's host cores: all threads of
    one GPU's CPU share on the whole 2 ms slice (the reported value), one
    thread on a bounded sample of its units, and both on one sector (C1) and
    one central collision (C2).  With the precision-stress chunk's GPU tracks
    (stress), the oracle also runs that chunk and the per-parameter deviation
    of the FP32 GPU fit from its FP64 fit is reported beside the timing."""
    import tpcsynth

    threads, ncpu = host_threads()
    v, nc, tt, reps, _ = _time_oracle(ev, threads, target_s)
    out = dict(value=v, unit="clusters/s", cores=threads, kind="oracle",
               sample=f"full chain on the whole 2 ms slice (seed 303), {reps} repetition(s): "
                      f"{nc} clusters in {tt:.1f} s on {threads} threads "
                      f"(host shows {ncpu} CPUs; one GPU's share is 16)")
    sub = tpcsynth.select_units(ev, [0, 9, 18, 27])
    v1, nc1, tt1, reps1, _ = _time_oracle(sub, 1, 0.0, max_reps=1)
    out["single_thread"] = dict(value=v1, unit="clusters/s", cores=1,
                                sample=f"4 of the slice's 36 sectors (0, 9, 18, 27), "
                                       f"{nc1} clusters in {tt1:.1f} s")
    for name, cfg, seed in (("c1", tpcsynth.config_c1(), 101), ("c2", tpcsynth.config_c2(), 202)):
        e = tpcsynth.generate(cfg, seed)
        va, nca, tta, ra, _ = _time_oracle(e, threads, 1.0)
        vs, ncs, tts, rs_, _ = _time_oracle(e, 1, 1.0)
        out[name] = dict(all_threads=va, single_thread=vs, unit="clusters/s",
                         clusters=nca // ra, ms_all_threads=tta / ra * 1e3,
                         ms_single_thread=tts / rs_ * 1e3)
    if stress is not None:
        sev, gpu = stress
        vsx, ncx, ttx, rx, res = _time_oracle(sev, threads, 0.0, max_reps=1, noise=2.0)
        out["precision_stress"] = dict(value=vsx, unit="clusters/s", cores=threads,
                                       clusters=ncx, s=ttx,
                                       error_vs_gpu=stress_errors(gpu, res))
    return out


def serve_leg(args, torch, tpcsynth, tuning):
    """Poisson stream of chunks (10-200 collisions each) admitted continuously
    on several streams; capacity first (every pool chunk arrives at once),
    then arrivals at 80% of it."""
    from paper_2208_07412_amd import serve

    t = time.perf_counter()
    pool = []
    for i in range(args.serve_pool):
        ev = tpcsynth.generate(tpcsynth.config_chunk(404, i), 404 + i)
        pool.append(serve.make_job(i, ev))
        del ev
    T = max(j.n_time_bins for j in pool)
    max_cl = max(j.cl_cap for j in pool)
    max_tl = max(j.tl_cap for j in pool)
    log(f"[bench] serving pool: {[j.n_time_bins // 100 - 5 for j in pool]} collisions, "
        f"{sum(j.n_samples for j in pool)} samples, made in {time.perf_counter() - t:.1f}s")
    ex = serve.GpuExecutor(args.serve_slots, 36, T, max_cl, max_tl, tuning=tuning,
                           max_samples=max(j.n_samples for j in pool))
    free, _ = torch.cuda.mem_get_info()
    budget = int(free * 0.8)

    def copies(idx):
        return [serve.Job(k, pool[i].zs, pool[i].n_units, pool[i].n_time_bins, pool[i].n_samples,
                          cl_cap=pool[i].cl_cap, tl_cap=pool[i].tl_cap) for k, i in enumerate(idx)]

    def run(jobs, arrivals):
        sched = serve.Scheduler(ex, args.serve_slots, budget)
        t0 = time.perf_counter()
        done = serve.run_stream(sched, jobs, arrivals)
        span = time.perf_counter() - t0
        bad = [j.error for j in done if j.error]
        if bad:
            raise RuntimeError(f"serving errors: {bad[:3]}")
        return done, span, sched

    idx = list(range(len(pool)))
    run(copies(idx), np.zeros(len(idx)))  # warm-up: allocator, first launches
    done, span, _ = run(copies(idx + idx), np.zeros(2 * len(idx)))
    cap_chunks = len(done) / span
    cap_clusters = sum(j.counts["n_clusters"] for j in done) / span
    rate = 0.8 * cap_chunks
    n = args.serve_chunks
    rng = np.random.default_rng(404)
    sel = [int(x) for x in rng.integers(0, len(pool), n)]
    arr = serve.poisson_arrivals(n, rate, seed=405)
    done, span, sched = run(copies(sel), arr)
    ncl = sum(j.counts["n_clusters"] for j in done)
    st = serve.latency_stats(done)
    ex.close()
    # the plain per-chunk form on the same pool: one synchronous call per
    # chunk, default launch shapes, no graph, one chunk on the GPU at a time
    from paper_2208_07412_amd import tpc

    ms_max = max(j.n_samples for j in pool)
    reco = tpc.Reco(36, T, max_cl, max_tl, max_samples=ms_max)
    bufs = (reco.alloc_clusters(36, T, max_cl), reco.alloc_links(max_cl),
            reco.alloc_tracklets(max_tl), reco.alloc_tracks(max_tl, max_cl, max_cl))
    plain_s, plain_c = 0.0, 0
    for rep in range(2):
        for j in pool:
            bufs[0].s.n_time_bins = j.n_time_bins
            t = time.perf_counter()
            reco.process(j.zs, *bufs)
            c = reco.sync()
            if rep:
                plain_s += time.perf_counter() - t
                plain_c += c["n_clusters"]
    reco.close()
    return dict(workload="Poisson stream of time-frame chunks, 10-200 minimum-bias collisions "
                         "each (100 n + 500 bins), seed 404", pool=len(pool), chunks=n,
                slots=args.serve_slots, capacity_chunks_per_s=cap_chunks,
                capacity_clusters_per_s=cap_clusters, rate_hz=rate, clusters_per_s=ncl / span,
                p50_ms=st["p50_ms"], p99_ms=st["p99_ms"], mean_ms=st["mean_ms"],
                max_concurrent=sched.max_concurrent,
                reruns=sum(j.retries for j in done),
                plain_chunks=dict(value=plain_c / plain_s, unit="clusters/s",
                                  form="each pool chunk in one synchronous call, default "
                                       "launch shapes, no graph"),
                capacity_over_plain_chunks=cap_clusters / (plain_c / plain_s))


def stress_leg(torch, tpcsynth, tpc, stream, n_coll=20):
    """Precision-stress chunk (30% loopers at 0.05-0.2 GeV/c, noise 2 ADC,
    10% dead pads): how often the FP32 refit hands a track to the FP64 one,
    and the time of the two refit stages."""
    ev = tpcsynth.generate(tpcsynth.config_chunk(505, 0, stress=True, n_coll=n_coll), 505)
    mc = max(ev.n_samples // 6, 1 << 16)
    mt = max(mc // 8, 1 << 14)
    reco = tpc.Reco(ev.n_units, ev.n_time_bins, mc, mt, noise_sigma=2.0, stream=stream,
                    max_samples=ev.n_samples)
    zs = tpc.to_device_zs(ev.pad, ev.time, ev.adc, ev.row_start, ev.n_units, ev.n_time_bins)
    b = buffers(reco, ev, mc, mt)
    with torch.cuda.stream(stream):
        reco.process(zs, *b)
    c = reco.sync()
    gtr = tpc.tracks_to_host(b[3], c["n_clusters"], 0)
    gpu = dict(tracklet=gtr["tracklet"], par=gtr["par"], hits=gtr["hits"],
               hit_start=gtr["hit_start"])
    reco.profile(True)
    with torch.cuda.stream(stream):
        for _ in range(3):
            reco.process(zs, *b)
    prof = reco.profile_read()
    reco.profile(False)
    reco.sync()
    reco.close()
    ms = {k: v[0] / max(v[1], 1) for k, v in prof.items()}
    res = dict(workload=f"precision-stress chunk, {n_coll} collisions, seed 505",
               samples=ev.n_samples, clusters=c["n_clusters"], tracks=c["n_tracks"],
               fp64_refits=c["n_fallback"], fp64_rate=c["n_fallback"] / max(c["n_tracks"], 1),
               fp64_not_pd=c["n_fallback_fail"], flagged_not_pd=c["n_not_pd"],
               refit_ms=ms["refit"], fp64_count_ms=ms["fp64_count"],
               total_ms=sum(ms.values()))
    return res, (ev, gpu)


def plain_sync(tpc, torch, reco, zs, b, stream, reps, warmup):
    """Per-call wall latency of synchronous reconstructions (enqueue + sync)."""
    lat = []
    with torch.cuda.stream(stream):
        for i in range(warmup + reps):
            t = time.perf_counter()
            reco.process(zs, *b)
            c = reco.sync()
            if i >= warmup:
                lat.append(time.perf_counter() - t)
    return np.array(lat), c


def plain_latency(tpc, torch, tpcsynth, stream, dev, args, reps=50):
    """One sector with 200 tracks (C1), one synchronous call at a time."""
    ev = tpcsynth.generate(tpcsynth.config_c1(), 101)
    mc = max(ev.n_samples // 4, 1 << 14)
    mt = max(mc // 4, 1 << 12)
    reco = make_reco(tpc, ev, stream, mc, mt, 1.0)
    zs = tpc.to_device_zs(ev.pad, ev.time, ev.adc, ev.row_start, ev.n_units, ev.n_time_bins, dev)
    b = buffers(reco, ev, mc, mt)
    lat, c = plain_sync(tpc, torch, reco, zs, b, stream, reps, max(args.warmup, 2))
    reco.close()
    return dict(workload="one sector, 200 tracks (seed 101)", clusters=c["n_clusters"],
                p50_ms=float(np.percentile(lat, 50) * 1e3),
                p99_ms=float(np.percentile(lat, 99) * 1e3), calls=reps)


def plain_collisions(tpc, torch, tpcsynth, stream, dev, cfg, seed=303):
    """The plain form on the slice's work: each of its collisions (the same
    multiplicities) as a frame of its own (500 bins, no pile-up), one
    synchronous call each, default launch shapes, no graph."""
    evs = []
    for i, col in enumerate(cfg.collisions):
        c1 = tpcsynth.EventConfig(f"C3-collision{i}", 500,
                                  [tpcsynth.Collision(0.0, col.n_prim, col.n_sec)])
        evs.append(tpcsynth.generate(c1, seed * 1000 + i))
    ns_max = max(e.n_samples for e in evs)
    mc = max(ns_max // 4, 1 << 16)
    mt = max(mc // 4, 1 << 14)
    reco = tpc.Reco(36, 500, mc, mt, stream=stream, max_samples=ns_max)
    b = buffers(reco, evs[0], mc, mt)
    zss = [tpc.to_device_zs(e.pad, e.time, e.adc, e.row_start, e.n_units, e.n_time_bins, dev)
           for e in evs]
    plain_sync(tpc, torch, reco, zss[0], b, stream, 0, 3)  # warm-up
    total_s, total_c, lat = 0.0, 0, []
    for zs in zss:
        l, c = plain_sync(tpc, torch, reco, zs, b, stream, 1, 0)
        total_s += float(l.sum())
        total_c += c["n_clusters"]
        lat.append(float(l[0]))
    reco.close()
    lat = np.array(lat)
    return dict(workload="the 2 ms slice's 100 collisions, each alone in 500 bins "
                         "(seed 303 multiplicities), one synchronous call each",
                collisions=len(evs), clusters=total_c, value=total_c / total_s,
                unit="clusters/s", s=total_s, p50_ms=float(np.percentile(lat, 50) * 1e3),
                p99_ms=float(np.percentile(lat, 99) * 1e3))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain-form leg")
    ap.add_argument("--no-graph", action="store_true", help="time eager launches instead")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving-form leg")
    ap.add_argument("--no-tune", action="store_true", help="keep the default launch shapes")
    ap.add_argument("--no-stress", action="store_true", help="skip the precision-stress leg")
    ap.add_argument("--no-h2d", action="store_true", help="skip the PCIe-inclusive figure")
    ap.add_argument("--no-pages", action="store_true", help="skip the raw-page decoding figure")
    ap.add_argument("--collisions", type=int, default=100)
    ap.add_argument("--slices", type=int, nargs="*", default=[2, 3, 4],
                    help="unit slices on concurrent streams tried for the batched form")
    ap.add_argument("--serve-pool", type=int, default=6, help="distinct chunks resident in HBM")
    ap.add_argument("--serve-chunks", type=int, default=36, help="chunks in the Poisson stream")
    ap.add_argument("--serve-slots", type=int, default=3, help="concurrent chunks (streams)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} not supported; the reconstruction path runs on one "
              "GPU (time frames are independent and would shard across GPUs with no exchange)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import tpcsynth
    from paper_2208_07412_amd import tpc
    from paper_2208_07412_amd.pipeline import Pipeline

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.calib_copy:
        # known traffic: 2^30 bytes read and 2^30 bytes written per launch
        a = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps(dict(calib_copy_bytes=1 << 30, launches=5)), flush=True)
        return
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

    tuning = None
    if not args.no_tune:
        from paper_2208_07412_amd.autotune import autotune

        def run_once():
            with torch.cuda.stream(stream):
                reco.process(zs, cl, links, tl, tr, zs_s)

        t = time.perf_counter()
        tuning = autotune(reco, run_once)
        log(f"[bench] autotune in {time.perf_counter() - t:.1f}s: {tuning}")

    # work counters of the following (a counting variant of its kernel, run once)
    reco.profile(False, count_work=True)
    with torch.cuda.stream(stream):
        reco.process(zs, cl, links, tl, tr, zs_s)
    fcounts = reco.sync()
    reco.profile(False)

    # per-stage timing (eager launches, events on the library's stream)
    reco.profile(True)
    with torch.cuda.stream(stream):
        for _ in range(3):
            reco.process(zs, cl, links, tl, tr, zs_s)
    prof = reco.profile_read()
    reco.profile(False)
    reco.sync()
    stages = {k: v[0] / 3 for k, v in prof.items()}  # per reconstruction
    log("[bench] stage ms: " + ", ".join(f"{k} {v:.3f}" for k, v in stages.items()))

    # quality-control histograms of the slice's outputs (HIP events on the
    # library's stream); algorithmic bytes: qtot, qmax (2 + 2) and
    # cluster_track (4) per cluster, hit_start (4) per track
    qc_hist = torch.empty(tpc.QC_BINS, dtype=torch.int32, device=dev)
    with torch.cuda.stream(stream):
        reco.qc_histograms(cl, tr, qc_hist)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(10):
            reco.qc_histograms(cl, tr, qc_hist)
        e1.record(stream)
    reco.sync()
    qc_ms = e0.elapsed_time(e1) / 10
    n_trk = int(tr["n_tracks"].item())
    qc_bytes = 8 * nc + 4 * (n_trk + 1)
    qc = dict(ms=qc_ms, bytes=qc_bytes, gb_per_s=qc_bytes / qc_ms / 1e6,
              hbm_frac=qc_bytes / qc_ms / 1e6 / 8000.0,
              clusters=int(qc_hist[tpc.QC_QTOT:tpc.QC_QTOT + 256].sum().item()),
              tracks=int(qc_hist[tpc.QC_NHITS:tpc.QC_NHITS + 153].sum().item()))
    log(f"[bench] qc histograms: {qc}")

    # track-model compression of the slice's outputs and its decoding (HIP
    # events on the library's stream).  Algorithmic bytes: per cluster y, z,
    # qtot, qmax, flags and its track (17 B) read, per track its parameters,
    # row, anchor and offsets (29 B) and 4 B per hit, the stream written;
    # decoding reads the stream and writes 20 B per cluster.
    comp = reco.alloc_compressed(max(nc, 1) * 2)
    dec = reco.alloc_decoded(max(nc, 1))
    with torch.cuda.stream(stream):
        reco.compress(cl, tr, comp)
        reco.decompress(comp["stream"], dec)
    reco.sync()
    reco.profile(True)
    with torch.cuda.stream(stream):
        for _ in range(5):
            reco.compress(cl, tr, comp)
            reco.decompress(comp["stream"], dec)
    cprof = reco.profile_read()
    reco.profile(False)
    reco.sync()
    n_words = int(comp["n_words"].item())
    n_hits_c = int(tr["n_hits"].item())
    c_ms = cprof["compress"][0] / max(cprof["compress"][1], 1)
    d_ms = cprof["decompress"][0] / max(cprof["decompress"][1], 1)
    c_bytes = 17 * nc + 29 * n_trk + 4 * n_hits_c + 4 * n_words
    d_bytes = 4 * n_words + 20 * nc
    out_comp = dict(stream_bytes=4 * n_words, bytes_per_cluster=4 * n_words / max(nc, 1),
                    ratio_vs_cluster_arrays=33 * nc / (4 * n_words),
                    ratio_vs_zs_samples=6 * ns / (4 * n_words),
                    compress_ms=c_ms, compress_gb_per_s=c_bytes / c_ms / 1e6,
                    compress_hbm_frac=c_bytes / c_ms / 1e6 / HBM_PEAK_GBS,
                    decompress_ms=d_ms, decompress_gb_per_s=d_bytes / d_ms / 1e6,
                    decompress_hbm_frac=d_bytes / d_ms / 1e6 / HBM_PEAK_GBS,
                    residual_hist_y_within_8_steps=float(
                        comp["res_hist"][56:72].sum().item() / max(n_hits_c, 1)))
    log(f"[bench] compression: {out_comp}")
    del comp, dec

    # segment merging and the T0 / z fit of the slice's tracks (HIP events)
    mg = reco.alloc_merged(max_tl)
    with torch.cuda.stream(stream):
        reco.merge_tracks(cl, tr, mg)
    reco.sync()
    reco.profile(True)
    with torch.cuda.stream(stream):
        for _ in range(3):
            reco.merge_tracks(cl, tr, mg)
    mprof = reco.profile_read()
    reco.profile(False)
    reco.sync()
    mh = tpc.merged_to_host(mg, n_trk)
    roots = mh["label"] == np.arange(n_trk)
    out_merge = dict(ms=mprof["merge"][0] / max(mprof["merge"][1], 1), segments=n_trk,
                     merged_tracks=mh["n_merged"],
                     multi_segment=int((np.bincount(mh["label"], minlength=n_trk) > 1).sum()),
                     with_t0=int((roots & (mh["flags"] == 3)).sum()),
                     near_ties=int(mh["near_tie"].sum()))
    log(f"[bench] merging: {out_merge}")
    del mg

    # raw zero-suppressed pages of the slice decoded on the GPU (HIP events on
    # the library's stream); algorithmic bytes: the pages read, 6 B written per
    # sample, the row offsets written
    if not args.no_pages:
        t = time.perf_counter()
        pages = tpcsynth.zs_pages(ev)
        pg_dev = tpc.pages_to_device(pages, dev)
        n_pages = pages.shape[0]
        del pages
        soa = reco.alloc_zs_soa(ev.n_units, ev.n_time_bins, ns)
        with torch.cuda.stream(stream):
            reco.decode_zs_pages(pg_dev, soa)
        reco.sync()
        reco.profile(True)
        with torch.cuda.stream(stream):
            for _ in range(5):
                reco.decode_zs_pages(pg_dev, soa)
        zprof = reco.profile_read()
        reco.profile(False)
        zc = reco.sync()
        assert int(soa["n_samples"].item()) == ns
        z_ms = zprof["zs_decode"][0] / max(zprof["zs_decode"][1], 1)
        z_bytes = n_pages * 8192 + 6 * ns + 4 * (ev.n_units * 152 + 1)
        out_pages = dict(pages=n_pages, page_bytes=n_pages * 8192, samples=ns, ms=z_ms,
                         bytes=z_bytes, gb_per_s=z_bytes / z_ms / 1e6,
                         hbm_frac=z_bytes / z_ms / 1e6 / HBM_PEAK_GBS)
        log(f"[bench] zs page decode ({time.perf_counter() - t:.1f}s): {out_pages}")
        del pg_dev, soa
    else:
        out_pages = None

    # the batched form: one context over the whole slice, or the slice's units
    # cut into n slices on n streams (pipeline.Pipeline), each captured as one
    # graph; the fastest form is the one timed
    def capture(enqueue):
        g = torch.cuda.CUDAGraph()
        with torch.cuda.stream(stream):
            enqueue()  # first use of every launch outside the capture
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=stream):
            enqueue()
        torch.cuda.synchronize()
        return g

    def time_steps(run, steps):
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        w0 = time.perf_counter()
        with torch.cuda.stream(stream):
            e0.record(stream)
            for _ in range(steps):
                run()
            e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps, (time.perf_counter() - w0) / steps * 1e3

    forms = {}
    one = lambda: reco.process(zs, cl, links, tl, tr, zs_s)
    if args.no_graph:
        forms[1] = (None, one, None)
    else:
        g1 = capture(one)
        forms[1] = (g1, g1.replay, None)
        for n in args.slices:
            if n <= 1:
                continue
            for st in ("cluster", "none"):
                pl = Pipeline(zs, n, tuning=tuning["chosen"] if tuning else None, stagger=st)
                gn = capture(pl.enqueue)
                forms[f"{n}/{st}"] = (gn, gn.replay, pl)
    form_ms = {n: time_steps(f[1], 5)[0] for n, f in forms.items()}
    best = min(form_ms, key=form_ms.get)
    log("[bench] batched forms (slices/start: ms/step): " +
        ", ".join(f"{n}: {v:.3f}" for n, v in form_ms.items()))
    for n, f in forms.items():
        if n != best and f[2] is not None:
            f[2].close()
    graph, run_best, pl_best = forms[best]
    n_slices = pl_best.n_parts if pl_best is not None else 1
    start_pt = pl_best.stagger if pl_best is not None else None

    # timed region: the chosen batched form, one graph replay per step
    ms_step, wall_ms = time_steps(run_best, args.steps)
    c2 = pl_best.sync() if pl_best is not None else reco.sync()
    assert c2["n_clusters"] == nc, "graph replay changed the result"
    assert c2["n_tracks"] == counts["n_tracks"], "graph replay changed the result"
    value = nc / (ms_step / 1e3)
    log(f"[bench] batched ({n_slices} slice(s), start {start_pt}): {ms_step:.3f} ms/step "
        f"({wall_ms:.3f} wall), "
        f"{value:.4g} clusters/s")

    # rooflines: the clusterizer's peak pass (one kernel, the longest single
    # launch; HBM bytes) and the following stage (its two pass launches and
    # their sorts; FP32 operations).  `roofline` is the one whose launch time
    # is the larger, i.e. the dominant kernel.
    n_ur = ev.n_units * 152
    tn = reco.tuning()  # the launch shapes the timed steps ran with
    sb = stage_bytes(ns, nc, n_ur, ev.n_time_bins, tn["cl_window"])
    dom = max(stages, key=lambda k: stages[k])
    # algorithmic bytes of the clusterizer: the samples it reads (u16 pad,
    # time, adc) and a 32-byte cluster record per cluster it produces
    peak_bytes = 6 * ns + 32 * nc
    ach = peak_bytes / (stages["cluster_peaks"] / 1e3) / 1e9
    kbase = {0: "k_cluster_peaks", 1: "k_cluster_stream", 2: "k_cluster_peaks_mw"}[tn["cl_mode"]]
    kname = (f"void k_cluster_stream<{tn['cl_window']}, {tn['cl_chunk']}>" if tn["cl_mode"] == 1 else
             f"void {kbase}<{tn['cl_window']}, {tn['cl_chunk']},")
    roof_peaks = dict(bound="hbm", kernel=kbase,
                      achieved=ach, peak=HBM_PEAK_GBS,
                      unit="GB/s", frac=ach / HBM_PEAK_GBS,
                      traffic=pmc_traffic(KERNEL_SOURCES["cluster_peaks"], "cluster_peaks", kname),
                      bytes_per_launch=peak_bytes, ms_per_launch=stages["cluster_peaks"],
                      bytes_model="6 B per sample + 32 B per cluster",
                      bytes_moved_by_design=sb["cluster_peaks"])
    flops = (FLOPS_STEP * fcounts["follow_steps"] + FLOPS_CAND * fcounts["follow_candidates"] +
             FLOPS_UPDATE * fcounts["follow_updates"])
    ach_f = flops / (stages["following"] / 1e3) / 1e12
    fb, fm = tn["follow_block"], tn["follow_mode"]
    fkern = (f"void k_follow<{fb}, 2, false>" if fm == 1 else
             " + ".join(f"void {'k_follow_q' if fm == 2 else 'k_follow'}<{fb}, {p}, false>"
                        for p in (0, 1)))
    roof_follow = dict(bound="alu", kernel=f"following ({fkern}, with the sorts)",
                       achieved=ach_f, peak=FP32_PEAK_TFLOPS, unit="TFLOP/s",
                       frac=ach_f / FP32_PEAK_TFLOPS,
                       traffic=pmc_traffic(KERNEL_SOURCES["following"], "following", fkern),
                       flops_per_launch=flops, ms_per_launch=stages["following"],
                       steps=fcounts["follow_steps"], candidates=fcounts["follow_candidates"],
                       updates=fcounts["follow_updates"],
                       lane_slots=fcounts["follow_lane_slots"],
                       lane_use=fcounts["follow_steps"] / max(fcounts["follow_lane_slots"], 1))
    if stages["cluster_peaks"] >= stages["following"]:
        roofline, roofline_2 = roof_peaks, roof_follow
    else:
        roofline, roofline_2 = roof_follow, roof_peaks
    roofline["dominant_stage"] = dom
    roofline["dominant_stage_ms"] = stages[dom]

    out = dict(metric=METRIC, value=value, unit="clusters/s", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=ms_step, higher_is_better=True, scaling="weak",
               vs_baseline=None, dtype="f32+int", data="synthetic",
               config=dict(workload="2 ms Pb-Pb slice at 50 kHz: 100 minimum-bias collisions, "
                           "36 sectors x 152 rows, 10500 time bins, seed 303",
                           form=(f"batched: {n_slices} unit slice(s) on {n_slices} stream(s) "
                                 f"(slice start: {start_pt}), one graph replay per step")
                           if graph is not None else "eager",
                           slices=n_slices, slice_start=start_pt, slice_ms=form_ms,
                           samples=ns, clusters=nc, tracks=counts["n_tracks"]),
               roofline=roofline, roofline_2=roofline_2, stages_ms=stages, qc=qc)
    # real-time factor: the slice's collisions per second of one GPU against
    # the 50 kHz interaction rate the slice is drawn at
    coll_per_s = len(cfg.collisions) / (ms_step / 1e3)
    out["realtime"] = dict(collisions=len(cfg.collisions), collisions_per_s=coll_per_s,
                           rate_hz=50e3, factor=coll_per_s / 50e3)
    if out_pages is not None:
        out["zs_pages"] = out_pages
    out["compression"] = out_comp
    out["merging"] = out_merge
    if tuning is not None:
        out["tuning"] = tuning["chosen"]
    # secondary throughput: the single-context graph preceded by the input's
    # copy from pinned host memory on the same stream (PCIe included; not the
    # metric, which takes the input resident in HBM)
    if graph is not None and not args.no_h2d:
        host = {k: zs[k].cpu().pin_memory() for k in ("pad", "time", "adc", "row_start")}
        g_one = forms[1][1]

        def with_h2d():
            for k, v in host.items():
                zs[k].copy_(v, non_blocking=True)
            g_one()

        h2d_ms, _ = time_steps(with_h2d, 3)
        c3 = reco.sync()
        assert c3["n_clusters"] == nc, "input copy changed the result"
        h2d_bytes = sum(v.numel() * v.element_size() for v in host.values())
        out["h2d_inclusive"] = dict(value=nc / (h2d_ms / 1e3), unit="clusters/s",
                                    ms_per_step=h2d_ms, bytes_copied=h2d_bytes,
                                    form="one context, one graph replay, input copied from "
                                         "pinned host memory first")
        log(f"[bench] h2d-inclusive: {out['h2d_inclusive']}")
        del host
    del graph, forms
    if pl_best is not None:
        pl_best.close()

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
        reco2.close()
        log(f"[bench] plain: {out['plain']}")
        out["c1_latency"] = plain_latency(tpc, torch, tpcsynth, stream, dev, args)
        log(f"[bench] c1 latency: {out['c1_latency']}")
        out["plain_collisions"] = plain_collisions(tpc, torch, tpcsynth, stream, dev, cfg)
        log(f"[bench] plain, the slice's collisions one call each: {out['plain_collisions']}")
        out["batched_over_plain"] = value / out["plain_collisions"]["value"]
        out["batched_over_plain_central"] = value / out["plain"]["value"]
    reco.close()
    del cl, links, tl, tr, zs
    torch.cuda.empty_cache()

    if not args.no_serve:
        out["serving"] = serve_leg(args, torch, tpcsynth, tuning["chosen"] if tuning else None)
        log(f"[bench] serving: {out['serving']}")

    stress = None
    if not args.no_stress:
        out["precision_stress"], stress = stress_leg(torch, tpcsynth, tpc, stream)
        log(f"[bench] precision stress: {out['precision_stress']}")

    if not args.no_cpu:
        t = time.perf_counter()
        out["cpu_baseline"] = cpu_baseline(ev, stress)
        log(f"[bench] cpu baseline in {time.perf_counter() - t:.1f}s: {out['cpu_baseline']}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

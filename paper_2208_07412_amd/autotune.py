"""Launch-shape autotuner.

Every launch shape the library offers (clusterizer window, windows per
workgroup and per-window or streamed peak pass; workgroup size and mode of the following; resident waves of the
FP32 refit) gives identical results, so
the choice is made by timing alone: each candidate runs the full launch
sequence on the caller's resident workload, the library's stage timers (HIP
events on its stream) give the time of the stages the shape affects, and the
fastest candidate of each group is kept on the context.
"""
from __future__ import annotations

from typing import Dict, List, Tuple

# (window, windows per workgroup, mode): mode 0 per window, 1 streamed per chunk
CLUSTER_SHAPES: List[Tuple[int, int, int]] = [
    (8, 4, 0), (8, 8, 0), (8, 16, 0), (16, 4, 0), (16, 8, 0), (16, 16, 0), (20, 8, 0), (24, 8, 0),
    (32, 4, 0), (32, 8, 0), (32, 16, 0), (16, 16, 1), (24, 8, 1), (32, 16, 1),
    (24, 8, 2), (32, 4, 2), (32, 8, 2), (32, 16, 2)]
FOLLOW_SHAPES: List[Tuple[int, int]] = [(fb, fm) for fm in (0, 1, 2) for fb in (64, 128, 256)]
CLUSTER_STAGES = ("sample_index", "cluster_peaks", "cluster_scan", "cluster_output")
FOLLOW_STAGES = ("following",)
REFIT_WAVES: List[int] = [0, 4, 5, 6, 8]
REFIT_STAGES = ("refit",)


def _stage_ms(prof: Dict[str, tuple], names, runs: int) -> float:
    return sum(prof[n][0] for n in names) / runs


def _time(reco, run, names, reps: int) -> float:
    run()  # untimed: first use of a shape
    reco.sync()
    reco.profile(True)
    for _ in range(reps):
        run()
    prof = reco.profile_read()
    reco.profile(False)
    reco.sync()
    return _stage_ms(prof, names, reps)


def _pick(times: Dict[str, float], keep: str, margin: float) -> str:
    """Fastest candidate, but the current one stays unless beaten by more
    than `margin` (timings within noise should not flip the choice)."""
    best = min(times, key=times.get)
    if keep in times and times[best] > (1.0 - margin) * times[keep]:
        return keep
    return best


def autotune(reco, run, reps: int = 3, margin: float = 0.02) -> dict:
    """run() enqueues one full reconstruction on reco's stream.  Leaves the
    fastest shapes set on reco and returns them with every timing (ms)."""
    start = reco.tuning()
    res = {"cluster": {}, "follow": {}}
    for w, k, m in CLUSTER_SHAPES:
        reco.set_tuning(cl_window=w, cl_chunk=k, cl_mode=m)
        res["cluster"][f"{w}x{k}x{m}"] = _time(reco, run, CLUSTER_STAGES, reps)
    best_c = _pick(res["cluster"], f"{start['cl_window']}x{start['cl_chunk']}x{start['cl_mode']}",
                   margin)
    w, k, m = (int(x) for x in best_c.split("x"))
    reco.set_tuning(cl_window=w, cl_chunk=k, cl_mode=m)
    for fb, fm in FOLLOW_SHAPES:
        reco.set_tuning(follow_block=fb, follow_mode=fm)
        res["follow"][f"{fb}x{fm}"] = _time(reco, run, FOLLOW_STAGES, reps)
    best_f = _pick(res["follow"], f"{start['follow_block']}x{start['follow_mode']}", margin)
    fb, fm = (int(x) for x in best_f.split("x"))
    reco.set_tuning(follow_block=fb, follow_mode=fm)
    res["refit"] = {}
    for rw in REFIT_WAVES:
        reco.set_tuning(refit_waves=rw)
        res["refit"][str(rw)] = _time(reco, run, REFIT_STAGES, reps)
    best_r = _pick(res["refit"], str(start["refit_waves"]), margin)
    reco.set_tuning(refit_waves=int(best_r))
    res["chosen"] = reco.tuning()
    res["start"] = start
    return res

"""Every launch shape the library offers gives the oracle's results.

Launch shapes (clusterizer window and windows per workgroup, workgroup size
and lane-refill mode of the following kernel) only change how work is spread
over the GPU, so each
one is held to the same parity rules as the default: clusters, links,
tracklets and hit sets bit-exact, parameters within tolerance.  The
dense-lattice frame gives windows with hundreds of peaks, more than one
moment batch.  The shared-window mode (two waves on one window's tile) is
held to the same rules in each of its shapes.
"""
import numpy as np
import pytest

import oracle
import tpcsynth
from paper_2208_07412_amd import tpc

from _parity import compare_clusters, compare_fit, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

NPADS, _, _ = oracle.geometry()
SHAPES = [(8, 8, 64, 0, 0), (8, 16, 128, 1, 4), (16, 4, 64, 2, 5), (16, 8, 128, 1, 6),
          (16, 16, 256, 0, 8), (20, 8, 128, 0, 6), (24, 8, 256, 1, 5), (32, 4, 256, 1, 0),
          (32, 8, 64, 1, 5), (32, 16, 128, 0, 4), (24, 8, 128, 2, 0), (8, 4, 256, 2, 6)]


# (window, windows per workgroup, mode) of the shared-window passes
SHARED = [(24, 8, 2), (32, 4, 2), (32, 8, 2), (32, 16, 2)]


@pytest.fixture(scope="module")
def frame():
    cfg = tpcsynth.EventConfig("pileup", 1000, [tpcsynth.Collision(t, 400, 80) for t in
                                                (0.0, 150.0, 420.0, 500.0)])
    ev = tpcsynth.generate(cfg, 61)
    return ev, run_oracle(ev, labels=True)


@pytest.mark.parametrize("cm", [0, 1])
@pytest.mark.parametrize("w,k,fb,fm,rw", SHAPES)
def test_shape_parity(frame, w, k, fb, fm, rw, cm):
    ev, o = frame
    g = run_gpu(ev, labels=True, tuning=dict(cl_window=w, cl_chunk=k, follow_block=fb,
                                              follow_mode=fm, refit_waves=rw, cl_mode=cm))
    compare_clusters(g["clusters"], o["clusters"], labels=True)
    assert np.array_equal(g["links"]["down"], o["down"])
    assert np.array_equal(g["links"]["up"], o["up"])
    assert np.array_equal(g["tracklets"]["tl_start"], o["tracklets"]["tl_start"])
    compare_fit(g, o)


@pytest.mark.parametrize("w,k,cm", SHARED)
def test_shared_window_parity(frame, w, k, cm):
    ev, o = frame
    g = run_gpu(ev, labels=True, tuning=dict(cl_window=w, cl_chunk=k, cl_mode=cm))
    compare_clusters(g["clusters"], o["clusters"], labels=True)
    assert np.array_equal(g["links"]["down"], o["down"])
    assert np.array_equal(g["tracklets"]["tl_start"], o["tracklets"]["tl_start"])


def _lattice_event(T, step_t, step_p, adc):
    pad, time, a = [], [], []
    rows = (0, 40, 151)
    rs = np.zeros(153, np.uint32)
    for r in rows:
        n = 0
        for t in range(0, T, step_t):
            for p in range(0, int(NPADS[r]), step_p):
                time.append(t)
                pad.append(p)
                a.append(adc(t, p))
                n += 1
        rs[r + 1] = n
    rs = np.cumsum(rs).astype(np.uint32)
    cfg = tpcsynth.config_small(0, n_time_bins=T)
    return tpcsynth.Event(cfg, np.array(pad, np.uint16), np.array(time, np.uint16),
                          np.array(a, np.uint16), rs, 1, T, {}, {}, None)


@pytest.mark.parametrize("w,k,cm", [(w, k, cm) for cm in (0, 1)
                                    for w, k in ((8, 4), (16, 8), (20, 8), (24, 8), (32, 4))] +
                         [(24, 8, 2), (32, 8, 2), (32, 16, 2)])
def test_most_peaks_per_window(w, k, cm):
    # isolated samples on every other pad and bin: each one is a peak, so a
    # window holds far more peaks than one moment batch (and the streaming
    # pass hands its chunks to the per-window pass)
    ev = _lattice_event(100, 2, 2, lambda t, p: 5 + (t * 7 + p * 3) % 900)
    g = run_gpu(ev, labels=True, max_tracklets=64, tuning=dict(cl_window=w, cl_chunk=k, cl_mode=cm))
    o = run_oracle(ev, labels=True)
    assert len(o["clusters"]["y_fx"]) == ev.n_samples
    compare_clusters(g["clusters"], o["clusters"], labels=True)


@pytest.mark.parametrize("w,k,cm", [(w, k, cm) for cm in (0, 1)
                                    for w, k in ((8, 16), (16, 8), (20, 8), (24, 8), (32, 16))] +
                         [(24, 8, 2), (32, 4, 2)])
def test_fully_occupied_rows(w, k, cm):
    # every (time, pad) present: the densest input a row can have
    ev = _lattice_event(120, 1, 1, lambda t, p: 3 + ((t * 131 + p * 71) * 2654435761 % 2**32) % 400)
    g = run_gpu(ev, labels=True, max_tracklets=64, tuning=dict(cl_window=w, cl_chunk=k, cl_mode=cm))
    o = run_oracle(ev, labels=True)
    compare_clusters(g["clusters"], o["clusters"], labels=True)


def test_shared_window_reports_overfull_window():
    # every (time, pad) of the widest row three times over: duplicates pass the
    # sample index when validation is off, and a window then holds more
    # samples than cells, which the shared-window pass reports (and skips)
    T, r = 40, 151
    npads = int(NPADS[r])
    time = np.repeat(np.arange(T), npads * 3).astype(np.uint16)
    pad = np.tile(np.repeat(np.arange(npads), 3), T).astype(np.uint16)
    adc = np.full(len(pad), 7, np.uint16)
    rs = np.zeros(153, np.uint32)
    rs[r + 1:] = len(pad)
    reco = tpc.Reco(1, T, len(pad), 64)
    reco.set_tuning(cl_window=32, cl_chunk=8, cl_mode=2)
    zs = tpc.to_device_zs(pad, time, adc, rs, 1, T)
    reco.cluster(zs, reco.alloc_clusters(1, T, len(pad)))
    assert reco.sync(raise_on_error=False)["status"] == -3
    # the context serves the next (valid) call
    ev = _lattice_event(T, 2, 2, lambda t, p: 5 + (t * 7 + p * 3) % 900)
    g = run_gpu(ev, reco=reco, labels=True, max_tracklets=64)
    compare_clusters(g["clusters"], run_oracle(ev, labels=True)["clusters"], labels=True)
    reco.close()


@pytest.mark.parametrize("fm", [0, 2])
def test_work_counting_variant_same_results(frame, fm):
    # the measurement variant of the following kernel counts its work and
    # must leave every output unchanged
    ev, o = frame
    from paper_2208_07412_amd import tpc

    ns = ev.n_samples
    reco = tpc.Reco(ev.n_units, ev.n_time_bins, ns, ns // 8)
    reco.set_tuning(follow_mode=fm)
    reco.profile(False, count_work=True)
    g1 = run_gpu(ev, reco=reco, max_tracklets=ns // 8)
    c = g1["counts"]
    assert c["follow_steps"] > 0 and c["follow_updates"] > 0 and c["follow_candidates"] > 0
    assert c["follow_updates"] <= c["follow_steps"] + 2 * c["n_tracklets"]
    # a lane slot per lane and wave round: at least one per step
    assert c["follow_lane_slots"] >= c["follow_steps"]
    print(f"follow_mode {fm}: lane use {c['follow_steps'] / c['follow_lane_slots']:.3f}")
    reco.profile(False)
    g2 = run_gpu(ev, reco=reco, max_tracklets=ns // 8)
    assert g2["counts"]["follow_steps"] == 0
    for k in ("tracklet", "par", "cov", "hits", "cluster_track"):
        assert np.array_equal(g1["tracks"][k], g2["tracks"][k])
    reco.close()


def test_set_tuning_rejects_unknown_shapes():
    reco = tpc.Reco(1, 100, 1024, 64)
    before = reco.tuning()
    for bad in (dict(cl_window=12), dict(cl_chunk=3), dict(cl_window=20, cl_chunk=4), dict(cl_window=28),
                dict(follow_block=96), dict(follow_mode=3), dict(refit_waves=3), dict(cl_mode=3),
                dict(cl_window=48), dict(cl_window=16, cl_mode=2), dict(cl_window=20, cl_mode=2)):
        with pytest.raises(tpc.TpcError):
            reco.set_tuning(**bad)
        assert reco.tuning() == before
    reco.set_tuning(refit_waves=0)
    assert reco.tuning()["refit_waves"] == 0
    reco.close()

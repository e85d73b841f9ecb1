"""GPU edge cases and stage-isolated parity.

* empty input, a lone sample, samples on the edges of the pad/time ranges;
* a long sparse frame near the largest time range of the configurations;
* capacity overflow and malformed input are reported, not written past;
* each stage fed with the oracle's output of the previous stage;
* the FP64 refit path (forced) against the FP64 oracle.
"""
import numpy as np
import pytest

import oracle
import tpcsynth
from paper_2208_07412_amd import tpc

from _parity import FLOORS, compare_clusters, compare_fit, ill_conditioned, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

NPADS, _, _ = oracle.geometry()


def _event(samples, n_units=1, T=64):
    """samples: list of (unit, row, time, pad, adc)."""
    samples = sorted(samples)
    pad = np.array([s[3] for s in samples], np.uint16)
    time = np.array([s[2] for s in samples], np.uint16)
    adc = np.array([s[4] for s in samples], np.uint16)
    rs = np.zeros(n_units * 152 + 1, np.uint32)
    for u, r, *_ in samples:
        rs[u * 152 + r + 1] += 1
    rs = np.cumsum(rs).astype(np.uint32)
    cfg = tpcsynth.config_small(0, n_time_bins=T)
    return tpcsynth.Event(cfg, pad, time, adc, rs, n_units, T, {}, {}, None)


def test_empty_input():
    ev = _event([])
    g = run_gpu(ev, max_tracklets=16)
    assert g["counts"]["n_clusters"] == 0 and g["counts"]["n_tracks"] == 0
    assert np.all(g["clusters"]["crow_start"] == 0)


def test_lone_and_edge_samples():
    T = 100
    s = [(0, 0, 0, 0, 40), (0, 0, T - 1, int(NPADS[0]) - 1, 41), (0, 151, 50, 137, 1023),
         (0, 151, 50, 136, 1023), (0, 70, 48, 20, 7), (0, 70, 47, 20, 4), (0, 70, 49, 21, 4),
         (0, 80, 95, 3, 2)]
    ev = _event(s, T=T)
    g = run_gpu(ev, labels=True, max_tracklets=16)
    o = run_oracle(ev, labels=True)
    compare_clusters(g["clusters"], o["clusters"], labels=True)
    assert g["counts"]["n_clusters"] == 4


def test_window_boundaries_dense_row():
    # a dense random row spanning many clusterizer windows and their halos
    rng = np.random.default_rng(5)
    T = 700
    s = []
    for t in range(T):
        for p in range(int(NPADS[40])):
            if rng.random() < 0.3:
                s.append((0, 40, t, p, int(rng.integers(3, 60))))
    ev = _event(s, T=T)
    g = run_gpu(ev, labels=True, max_tracklets=64)
    o = run_oracle(ev, labels=True)
    compare_clusters(g["clusters"], o["clusters"], labels=True)


def test_long_sparse_frame():
    # 200-collision time range (20,500 bins) with only a few tracks
    cfg = tpcsynth.EventConfig("long", 20500, [tpcsynth.Collision(t, 30, 5) for t in
                                               (0.0, 9000.0, 19990.0)])
    ev = tpcsynth.generate(cfg, 31)
    g = run_gpu(ev)
    o = run_oracle(ev)
    compare_clusters(g["clusters"], o["clusters"])
    assert np.array_equal(g["tracklets"]["tl_start"], o["tracklets"]["tl_start"])
    compare_fit(g, o)


def test_cluster_capacity_overflow_reported():
    ev = tpcsynth.generate(tpcsynth.config_small(20), 4)
    n_true = len(run_oracle(ev)["clusters"]["y_fx"])
    reco = tpc.Reco(1, ev.n_time_bins, ev.n_samples, 1024)
    zs = tpc.to_device_zs(ev.pad, ev.time, ev.adc, ev.row_start, 1, ev.n_time_bins)
    cl = reco.alloc_clusters(1, ev.n_time_bins, n_true - 1)
    reco.cluster(zs, cl)
    counts = reco.sync(raise_on_error=False)
    assert counts["status"] == -2 and counts["required"] == n_true
    assert counts["required_by"] == {"clusters": n_true}
    # the next call on the same context works again
    cl2 = reco.alloc_clusters(1, ev.n_time_bins, n_true)
    reco.cluster(zs, cl2)
    assert reco.sync()["n_clusters"] == n_true
    reco.close()


def test_tracklet_capacity_overflow_reported():
    ev = tpcsynth.generate(tpcsynth.config_small(40), 6)
    o = run_oracle(ev)
    nt = len(o["tracklets"]["tl_start"])
    reco = tpc.Reco(1, ev.n_time_bins, ev.n_samples, 1024)
    with pytest.raises(tpc.TpcError) as e:
        run_gpu(ev, reco=reco, max_tracklets=nt - 1)
    assert e.value.code == -2
    reco.close()


def test_tracklet_overflow_after_a_larger_frame():
    # the context first reconstructs a larger frame, so its scratch holds
    # larger totals; the overflow must report the true tracklet count
    big = tpcsynth.generate(tpcsynth.config_small(160), 61)
    ev = tpcsynth.generate(tpcsynth.config_small(40), 6)
    nt = len(run_oracle(ev)["tracklets"]["tl_start"])
    n_big = len(run_oracle(big)["tracklets"]["tl_start"])
    assert n_big > nt + 10
    reco = tpc.Reco(1, max(big.n_time_bins, ev.n_time_bins), big.n_samples, 4 * n_big)
    g = run_gpu(big, reco=reco, max_tracklets=2 * n_big)
    assert g["counts"]["n_tracklets"] == n_big
    zs = tpc.to_device_zs(ev.pad, ev.time, ev.adc, ev.row_start, 1, ev.n_time_bins)
    cl = reco.alloc_clusters(1, ev.n_time_bins, ev.n_samples)
    links = reco.alloc_links(ev.n_samples)
    tl = reco.alloc_tracklets(nt - 1)
    tr = reco.alloc_tracks(nt - 1, ev.n_samples, ev.n_samples)
    reco.process(zs, cl, links, tl, tr)
    counts = reco.sync(raise_on_error=False)
    assert counts["status"] == -2
    assert counts["required_by"] == {"tracklets": nt}, counts["required_by"]
    assert counts["required"] == nt
    reco.close()


@pytest.mark.parametrize("bad_adc", [0, 1024])
def test_adc_outside_ten_bits_reported(bad_adc):
    ev = _event([(0, 10, 5, 3, 50), (0, 10, 5, 4, 60), (0, 11, 6, 3, 40)])
    adc = ev.adc.copy()
    reco = tpc.Reco(1, ev.n_time_bins, 16, 16, param_overrides=dict(validate=1))
    cl = reco.alloc_clusters(1, ev.n_time_bins, 16)
    reco.cluster(tpc.to_device_zs(ev.pad, ev.time, adc, ev.row_start, 1, ev.n_time_bins), cl)
    assert reco.sync(raise_on_error=False)["status"] == 0
    adc[1] = bad_adc
    reco.cluster(tpc.to_device_zs(ev.pad, ev.time, adc, ev.row_start, 1, ev.n_time_bins), cl)
    assert reco.sync(raise_on_error=False)["status"] == -3
    reco.close()


def test_malformed_input_reported():
    ev = _event([(0, 10, 5, 3, 50), (0, 10, 5, 4, 60)])
    bad_pad = ev.pad.copy()
    bad_pad[1] = 140  # beyond the row's pads: always rejected
    reco = tpc.Reco(1, ev.n_time_bins, 16, 16)
    zs = tpc.to_device_zs(bad_pad, ev.time, ev.adc, ev.row_start, 1, ev.n_time_bins)
    cl = reco.alloc_clusters(1, ev.n_time_bins, 16)
    reco.cluster(zs, cl)
    assert reco.sync(raise_on_error=False)["status"] == -3
    reco.close()
    # unsorted samples are rejected in validate mode
    reco = tpc.Reco(1, ev.n_time_bins, 16, 16, param_overrides=dict(validate=1))
    unsorted = ev.pad[::-1].copy()
    zs = tpc.to_device_zs(unsorted, ev.time, ev.adc, ev.row_start, 1, ev.n_time_bins)
    reco.cluster(zs, cl := reco.alloc_clusters(1, ev.n_time_bins, 16))
    assert reco.sync(raise_on_error=False)["status"] == -3
    reco.close()


def test_stages_on_oracle_inputs():
    ev = tpcsynth.generate(tpcsynth.config_small(120, sector_mode=0), 12)
    o = run_oracle(ev)
    ns = ev.n_samples
    reco = tpc.Reco(ev.n_units, ev.n_time_bins, ns, 8192)
    cl = reco.clusters_from_host(o["clusters"], ev.n_units, ev.n_time_bins)
    n = len(o["clusters"]["y_fx"])
    links = reco.alloc_links(cl.s.capacity)
    reco.find_neighbours(cl, links)
    reco.sync()
    gl = tpc.links_to_host(links, n)
    assert np.array_equal(gl["down"], o["down"]) and np.array_equal(gl["up"], o["up"])
    tl = reco.alloc_tracklets(8192)
    reco.build_tracklets(cl, links, tl)
    reco.sync()
    gt = tpc.tracklets_to_host(tl)
    assert np.array_equal(gt["tl_start"], o["tracklets"]["tl_start"])
    assert np.array_equal(tpc.links_to_host(links, n)["upc"], o["tracklets"]["upc"])
    tr = reco.alloc_tracks(8192, ns, cl.s.capacity, follow_capacity=8192)
    reco.fit_tracks(cl, links, tl, tr)
    counts = reco.sync()
    g = dict(tracks=tpc.tracks_to_host(tr, n, counts["n_tracklets"] or len(gt["tl_start"])))
    compare_fit(g, o)
    reco.close()


def test_forced_fp64_refit_matches_oracle():
    ev = tpcsynth.generate(tpcsynth.config_c1(), 101)
    p = oracle.default_params()
    g = run_gpu(ev, params=dict(force_fallback=1))
    o = run_oracle(ev)
    n = len(g["tracks"]["tracklet"])
    assert g["counts"]["n_fallback"] == n and n > 50
    assert np.all(g["tracks"]["flags"] & 4)
    compare_fit(g, o)
    # the same FP64 refit as the oracle's (UD factors instead of the dense
    # update: equal up to FP64 rounding), stored in FP32
    sel = [j for j, t in enumerate(g["tracks"]["tracklet"]) if not ill_conditioned(o["fit"], t)]
    par_o = o["fit"]["par"][g["tracks"]["tracklet"][sel]]
    rel = np.abs(g["tracks"]["par"][sel] - par_o) / np.maximum(np.abs(par_o), FLOORS)
    assert rel.max() <= 1e-6, rel.max()

"""GPU parity: every stage of the HIP path against the CPU oracle.

Inputs are seeded synthetic events.  Sizes span many LDS tiles and ragged
tails (one sector with a few tracks; a full central collision; a noisy
high-occupancy frame; a multi-collision frame with pile-up).
"""
import numpy as np
import pytest

import oracle
import tpcsynth

from _parity import (compare_clusters, compare_fit, cov_pd, run_gpu, run_oracle)

pytestmark = pytest.mark.gpu


def _small_dense_event(seed, n_tracks=60, T=300, noise=2.0):
    cfg = tpcsynth.config_small(n_tracks, n_time_bins=T, sigma_noise=noise)
    return tpcsynth.generate(cfg, seed)


@pytest.mark.parametrize("seed", [1, 2])
def test_cluster_parity_small(seed):
    ev = _small_dense_event(seed)
    g = run_gpu(ev, labels=True, params=oracle.default_params(2.0))
    o = run_oracle(ev, labels=True, params=oracle.default_params(2.0))
    compare_clusters(g["clusters"], o["clusters"], labels=True)


def test_cluster_parity_c1():
    ev = tpcsynth.generate(tpcsynth.config_c1(), 101)
    g = run_gpu(ev, labels=True)
    o = run_oracle(ev, labels=True)
    compare_clusters(g["clusters"], o["clusters"], labels=True)


@pytest.fixture(scope="module")
def c2():
    ev = tpcsynth.generate(tpcsynth.config_c2(), 202)
    return ev, run_gpu(ev, labels=True), run_oracle(ev, labels=True)


def test_c2_clusters(c2):
    ev, g, o = c2
    compare_clusters(g["clusters"], o["clusters"], labels=True)
    # charge conservation on the GPU output
    lab = g["clusters"]["sample_label"][: ev.n_samples]
    assert int(ev.adc[lab >= 0].astype(np.int64).sum()) == int(
        g["clusters"]["qtot"].astype(np.int64).sum())


def test_c2_links_and_tracklets(c2):
    ev, g, o = c2
    assert np.array_equal(g["links"]["down"], o["down"])
    assert np.array_equal(g["links"]["up"], o["up"])
    assert np.array_equal(g["links"]["downc"], o["tracklets"]["downc"])
    assert np.array_equal(g["links"]["upc"], o["tracklets"]["upc"])
    assert np.array_equal(g["tracklets"]["tl_start"], o["tracklets"]["tl_start"])
    assert np.array_equal(g["tracklets"]["tl_len"], o["tracklets"]["tl_len"])


def test_c2_fit(c2):
    ev, g, o = c2
    n_ex = compare_fit(g, o)
    nt = len(o["tracklets"]["tl_start"])
    assert n_ex <= 0.01 * nt, (n_ex, nt)
    tr = g["tracks"]
    ok = tr["flags"] & 1 == 0
    assert np.all(cov_pd(tr["cov"][ok]))
    # each cluster used by at most one track
    assert len(np.unique(tr["hits"])) == len(tr["hits"])
    print(f"C2: {len(tr['tracklet'])} tracks, {n_ex} exempt of {nt} tracklets, "
          f"fallback {g['counts']['n_fallback']}")


def test_c1_end_to_end():
    ev = tpcsynth.generate(tpcsynth.config_c1(), 101)
    g = run_gpu(ev)
    o = run_oracle(ev)
    compare_clusters(g["clusters"], o["clusters"])
    assert np.array_equal(g["tracklets"]["tl_start"], o["tracklets"]["tl_start"])
    compare_fit(g, o)


def test_pileup_frame_end_to_end():
    # five minimum-bias collisions overlapping in a 1000-bin frame
    cfg = tpcsynth.EventConfig("pileup", 1000, [tpcsynth.Collision(t, n, n // 5) for t, n in
                                                ((0, 400), (120, 700), (300, 250), (420, 900),
                                                 (480, 300))])
    ev = tpcsynth.generate(cfg, 77)
    g = run_gpu(ev)
    o = run_oracle(ev)
    compare_clusters(g["clusters"], o["clusters"])
    assert np.array_equal(g["links"]["up"], o["up"])
    assert np.array_equal(g["tracklets"]["tl_start"], o["tracklets"]["tl_start"])
    n_ex = compare_fit(g, o)
    assert n_ex <= 0.01 * max(1, len(o["tracklets"]["tl_start"]))


def test_determinism():
    ev = tpcsynth.generate(tpcsynth.config_small(80, n_time_bins=400, sector_mode=0), 9)
    a = run_gpu(ev)
    b = run_gpu(ev)
    for k in ("y_fx", "z_fx", "qtot"):
        assert np.array_equal(a["clusters"][k], b["clusters"][k])
    for k in ("tracklet", "hits", "cluster_track"):
        assert np.array_equal(a["tracks"][k], b["tracks"][k])
    assert np.array_equal(a["tracks"]["par"], b["tracks"]["par"])

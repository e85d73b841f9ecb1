"""Parity on a full-size precision-stress chunk: 100 minimum-bias collisions
(10,500 bins, 36 sectors x 152 rows) with 30% low-pT loopers at 0.05-0.2
GeV/c, noise sigma 2 ADC (peak threshold 10) and 10% dead pads, seed 505,
reconstructed in one launch sequence over all units (the configuration the
benchmark's precision leg times).  The oracle is run on sampled units one by
one; properties that hold at any size are checked over the whole chunk, and
the FP64 refit count and per-parameter errors are printed."""
import numpy as np
import pytest

import oracle
import tpcsynth
from paper_2208_07412_amd import tpc

from _parity import PAR_NAMES, compare_clusters, compare_fit, run_oracle
from _units import unit_event, unit_view

pytestmark = pytest.mark.gpu

PAR = oracle.default_params(2.0)
UNITS = (3, 30)
N_COLL = 100


@pytest.fixture(scope="module")
def chunk_run():
    ev = tpcsynth.generate(tpcsynth.config_chunk(505, 0, stress=True, n_coll=N_COLL), 505)
    print(f"stress chunk: {N_COLL} collisions, {ev.n_samples} samples, {ev.n_time_bins} bins",
          flush=True)
    mc = max(ev.n_samples // 6, 1 << 16)
    mt = max(mc // 8, 1 << 14)
    reco = tpc.Reco(ev.n_units, ev.n_time_bins, mc, mt, noise_sigma=2.0,
                    max_samples=ev.n_samples)
    zs = tpc.to_device_zs(ev.pad, ev.time, ev.adc, ev.row_start, ev.n_units, ev.n_time_bins)
    cl = reco.alloc_clusters(ev.n_units, ev.n_time_bins, mc)
    links = reco.alloc_links(mc)
    tl = reco.alloc_tracklets(mt)
    tr = reco.alloc_tracks(mt, mc, mc)
    reco.process(zs, cl, links, tl, tr)
    counts = reco.sync()
    n = counts["n_clusters"]
    out = dict(u0=0, u1=ev.n_units, clusters=tpc.clusters_to_host(cl, ev.n_units),
               links=tpc.links_to_host(links, n), tracklets=tpc.tracklets_to_host(tl),
               tracks=tpc.tracks_to_host(tr, n))
    reco.close()
    return ev, counts, out


@pytest.mark.parametrize("u", UNITS)
def test_sampled_unit_equals_oracle(chunk_run, u):
    ev, counts, out = chunk_run
    g = unit_view(out, u)
    o = run_oracle(unit_event(ev, u), params=PAR)
    compare_clusters(g["clusters"], o["clusters"])
    assert np.array_equal(g["links"]["down"], o["down"])
    assert np.array_equal(g["links"]["up"], o["up"])
    assert np.array_equal(g["links"]["upc"], o["tracklets"]["upc"])
    assert np.array_equal(g["tracklets"]["tl_start"], o["tracklets"]["tl_start"])
    assert np.array_equal(g["tracklets"]["tl_len"], o["tracklets"]["tl_len"])
    compare_fit(g, o)


def test_whole_chunk_properties(chunk_run):
    ev, counts, out = chunk_run
    c, tr = out["clusters"], out["tracks"]
    nc = len(c["y_fx"])
    crow = c["crow_start"].astype(np.int64)
    assert crow[0] == 0 and crow[-1] == nc and np.all(np.diff(crow) >= 0)
    hs = tr["hit_start"].astype(np.int64)
    nk = np.diff(hs)
    assert np.all(nk >= 15)
    h = tr["hits"].astype(np.int64)
    owner = np.repeat(np.arange(len(nk)), nk)
    ct = tr["cluster_track"].astype(np.int64)
    assert np.all(ct[h] == owner)
    assert np.count_nonzero(ct >= 0) == len(h)
    assert np.all(np.isfinite(tr["par"])) and np.all(np.isfinite(tr["cov"]))
    # every output covariance positive definite
    iu = np.triu_indices(5)
    M = np.zeros((len(nk), 5, 5))
    M[:, iu[0], iu[1]] = tr["cov"]
    M = M + np.transpose(M, (0, 2, 1)) - M * np.eye(5)
    assert np.all(np.linalg.eigvalsh(M.astype(np.float64))[:, 0] > 0)
    n_tr = len(nk)
    print(f"stress chunk: {nc} clusters, {n_tr} tracks; FP64 refits {counts['n_fallback']} "
          f"({100 * counts['n_fallback'] / max(n_tr, 1):.3f}%: low-pT tracks whose FP32 pivots "
          f"failed), FP32 tracks flagged not PD {counts['n_not_pd']}, FP64 still not PD "
          f"{counts['n_fallback_fail']}, refits failed {counts['n_refit_fail']}")
    assert counts["n_fallback_fail"] == 0
    assert nc > 1.5e7 and n_tr > 2e5
    assert len(PAR_NAMES) == 5

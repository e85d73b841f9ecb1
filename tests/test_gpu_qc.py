"""GPU quality-control histograms against the oracle's definition.

The QC step's inputs are the reconstruction's outputs: the kernel's counts
are compared bin by bin (exactly: integer binning) with the oracle's
histograms of the same outputs copied to the host, and the cluster
histograms also with those of the oracle's own chain (clusters are
bit-exact).  Edge cases: an empty frame, a second call reusing the
per-workgroup buffers, a frame with more clusters than one grid pass.
"""
import numpy as np
import pytest

import oracle
import tpcsynth
from paper_2208_07412_amd import tpc

from _parity import run_oracle

pytestmark = pytest.mark.gpu


def _run(ev, calls=1):
    ns = max(ev.n_samples, 1)
    mt = max(ns // 8, 1024)
    reco = tpc.Reco(ev.n_units, ev.n_time_bins, ns, mt)
    try:
        zs = tpc.to_device_zs(ev.pad, ev.time, ev.adc, ev.row_start, ev.n_units, ev.n_time_bins)
        cl = reco.alloc_clusters(ev.n_units, ev.n_time_bins, ns, n_samples=ns)
        links = reco.alloc_links(ns)
        tl = reco.alloc_tracklets(mt)
        tr = reco.alloc_tracks(mt, ns, ns)
        reco.process(zs, cl, links, tl, tr)
        hs = [reco.qc_histograms(cl, tr).clone() for _ in range(calls)]
        counts = reco.sync()
        n = counts["n_clusters"]
        c = tpc.clusters_to_host(cl, ev.n_units)
        t = tpc.tracks_to_host(tr, n, 0)
        hh = [h.cpu().numpy().view(np.uint32).astype(np.int64) for h in hs]
        return hh, c, t, counts
    finally:
        reco.close()


def _oracle_of(c, t):
    return oracle.qc_histograms(c["qtot"], c["qmax"], t["cluster_track"], t["hit_start"])


def test_qc_matches_oracle():
    ev = tpcsynth.generate(tpcsynth.config_c1(), 101)
    (h,), c, t, counts = _run(ev)
    exp = _oracle_of(c, t)
    assert np.array_equal(h, exp)
    assert h[oracle.QC_QTOT:oracle.QC_QTOT + 256].sum() == counts["n_clusters"]
    assert h[oracle.QC_NHITS:oracle.QC_NHITS + 153].sum() == counts["n_tracks"]
    o = run_oracle(ev)
    oc = oracle.qc_histograms(o["clusters"]["qtot"], o["clusters"]["qmax"], [], [0])
    assert np.array_equal(h[:oracle.QC_NHITS], oc[:oracle.QC_NHITS])


def test_qc_empty_frame():
    cfg = tpcsynth.config_small(0, n_time_bins=64)
    rs = np.zeros(152 + 1, np.uint32)
    ev = tpcsynth.Event(cfg, np.zeros(0, np.uint16), np.zeros(0, np.uint16),
                        np.zeros(0, np.uint16), rs, 1, 64, {}, {}, None)
    (h,), _, _, _ = _run(ev)
    assert not h.any()


def test_qc_repeated_calls_and_large_frame():
    # more clusters than one pass of the fill grid (1024 x 256 threads)
    ev = tpcsynth.generate(tpcsynth.config_c2(), 202)
    hh, c, t, counts = _run(ev, calls=2)
    assert counts["n_clusters"] > 1024 * 256
    exp = _oracle_of(c, t)
    for h in hh:
        assert np.array_equal(h, exp)

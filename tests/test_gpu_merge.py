"""GPU segment merging and T0 / z fit against the oracle's.

Stage-isolated parity: both take the same clusters and the same tracks (the
oracle's, parameters rounded to float32), so the merged tracks (labels: index
work, bit-exact) must agree except where a joining decision was a near tie
(both flag them; such merged tracks and their members are exempt and
counted), and the fits, FP64 on both sides in the same order, agree to 1e-9
relative (library square roots and arc tangents may differ in the last
bit).  Cases: exact-helix frames (tests/_helix_frames.py), one central
collision, a pile-up frame, and three adjacent sectors of the 2 ms slice.
The full chain: the GPU's reconstruction of the slice merged on the GPU,
with properties that hold at any size, and on one central collision
against generator truth (purity, joined splits, T0 of primaries).
"""
import numpy as np
import pytest

import oracle
import tpcsynth
from paper_2208_07412_amd import tpc
from tpcsynth import truth

from _helix_frames import build_frame, helix_segments

pytestmark = pytest.mark.gpu

FIELDS = ("n_segments", "n_hits", "xc", "yc", "radius", "dzdpsi", "zd_axis", "t0", "tgl",
          "flags", "turn")


def _gpu_merge(clusters, tracks, n_units, n_time_bins):
    nc = len(clusters["y_fx"])
    nt = len(tracks["hit_start"]) - 1
    reco = tpc.Reco(n_units, n_time_bins, max(nc, 1), max(nt, 1))
    try:
        cl = reco.clusters_from_host(clusters, n_units, n_time_bins)
        tr = reco.tracks_from_host(tracks, max(nc, 1))
        out = reco.alloc_merged(tr.s.capacity)
        reco.merge_tracks(cl, tr, out)
        reco.sync()
        return tpc.merged_to_host(out, nt)
    finally:
        reco.close()


def _compare(g, o):
    lab_g, lab_o = g["label"].astype(np.int64), o["label"]
    tie = g["near_tie"] | o["near_tie"]
    ex = np.zeros(len(lab_o), bool)
    for lab in (lab_g, lab_o):
        bad = np.unique(lab[tie])
        ex |= np.isin(lab, bad)
    # exempt whole merged tracks touching a near tie, under either labelling
    ex = np.isin(lab_o, np.unique(lab_o[ex])) | np.isin(lab_g, np.unique(lab_g[ex]))
    assert np.array_equal(lab_g[~ex], lab_o[~ex])
    roots = np.nonzero((lab_o == np.arange(len(lab_o))) & ~ex)[0]
    assert g["n_merged"] == len(np.unique(lab_g))
    worst = 0.0
    for k in FIELDS:
        a, b = g[k][roots], o[k][roots]
        if k in ("n_segments", "n_hits", "flags"):
            assert np.array_equal(a, b), k
        else:
            d = np.abs(a - b) / np.maximum(np.abs(b), 1.0)
            worst = max(worst, float(d.max(initial=0)))
            assert np.all(d <= 1e-9), (k, float(d.max()))
    print(f"merge parity: {len(lab_o)} segments, {len(np.unique(lab_o))} merged tracks, "
          f"{ex.sum()} exempt (near ties), worst fit deviation {worst:.1e}")


def test_exact_helix_frames():
    hel = []
    for phi0, qpt, tgl, t0 in ((0.45, 1.0, 0.4, 37.0), (1.0, -1 / 0.15, 0.1, 120.0),
                               (2.0, 0.5, -0.3, 15.0), (4.0, -3.0, 0.7, 60.0)):
        segs, C = helix_segments(phi0=phi0, qpt=qpt, tgl=tgl, t0=t0)
        hel.append((segs, C, tgl))
    cl, tr, hid = build_frame(hel, 36)
    o = oracle.merge_tracks(cl, tr, 36)
    g = _gpu_merge(cl, tr, 36, 1000)
    _compare(g, o)
    for h in range(len(hel)):
        assert len(set(g["label"][hid == h])) == 1


@pytest.mark.parametrize("which", ["c2", "pileup", "slice3"])
def test_stage_parity_on_oracle_tracks(which):
    if which == "slice3":
        full = tpcsynth.generate(tpcsynth.config_c3(303, 100), 303)
        ev = tpcsynth.select_units(full, [0, 1, 2])
        del full
    else:
        cfg, seed = {"c2": (tpcsynth.config_c2(), 202),
                     "pileup": (tpcsynth.config_chunk(404, 1, n_coll=6), 4041)}[which]
        ev = tpcsynth.generate(cfg, seed)
    o = oracle.process(ev.pad, ev.time, ev.adc, ev.row_start, ev.n_units, ev.n_time_bins,
                       n_threads=8)
    tracks = oracle.tracks_from_fit(o)
    om = oracle.merge_tracks(o["clusters"], tracks, ev.n_units)
    g = _gpu_merge(o["clusters"], tracks, ev.n_units, ev.n_time_bins)
    _compare(g, om)


def test_full_chain_slice_and_truth():
    # one central collision against truth, the GPU's own tracks
    ev = tpcsynth.generate(tpcsynth.config_c2(), 202)
    ns = ev.n_samples
    reco = tpc.Reco(ev.n_units, ev.n_time_bins, ns, ns // 8)
    try:
        zs = tpc.to_device_zs(ev.pad, ev.time, ev.adc, ev.row_start, ev.n_units, ev.n_time_bins)
        cl = reco.alloc_clusters(ev.n_units, ev.n_time_bins, ns)
        links = reco.alloc_links(ns)
        tl = reco.alloc_tracklets(ns // 8)
        tr = reco.alloc_tracks(ns // 8, ns, ns)
        reco.process(zs, cl, links, tl, tr)
        mg = reco.alloc_merged(ns // 8)
        reco.merge_tracks(cl, tr, mg)
        c = reco.sync()
        n = c["n_tracks"]
        m = tpc.merged_to_host(mg, n)
        hc = tpc.clusters_to_host(cl, ev.n_units)
        ht = tpc.tracks_to_host(tr, c["n_clusters"])
    finally:
        reco.close()
    lab = m["label"].astype(np.int64)
    assert np.all(lab <= np.arange(n)) and np.array_equal(lab[lab], lab)
    labels = truth.cluster_labels(ev.deposits, hc, ev.n_units)
    hs = ht["hit_start"].astype(np.int64)
    seg_trk = np.full(n, -1)
    for j in range(n):
        l = labels[ht["hits"][hs[j]:hs[j + 1]]]
        l = l[l >= 0]
        if len(l):
            v, cnt = np.unique(ev.deposits["track"][l], return_counts=True)
            seg_trk[j] = v[np.argmax(cnt)]
    multi = [r for r in np.unique(lab) if (lab == r).sum() > 1]
    pure = sum(1 for r in multi if len(set(seg_trk[lab == r])) == 1)
    prim = np.zeros(n, bool)
    prim[seg_trk >= 0] = ev.tracks["primary"][seg_trk[seg_trk >= 0]]
    pure_c = np.array([len(set(seg_trk[lab == lab[j]])) == 1 for j in range(n)])
    sel = (lab == np.arange(n)) & (m["flags"] == 3) & prim & pure_c
    t0 = m["t0"][sel]
    print(f"GPU chain: {n} segments -> {m['n_merged']} tracks, {len(multi)} merged "
          f"({pure} pure); T0 of {sel.sum()} primaries within 2 bins: {np.mean(np.abs(t0) < 2):.3f}")
    assert pure >= 0.98 * len(multi)
    assert np.mean(np.abs(t0) < 2) > 0.85

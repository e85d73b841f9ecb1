"""Pins of the oracle's segment merging and T0 / z fit.

The paper (section "Hardware and data flow") asks for full online TPC track
reconstruction with continuous readout; no merging rule or T0 method is
given, so the reading is the one stated with oracle_merge_tracks.  Pins:
* exact helices from the origin split into the per-sector, per-leg segments a
  tracker produces (tests/_helix_frames.py, written from the detector and
  drift definitions): a track crossing sector boundaries and a looper whose
  legs meet at its turning radius each become one merged track, and the fit
  returns the helix's radius, dip and the frame's T0;
* particles that must stay apart (other frame, other side, other curvature
  through the same point) do;
* on a generated central collision with the oracle's own tracks against
  generator truth: merged tracks are pure, most split particles are joined,
  and T0 of primaries is found to a fraction of a time bin.
"""
import numpy as np
import pytest

import oracle
import tpcsynth
from tpcsynth import truth

from _helix_frames import build_frame, helix_segments


def _merge(helices, n_units):
    cl, tr, hid = build_frame(helices, n_units)
    return oracle.merge_tracks(cl, tr, n_units), hid, tr


def test_boundary_crossing_track_is_one_track():
    segs, C = helix_segments(phi0=0.45, qpt=1.0, tgl=0.4, t0=37.0)
    units = sorted({u for u, _, _ in segs})
    assert len(units) >= 2  # crosses at least one sector boundary
    m, hid, tr = _merge([(segs, C, 0.4)], 36)
    assert len(set(m["label"])) == 1 and not m["near_tie"].any()
    r = m["label"][0]
    assert m["flags"][r] == 3
    assert abs(m["radius"][r] * abs(C) - 1) < 2e-3
    assert abs(m["t0"][r] - 37.0) < 0.05
    assert abs(m["tgl"][r] - 0.4) < 1e-3


def test_looper_legs_join_at_the_turning_radius():
    # pT 0.15 GeV/c: radius 66.7 cm, turning radius 133 cm inside the chamber
    segs, C = helix_segments(phi0=1.0, qpt=-0.15 ** -1, tgl=0.1, t0=120.0)
    legs = {leg for _, leg, _ in segs}
    assert legs == {1, -1}
    m, hid, tr = _merge([(segs, C, 0.1)], 36)
    assert len(set(m["label"])) == 1
    r = m["label"][0]
    assert abs(m["radius"][r] * abs(C) - 1) < 2e-3
    assert abs(m["t0"][r] - 120.0) < 0.05
    assert m["turn"][r] > np.pi  # both legs


def test_separate_particles_stay_apart():
    # same start, other curvature: ends may come close, curvature differs
    a, Ca = helix_segments(phi0=0.30, qpt=1.0, tgl=0.4, t0=0.0)
    b, Cb = helix_segments(phi0=0.30, qpt=0.5, tgl=0.4, t0=0.0)
    # the same helix in the next frame, and on the other side
    c, Cc = helix_segments(phi0=0.30, qpt=1.0, tgl=0.4, t0=0.0, frame=1)
    d, Cd = helix_segments(phi0=0.30, qpt=1.0, tgl=-0.4, t0=0.0)
    m, hid, tr = _merge([(a, Ca, 0.4), (b, Cb, 0.4), (c, Cc, 0.4), (d, Cd, -0.4)], 72)
    lab = m["label"]
    for h in range(4):
        assert len(set(lab[hid == h])) == 1, h  # each particle whole
    assert len({lab[hid == h][0] for h in range(4)}) == 4  # and apart


def test_generated_collision_against_truth():
    ev = tpcsynth.generate(tpcsynth.config_c2(), 202)
    o = oracle.process(ev.pad, ev.time, ev.adc, ev.row_start, ev.n_units, ev.n_time_bins,
                       n_threads=8)
    tr = oracle.tracks_from_fit(o)
    m = oracle.merge_tracks(o["clusters"], tr, ev.n_units)
    lab = m["label"]
    n = len(lab)
    labels = truth.cluster_labels(ev.deposits, o["clusters"], ev.n_units)
    hs = tr["hit_start"].astype(np.int64)
    seg_trk = np.full(n, -1)
    for j in range(n):
        l = labels[tr["hits"][hs[j]:hs[j + 1]]]
        l = l[l >= 0]
        if len(l):
            v, c = np.unique(ev.deposits["track"][l], return_counts=True)
            seg_trk[j] = v[np.argmax(c)]
    roots = np.unique(lab)
    multi = [r for r in roots if (lab == r).sum() > 1]
    pure = sum(1 for r in multi if len(set(seg_trk[lab == r])) == 1)
    by_trk = {}
    for j in range(n):
        if seg_trk[j] >= 0:
            by_trk.setdefault(seg_trk[j], []).append(j)
    extra = sum(len(v) - 1 for v in by_trk.values())
    unjoined = sum(len(set(lab[v])) - 1 for v in by_trk.values())
    pure_c = np.array([len(set(seg_trk[lab == lab[j]])) == 1 for j in range(n)])
    prim = np.zeros(n, bool)
    prim[seg_trk >= 0] = ev.tracks["primary"][seg_trk[seg_trk >= 0]]
    sel = (lab == np.arange(n)) & (m["flags"] == 3) & prim & pure_c
    t0 = m["t0"][sel]
    print(f"{n} segments -> {len(roots)} tracks; {len(multi)} merged, {pure} pure; "
          f"{extra - unjoined} of {extra} splits joined; T0 of {sel.sum()} primaries: "
          f"median {np.median(t0):.3f} bins, {np.mean(np.abs(t0) < 2):.3f} within 2 bins")
    assert pure >= 0.98 * len(multi)
    assert extra - unjoined >= 0.6 * extra
    assert abs(np.median(t0)) < 0.2 and np.mean(np.abs(t0) < 2) > 0.85
    assert not m["near_tie"].any()

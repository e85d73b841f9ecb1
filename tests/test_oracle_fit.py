"""Pins of the oracle's following, conflict resolution and refit.

* on small events the whole-row candidate scan gives the same tracks as the
  time-window scan (the Cauchy-Schwarz prefilter is exact);
* invariants: each cluster is kept by at most one track, every kept track has
  at least MIN_TRACK_HITS hits in distinct rows, the owner of a contested
  cluster is the highest-priority track holding it;
* the refit equals a Kalman fit of the kept hits started from the circle
  through three of them (an independent construction), its covariance is
  PD, and fitted q/pT agrees with generator truth;
* efficiency and fake rate on the one-sector configuration are sane.
"""
import numpy as np
import pytest

import oracle
import tpcsynth
from tpcsynth import truth

PAR = oracle.default_params()
NPADS, XFX, PFX = oracle.geometry()
XR = XFX / 65536.0


def run(ev, brute=False):
    cl = oracle.cluster(ev.pad, ev.time, ev.adc, ev.row_start, ev.n_units, ev.n_time_bins)
    down, up = oracle.find_neighbours(cl, brute_force=brute)
    tl = oracle.build_tracklets(down, up)
    fit = oracle.fit_tracks(cl, tl, brute_force=brute)
    return cl, tl, fit


def kept_hits(fit, t):
    h = fit["hits"][t]
    rows = np.nonzero(h >= 0)[0]
    c = h[rows]
    m = fit["cluster_owner"][c] == t
    return rows[m], c[m]


@pytest.mark.parametrize("ntr,seed", [(1, 1), (3, 2), (5, 3), (40, 4)])
def test_window_search_equals_whole_row_scan(ntr, seed):
    ev = tpcsynth.generate(tpcsynth.config_small(ntr), seed)
    cl, tl, fit = run(ev)
    cl2, tl2, fit2 = run(ev, brute=True)
    assert np.array_equal(fit["hits"], fit2["hits"])
    assert np.array_equal(fit["kept"], fit2["kept"])
    assert np.array_equal(fit["par"], fit2["par"])


@pytest.mark.parametrize("seed", [5, 6])
def test_resolution_invariants(seed):
    ev = tpcsynth.generate(tpcsynth.config_small(120), seed)
    cl, tl, fit = run(ev)
    nt = len(tl["tl_start"])
    owner = fit["cluster_owner"]
    seen = set()
    for t in range(nt):
        h = fit["hits"][t]
        if fit["kept"][t]:
            rows, c = kept_hits(fit, t)
            assert len(c) >= PAR["min_track_hits"]
            assert fit["nhits"][t] == len(c)
            assert not (set(c.tolist()) & seen)
            seen |= set(c.tolist())
            assert fit["row"][t] == rows.min()
    # owner has the highest key among the followed tracks (with >= 15 hits) holding it
    nh = np.array([(fit["hits"][t] >= 0).sum() if fit["follow_ok"][t] else 0 for t in range(nt)])
    best = {}
    for t in range(nt):
        if nh[t] < PAR["min_track_hits"]:
            continue
        for c in fit["hits"][t][fit["hits"][t] >= 0]:
            key = (nh[t], -t)
            if c not in best or key > best[c]:
                best[c] = key
    for c, (n, mt) in best.items():
        t = -mt
        if fit["kept"][t]:
            assert owner[c] == t
        else:
            assert owner[c] == -1


def _circle_seed_at_outer(cl, rows_desc, c_desc, anchor):
    """Independent start of the refit: the circle through the innermost,
    middle and outermost kept clusters (centre from perpendicular bisectors),
    its tangent at the outermost one, dip from the turning angle."""
    import math

    n = len(rows_desc)
    asc_r, asc_c = rows_desc[::-1], c_desc[::-1]
    ia, im, ie = 0, (n + 1) // 2 - 1, n - 1
    pts = [(XR[asc_r[i]], cl["y_fx"][asc_c[i]] / 65536.0) for i in (ia, im, ie)]
    (x1, y1), (x2, y2), (x3, y3) = pts
    A = np.array([[x2 - x1, y2 - y1], [x3 - x1, y3 - y1]])
    rhs = 0.5 * np.array([x2 ** 2 - x1 ** 2 + y2 ** 2 - y1 ** 2, x3 ** 2 - x1 ** 2 + y3 ** 2 - y1 ** 2])
    cx, cy = np.linalg.solve(A, rhs)
    R = math.hypot(x1 - cx, y1 - cy)
    orient = np.sign((x2 - x1) * (y3 - y1) - (y2 - y1) * (x3 - x1))
    rx, ry = x3 - cx, y3 - cy
    tx, ty = (-ry, rx) if orient > 0 else (ry, -rx)
    snp = ty / math.hypot(tx, ty)
    ang = math.atan2(y3 - cy, x3 - cx) - math.atan2(y1 - cy, x1 - cx)
    ang = (ang + math.pi) % (2 * math.pi) - math.pi
    zA = int(cl["z_fx"][asc_c[ia]])
    zE = int(cl["z_fx"][asc_c[ie]])
    tgl = (zE - zA) / 65536.0 / (abs(ang) * R)
    qpt = -(orient / R) / PAR["bz_b"]
    return np.array([y3, (zE - int(anchor)) / 65536.0, snp, tgl, qpt])


def test_refit_is_kalman_fit_of_kept_hits():
    ev = tpcsynth.generate(tpcsynth.config_small(30), 8)
    cl, tl, fit = run(ev)
    rp = dict(PAR, snp_max=PAR["refit_snp_max"])
    C0 = np.diag([PAR["c0r_y"] ** 2, PAR["c0r_z"] ** 2, PAR["c0r_snp"] ** 2, PAR["c0r_tgl"] ** 2,
                  PAR["c0r_qpt"] ** 2])
    checked = 0
    for t in np.nonzero(fit["kept"])[0]:
        rows, c = kept_hits(fit, t)
        order = np.argsort(-rows)
        rows, c = rows[order], c[order]
        anchor = cl["z_fx"][tl["tl_start"][t]]
        my = cl["y_fx"][c] / 65536.0
        mz = (cl["z_fx"][c].astype(np.int64) - anchor) / 65536.0
        p0 = _circle_seed_at_outer(cl, rows, c, anchor)
        vy = [PAR["sigma_y"][r] ** 2 for r in rows]
        vz = [PAR["sigma_z"][r] ** 2 for r in rows]
        rc, p, C, chi2 = oracle.kalman_fit(rows, my, mz, vy, vz, p0, C0, params=rp)
        assert rc == 0
        assert np.allclose(p, fit["par"][t], rtol=1e-9, atol=1e-9)
        iu = np.triu_indices(5)
        assert np.allclose(C[iu], fit["cov"][t], rtol=1e-8, atol=1e-14)
        assert abs(chi2 - fit["chi2"][t]) < 1e-7 * max(1, chi2)
        assert oracle.is_pd(C)
        checked += 1
    assert checked > 5


def test_fitted_momentum_matches_truth():
    ev = tpcsynth.generate(tpcsynth.config_small(60), 10)
    cl, tl, fit = run(ev)
    labels = truth.cluster_labels(ev.deposits, cl, ev.n_units)
    pulls = []
    for t in np.nonzero(fit["kept"])[0]:
        rows, c = kept_hits(fit, t)
        lab = labels[c]
        if np.any(lab < 0):
            continue
        trk = ev.deposits["track"][lab]
        leg = ev.deposits["leg"][lab]
        if len(np.unique(trk)) != 1 or len(np.unique(leg)) != 1:
            continue
        tr = trk[0]
        qpt_true = -ev.tracks["curv"][tr] / tpcsynth.BZ_B
        if leg[0] < 0:
            qpt_true = -qpt_true  # an incoming leg is fitted as the reversed particle
        sig = np.sqrt(fit["cov"][t][14])
        pulls.append((fit["par"][t][4] - qpt_true) / sig)
    pulls = np.array(pulls)
    assert len(pulls) > 20
    # the charge is always right and the momentum within a few sigma
    assert np.median(np.abs(pulls)) < 2.0
    assert np.mean(np.abs(pulls) < 6) > 0.9


def test_one_sector_efficiency_sane():
    ev = tpcsynth.generate(tpcsynth.config_c1(), 101)
    cl, tl, fit = run(ev)
    hits = [kept_hits(fit, t)[1] for t in np.nonzero(fit["kept"])[0]]
    perf = truth.performance(ev.deposits, ev.tracks, cl, ev.n_units, hits)
    assert perf["efficiency"] > 0.85
    assert perf["fake_rate"] < 0.15
    assert np.all(fit["flags"][fit["kept"] == 1] == 0)


def test_empty_event():
    rs = np.zeros(153, np.uint32)
    e = np.zeros(0, np.uint16)
    cl = oracle.cluster(e, e, e, rs, 1, 500)
    down, up = oracle.find_neighbours(cl)
    tl = oracle.build_tracklets(down, up)
    fit = oracle.fit_tracks(cl, tl)
    assert len(tl["tl_start"]) == 0 and fit["kept"].sum() == 0

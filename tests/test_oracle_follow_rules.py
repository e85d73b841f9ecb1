"""Pins of the oracle's track following on hand-built events.

Each event is a handful of clusters placed by hand in one sector: straight
tracks (no curvature, constant z) so that the expected hit set of the
tracklet follows from the stated rules and elementary geometry alone.  The
rules pinned here (following: outward pass A from the tracklet, inward pass
B from the outermost pass-A hit with the covariance reset):

* a search row without an accepted candidate is a miss; following stops at
  the MAX_MISS-th (6th) consecutive miss: a gap of 5 empty rows is bridged,
  a gap of 6 is not (pass A above the tracklet, pass B below it);
* following stops where the predicted |y| exceeds the half-width of the pad
  plane plus 1 cm (pass A outward on an inclined track, pass B inward on a
  track at constant y near the sector edge);
* the accepted candidate is the minimum of (chi2, cluster id) among those with
  chi2 <= CHI2_MAX (16), not the first or the last one found;
* pass B restarts from the seed covariance at the outermost pass-A hit, so a
  candidate is judged with the predicted covariance of a fit of the pass-B
  hits alone.

The chi2 of a planted candidate needs the predicted variance of y at its
row.  For these tracks (sin phi = 0, q/pT = 0, tan lambda = 0 exactly) the
Kalman filter without process noise is a linear Gaussian estimator, so that
variance is the one of the batch least-squares solution with the same prior;
``pred_var_y`` computes it by linear algebra from the straight-line
expansion of the helix, y(x) = y_R + sin(phi_R) dx - b (q/pT) dx^2 / 2,
which is independent of the oracle's propagation code.

Of the rules listed with the method, "pass-B misses count only below the
tracklet's first row" has no observable effect on its own: above that row
the pass-B search rows are exactly the rows pass A searched without success
between its hits, at most MAX_MISS - 1 in a row (pass A stops at MAX_MISS),
and every tracklet row resets the count.  It is pinned here only in that
form: a gap of MAX_MISS - 1 rows above the tracklet is bridged by both
passes.
"""
import math

import numpy as np

import oracle

PAR = oracle.default_params()
NPADS, XFX, _ = oracle.geometry()
X = XFX / 65536.0                      # row radii (cm), pinned in test_geometry
B = PAR["bz_b"]
SY2 = 0.06 ** 2                        # measurement variance of y (cm^2)
PRIOR = np.array([SY2, PAR["c0_snp"] ** 2, PAR["c0_qpt"] ** 2])  # seed variances of (y, snp, q/pT)
Z0 = 100.0                             # drift z of every cluster (cm): peak time 200 bins
TAN10 = math.tan(math.radians(10.0))


def half_width(r):
    """Half-width of the pad plane of row r: the sector spans +-10 degrees."""
    return X[r] * TAN10


def make_event(rows_y):
    """Clusters of one sector: {row: [y (cm), ...]}, all at drift z = Z0.
    Within a row, clusters are numbered by ascending y (same peak time, so
    ascending pad is the canonical order)."""
    y, crow = [], np.zeros(153, np.uint32)
    for r in range(152):
        ys = sorted(rows_y.get(r, []))
        y.extend(ys)
        crow[r + 1] = crow[r] + len(ys)
    n = len(y)
    return dict(y_fx=np.round(np.array(y, np.float64) * 65536).astype(np.int32),
                z_fx=np.full(n, int(Z0 * 65536), np.int32),
                ptime=np.full(n, int(2 * Z0), np.uint16), crow_start=crow, n_units=1)


def run(rows_y, params=None):
    cl = make_event(rows_y)
    down, up = oracle.find_neighbours(cl, params)
    tl = oracle.build_tracklets(down, up, params)
    fit = oracle.fit_tracks(cl, tl, params)
    return cl, tl, fit


def row_of(cl, c):
    return int(np.searchsorted(cl["crow_start"], c, side="right") - 1)


def tracklet_from(cl, tl, r1):
    """Index of the tracklet whose first cluster lies in row r1."""
    rows = [row_of(cl, c) for c in tl["tl_start"]]
    assert r1 in rows, (r1, rows)
    return rows.index(r1)


def hit_rows(fit, t):
    return sorted(np.nonzero(fit["hits"][t] >= 0)[0].tolist())


def line(rows, y=0.0):
    return {r: [y] for r in rows}


def pred_var_y(prior_row, meas_rows, pred_row, prior=PRIOR):
    """Predicted variance of y at pred_row for a straight track with the seed
    prior (variances of y, sin phi, q/pT) at prior_row and one y measurement
    at each of meas_rows (rows may repeat: pass B re-uses pass-A hits), as
    the batch least-squares solution in the parameters (y, sin phi, q/pT) at
    pred_row."""
    xr = X[pred_row]

    def transport(x):  # (y, snp, q/pT) at x from the same at xr, to first order
        d = x - xr
        return np.array([[1.0, d, -B * d * d / 2], [0.0, 1.0, -B * d], [0.0, 0.0, 1.0]])

    G = transport(X[prior_row])
    info = G.T @ np.diag(1.0 / np.asarray(prior)) @ G
    for r in meas_rows:
        h = transport(X[r])[0]
        info += np.outer(h, h) / SY2
    return np.linalg.inv(info)[0, 0]


# ------------------------------------------------------------ max-miss rule
def test_pass_a_bridges_five_empty_rows_not_six():
    # tracklet rows 11..18 (row 10 and 19 unlinked ends), gap of 5 (rows
    # 20-24) before row 25, gap of 6 (rows 26-31) before row 32
    rows = list(range(10, 20)) + [25, 32]
    cl, tl, fit = run(line(rows))
    t = tracklet_from(cl, tl, 11)
    assert tl["tl_len"][t] == 8
    assert hit_rows(fit, t) == list(range(10, 20)) + [25]
    # the count is the parameter: with MAX_MISS = 7 the 6-row gap is bridged
    cl, tl, fit = run(line(rows), dict(max_miss=7))
    assert hit_rows(fit, tracklet_from(cl, tl, 11)) == list(range(10, 20)) + [25, 32]


def test_pass_b_bridges_five_empty_rows_below_the_tracklet_not_six():
    cl, tl, fit = run(line(list(range(10, 20)) + [4]))      # rows 5-9 empty
    assert hit_rows(fit, tracklet_from(cl, tl, 11)) == [4] + list(range(10, 20))
    cl, tl, fit = run(line(list(range(10, 20)) + [3]))      # rows 4-9 empty
    assert hit_rows(fit, tracklet_from(cl, tl, 11)) == list(range(10, 20))
    cl, tl, fit = run(line(list(range(10, 20)) + [3]), dict(max_miss=7))
    assert hit_rows(fit, tracklet_from(cl, tl, 11)) == [3] + list(range(10, 20))


def test_pass_b_gap_above_the_tracklet_does_not_stop_it():
    # pass B steps from row 25 through the 5 empty rows 20-24 and the
    # tracklet to rows 10 and 4 below it
    cl, tl, fit = run(line(list(range(10, 20)) + [25, 4]))
    assert hit_rows(fit, tracklet_from(cl, tl, 11)) == [4] + list(range(10, 20)) + [25]


def test_pass_b_miss_count_restarts_after_each_hit():
    # below the tracklet: 3 empty rows, a hit at row 6, 4 empty rows, a hit
    # at row 1 (7 misses in all, never 6 in a row)
    cl, tl, fit = run(line(list(range(10, 20)) + [6, 1]))
    assert hit_rows(fit, tracklet_from(cl, tl, 11)) == [1, 6] + list(range(10, 20))


# ------------------------------------------------------------ edge rule
def test_pass_a_stops_where_the_track_leaves_the_pad_plane():
    # inclined straight track y = m (x - x0); the row where |y| first exceeds
    # the half-width + 1 cm is placed mid-way between two rows
    m, R = 0.4, 40
    g = lambda r, x0: m * (X[r] - x0) - (half_width(r) + PAR["edge_margin"])  # noqa: E731
    x0 = X[R] - (half_width(R) + PAR["edge_margin"] + 0.1) / m
    assert g(R, x0) > 0.05 and g(R - 1, x0) < -0.05
    # tracklet rows 11-18; row 20 empty so the outer clusters form their own
    # tracklet and pass A of the first one has to search rows 21 onward
    rows = [r for r in range(10, 80) if r != 20]
    cl, tl, fit = run({r: [m * (X[r] - x0)] for r in rows})
    t = tracklet_from(cl, tl, 11)
    assert tl["tl_len"][t] == 8
    assert hit_rows(fit, t) == [r for r in range(10, R) if r != 20]
    # with no margin the stop comes where |y| exceeds the half-width itself
    R0 = next(r for r in range(19, 80) if m * (X[r] - x0) > half_width(r))
    assert R0 < R and m * (X[R0] - x0) - half_width(R0) > 0.05
    cl, tl, fit = run({r: [m * (X[r] - x0)] for r in rows}, dict(edge_margin=0.0))
    assert hit_rows(fit, tracklet_from(cl, tl, 11)) == [r for r in range(10, R0) if r != 20]


def test_pass_b_stops_where_the_track_leaves_the_pad_plane():
    # a track at constant y near the edge: the pad plane narrows inward, so
    # pass B (inward) crosses the limit at row R; tracklet rows R+1..R+11
    R = 50
    lim = lambda r: half_width(r) + PAR["edge_margin"]  # noqa: E731
    rows = list(range(R, R + 13))
    y_out = 0.5 * (lim(R) + lim(R + 1))       # beyond the limit at row R only
    cl, tl, fit = run(line(rows, y_out))
    assert hit_rows(fit, tracklet_from(cl, tl, R + 1)) == list(range(R + 1, R + 13))
    y_in = lim(R) - 0.05                      # beyond the pad plane, inside the margin
    assert y_in - half_width(R) > 0.5
    cl, tl, fit = run(line(rows, y_in))
    assert hit_rows(fit, tracklet_from(cl, tl, R + 1)) == list(range(R, R + 13))
    # the same side of the limit for negative y
    cl, tl, fit = run(line(rows, -y_out))
    assert hit_rows(fit, tracklet_from(cl, tl, R + 1)) == list(range(R + 1, R + 13))


# ------------------------------------------------------------ candidate choice
def _s19():
    """Residual variance of y at row 19 in pass A: seed prior at row 11,
    updates at the tracklet rows 11..18."""
    return pred_var_y(11, range(11, 19), 19) + SY2


def test_smallest_chi2_wins_over_a_lower_cluster_id():
    s = math.sqrt(_s19())
    rows = line(range(10, 19))
    rows[19] = [-3.0 * s, 2.0 * s]           # chi2 9 (lower id), chi2 4
    cl, tl, fit = run(rows)
    t = tracklet_from(cl, tl, 11)
    assert fit["hits"][t][19] == cl["crow_start"][19] + 1
    rows[19] = [-2.0 * s, 3.0 * s]           # chi2 4 (lower id), chi2 9
    cl, tl, fit = run(rows)
    assert fit["hits"][tracklet_from(cl, tl, 11)][19] == cl["crow_start"][19]


def test_equal_chi2_goes_to_the_lower_cluster_id():
    s = math.sqrt(_s19())
    rows = line(range(10, 19))
    rows[19] = [-2.0 * s, 2.0 * s]           # the same chi2, exactly
    cl, tl, fit = run(rows)
    t = tracklet_from(cl, tl, 11)
    assert fit["hits"][t][19] == cl["crow_start"][19]
    assert fit["near_tie"][t] > 0            # logged as a near tie


def test_chi2_cut_at_sixteen():
    s = math.sqrt(_s19())
    for chi2, picked in ((15.0, True), (17.0, False)):
        rows = line(range(10, 19))
        rows[19] = [math.sqrt(chi2) * s]
        cl, tl, fit = run(rows)
        t = tracklet_from(cl, tl, 11)
        assert (fit["hits"][t][19] >= 0) == picked, chi2
    # the cut is the parameter
    rows = line(range(10, 19))
    rows[19] = [math.sqrt(17.0) * s]
    cl, tl, fit = run(rows, dict(chi2_max=18.0))
    assert fit["hits"][tracklet_from(cl, tl, 11)][19] >= 0


def test_tracklet_hits_are_taken_without_a_search():
    # a tracklet cluster inside the tracklet (row 16; not one of the seed
    # points of rows 11, 14 and 18) is off the line by 0.45 cm: the neighbour
    # finder links it (midpoint deviations 0.45 and 0.9 cm <= 1 cm), but its
    # chi2 against the prediction of either pass is far above the cut, so it
    # is on the track only because tracklet rows are updated unconditionally
    par = dict(c0_snp=0.02)
    prior = [SY2, 0.02 ** 2, PAR["c0_qpt"] ** 2]
    dy = 0.45
    assert dy * dy / (pred_var_y(11, range(11, 16), 16, prior) + SY2) > 20
    assert dy * dy / (pred_var_y(19, [19, 18, 17], 16, prior) + SY2) > 20
    rows = line(range(10, 20))
    rows[16] = [dy]
    cl, tl, fit = run(rows, par)
    t = tracklet_from(cl, tl, 11)
    assert tl["tl_len"][t] == 8
    assert fit["hits"][t][16] == cl["crow_start"][16]


def test_pass_b_searches_from_the_row_below_its_start():
    # pass A refuses the cluster of row 19 (0.6 cm off a tightly fitted
    # line) and takes row 20; pass B restarts at row 20 with the seed
    # covariance (sin phi sigma 0.2 here) and accepts row 19 at once
    par = dict(c0_snp=0.2)
    prior = [SY2, 0.2 ** 2, PAR["c0_qpt"] ** 2]
    dy = 0.6
    chi2_a = dy * dy / (pred_var_y(11, range(11, 19), 19, prior) + SY2)
    chi2_b = dy * dy / (pred_var_y(20, [20], 19, prior) + SY2)
    assert chi2_a > 20 and chi2_b < 12
    rows = line(list(range(10, 19)) + [20])
    rows[19] = [dy]
    cl, tl, fit = run(rows, par)
    t = tracklet_from(cl, tl, 11)
    assert tl["tl_len"][t] == 8
    assert hit_rows(fit, t) == list(range(10, 21))


def test_pass_b_judges_candidates_with_the_reset_covariance():
    # pass A: tracklet 11..18 and row 19; pass B restarts at row 19 with the
    # seed covariance, updates rows 19..11 and meets a candidate at row 10
    s_reset = pred_var_y(19, range(19, 10, -1), 10) + SY2
    # without the reset, pass B would carry pass A's information twice
    s_carry = pred_var_y(11, list(range(11, 20)) + list(range(19, 10, -1)), 10) + SY2
    dy = math.sqrt(12.0 * s_reset)
    assert dy * dy / s_carry > 16.0          # the two readings decide differently
    rows = line(range(11, 20))
    rows[10] = [dy]
    cl, tl, fit = run(rows)
    t = tracklet_from(cl, tl, 11)
    assert tl["tl_len"][t] == 8
    assert hit_rows(fit, t) == list(range(10, 20))
    # and at chi2 17 under the reset it is refused
    rows[10] = [math.sqrt(17.0 * s_reset)]
    cl, tl, fit = run(rows)
    assert hit_rows(fit, tracklet_from(cl, tl, 11)) == list(range(11, 20))

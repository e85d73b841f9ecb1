"""Evidence for the refit's start (the reading of the final refit).

Two readings of "refit the kept hits" were considered:

* pass-B reading: take the pass-B state at its innermost row, propagate it
  out to the outermost kept row, reset the covariance to the seed covariance
  (sigma_y, sigma_z of one measurement, 0.1, 0.1, 10) and filter inward;
* chosen reading (the oracle's): start from the circle through the
  innermost, middle and outermost kept clusters at the outermost one, with a
  broad prior (5 cm, 5 cm, 0.5, 0.5, 10), and filter inward.

The pass-B reading treats the propagated pass-B state as a measurement of y
and z at the outermost row with the error of one cluster, although it comes
from a propagation over up to 150 rows.  Against generator truth this shows
as wider q/pT pulls and more outliers; the chosen reading's result depends on
the kept clusters alone.  This test computes both readings on the same kept
hit sets (the pass-B reading from the oracle's pass-B state with its exposed
propagation and Kalman primitives) and compares their q/pT pulls.
"""
import numpy as np

import oracle
import tpcsynth
from tpcsynth import truth

PAR = oracle.default_params()
_, XFX, _ = oracle.geometry()
X = XFX / 65536.0


def _pulls(seeds):
    rp = dict(PAR, snp_max=PAR["refit_snp_max"])
    C0 = np.diag([PAR["sigma_y"][0] ** 2, PAR["sigma_z"][0] ** 2, PAR["c0_snp"] ** 2,
                  PAR["c0_tgl"] ** 2, PAR["c0_qpt"] ** 2])
    chosen, passb, passb_fail = [], [], 0
    for seed in seeds:
        ev = tpcsynth.generate(tpcsynth.config_small(1500, sector_mode=0), seed)
        res = oracle.process(ev.pad, ev.time, ev.adc, ev.row_start, ev.n_units, ev.n_time_bins,
                             n_threads=8)
        cl, tl, fit = res["clusters"], res["tracklets"], res["fit"]
        labels = truth.cluster_labels(ev.deposits, cl, ev.n_units)
        for t in np.nonzero(fit["kept"])[0]:
            h = fit["hits"][t]
            rows = np.nonzero(h >= 0)[0]
            c = h[rows]
            m = fit["cluster_owner"][c] == t
            rows, c = rows[m], c[m]
            lab = labels[c]
            if np.any(lab < 0):
                continue
            trk, leg = ev.deposits["track"][lab], ev.deposits["leg"][lab]
            if len(np.unique(trk)) != 1 or len(np.unique(leg)) != 1:
                continue  # one true track leg per fitted track
            q_true = -ev.tracks["curv"][trk[0]] / tpcsynth.BZ_B
            if leg[0] < 0:
                q_true = -q_true  # an incoming leg is fitted as the reversed particle
            chosen.append((fit["par"][t][4] - q_true) / np.sqrt(fit["cov"][t][14]))
            pb = fit["pb_state"][t]
            order = np.argsort(-rows)
            rd, cd = rows[order], c[order]
            rc, p = oracle.helix_propagate(pb[:5], X[int(pb[5])], X[rd[0]], rp)
            if rc:
                passb_fail += 1
                passb.append(np.inf)
                continue
            anchor = int(cl["z_fx"][tl["tl_start"][t]])
            my = cl["y_fx"][cd] / 65536.0
            mz = (cl["z_fx"][cd].astype(np.int64) - anchor) / 65536.0
            vy = [PAR["sigma_y"][r] ** 2 for r in rd]
            vz = [PAR["sigma_z"][r] ** 2 for r in rd]
            rc, p2, C2, _ = oracle.kalman_fit(rd, my, mz, vy, vz, p, C0, params=rp)
            if rc in (1, 2):
                passb_fail += 1
                passb.append(np.inf)
                continue
            passb.append((p2[4] - q_true) / np.sqrt(C2[4, 4]))
    return np.abs(np.array(chosen)), np.abs(np.array(passb)), passb_fail


def test_chosen_refit_start_gives_narrower_pulls_than_the_pass_b_start():
    chosen, passb, passb_fail = _pulls([1000, 1001])
    n = len(chosen)
    assert n > 5000
    q68_c, q68_s = np.percentile(chosen, 68.27), np.percentile(passb, 68.27)
    out_c, out_s = np.mean(chosen > 5), np.mean(passb > 5)
    print(f"q/pT pulls on {n} tracks: 68% quantile of |pull| chosen {q68_c:.3f}, "
          f"pass-B reading {q68_s:.3f}; |pull| > 5: {out_c:.4f} vs {out_s:.4f} "
          f"(pass-B reading failures {passb_fail})")
    assert q68_c < q68_s - 0.04
    assert out_c < out_s
    assert np.all(np.isfinite(chosen))

"""Helpers shared by the GPU parity tests: run the library, run the oracle,
and compare stage outputs under the stated rules.

Rules (from the acceptance statement of the method):
* integer outputs bit-exact: clusters (order, peaks, charges, moments, flags,
  fixed-point positions), links, tracklets, hit sets and cluster ownership;
* centroids within 1e-4 pad / time bin;
* track parameters within 1e-4 relative, with floors where a relative error
  is undefined at zero (y, z: 1 cm; sin phi, tan lambda: 0.01; q/pT: 0.1
  c/GeV, i.e. pT above 10 GeV/c);
* a track whose FP64 oracle refit is not determined to that bar by inputs
  known to binary32 precision -- its parameters move by more than 1% of the
  bar when the refit restarts from a start scaled by 1 + 2^-24 -- is exempt
  from the parameter comparison only (its hits and ownership are still
  compared); their number is reported;
* hit decisions that the oracle logs as near ties (chi2 against the cut or
  best against second best within 1e-3, |sin phi| against its limit within
  1e-5, |y| against the edge within 1e-4 cm) may differ between FP32 and
  FP64: such tracklets, and every tracklet sharing a cluster with them, are
  exempt from the hit and parameter comparison; their number is reported.
"""
import numpy as np

import oracle
from paper_2208_07412_amd import tpc

NROW = 152
FLOORS = np.array([1.0, 1.0, 1e-2, 1e-2, 0.1])
PAR_RTOL = 1e-4
COND_LIMIT = 0.01  # fraction of the bar the oracle may move under one FP32 unit
PAR_NAMES = ("y", "z", "snp", "tgl", "qpt")


def run_gpu(ev, params=None, max_tracklets=None, labels=False, moments=True, follow=True,
            reco=None, tuning=None):
    ns = max(ev.n_samples, 1)
    mt = max_tracklets or max(ns // 8, 1024)
    own = reco is None
    if own:
        reco = tpc.Reco(ev.n_units, ev.n_time_bins, ns, mt, param_overrides=params)
    if tuning:
        reco.set_tuning(**tuning)
    zs = tpc.to_device_zs(ev.pad, ev.time, ev.adc, ev.row_start, ev.n_units, ev.n_time_bins)
    cl = reco.alloc_clusters(ev.n_units, ev.n_time_bins, ns, n_samples=ns, moments=moments,
                             labels=labels)
    links = reco.alloc_links(ns)
    tl = reco.alloc_tracklets(mt)
    tr = reco.alloc_tracks(mt, ns, ns, follow_capacity=mt if follow else 0)
    reco.process(zs, cl, links, tl, tr)
    counts = reco.sync()
    n = counts["n_clusters"]
    out = dict(counts=counts, clusters=tpc.clusters_to_host(cl, ev.n_units),
               links=tpc.links_to_host(links, n), tracklets=tpc.tracklets_to_host(tl))
    out["tracks"] = tpc.tracks_to_host(tr, n, counts["n_tracklets"] if follow else 0)
    if own:
        reco.close()
    return out


def run_oracle(ev, params=None, labels=False, n_threads=8):
    return oracle.process(ev.pad, ev.time, ev.adc, ev.row_start, ev.n_units, ev.n_time_bins,
                          params=params, n_threads=n_threads, labels=labels, cond=True)


def ill_conditioned(ofit, t):
    """The FP64 refit of tracklet t moves by more than COND_LIMIT of the bar
    (or fails) when restarted from a start perturbed by one FP32 unit."""
    pc = ofit.get("par_cond")
    if pc is None:
        return False
    op = ofit["par"][t]
    d = np.abs(pc[t] - op) / (PAR_RTOL * np.maximum(np.abs(op), FLOORS))
    return not np.all(d <= COND_LIMIT)


def _diff_report(g, o, keys):
    lines = []
    for k in keys:
        if k not in g:
            continue
        a = g[k].astype(np.float64)
        b = o[k].astype(np.float64)
        bad = np.nonzero(a != b)[0]
        if len(bad):
            i = bad[:5]
            lines.append(f"{k}: {len(bad)} differ, first {i.tolist()} gpu {a[i].tolist()} "
                         f"oracle {b[i].tolist()}")
    return "\n".join(lines)


def compare_clusters(g, o, labels=False):
    n = len(o["y_fx"])
    assert len(g["y_fx"]) == n, (len(g["y_fx"]), n)
    assert np.array_equal(g["crow_start"], o["crow_start"])
    rep = _diff_report(g, o, ("ppad", "ptime", "qtot", "qmax", "sp", "st", "spp", "stt", "nsamp",
                              "flags", "y_fx", "z_fx"))
    if rep:
        print(rep)
    for k in ("y_fx", "z_fx", "qtot", "qmax", "ppad", "ptime", "flags"):
        assert np.array_equal(g[k].astype(np.int64), o[k].astype(np.int64)), k
    for k in ("sp", "st", "spp", "stt", "nsamp"):
        if k in g:
            assert np.array_equal(g[k].astype(np.int64), o[k].astype(np.int64)), k
    # centroid = peak + offset, compared in pads / time bins
    for k, pk, dk in (("pad", "ppad", "dpad"), ("time", "ptime", "dtime")):
        cen = g[pk].astype(np.float64) + g[dk].astype(np.float64)
        assert np.max(np.abs(cen - o[k]), initial=0) <= 1e-4, k
    for k in ("s2pad", "s2time"):
        assert np.max(np.abs(g[k] - o[k]), initial=0) <= 1e-4, k
    if labels:
        assert np.array_equal(g["sample_label"][: len(o["sample_label"])], o["sample_label"])


def kept_hits_oracle(fit, t):
    h = fit["hits"][t]
    rows = np.nonzero(h >= 0)[0]
    c = h[rows]
    return c[fit["cluster_owner"][c] == t]


def exempt_tracklets(ofit, gfollow):
    """Near-tie tracklets and every tracklet sharing a cluster with them."""
    nt = len(ofit["near_tie"])
    near = set(np.nonzero(ofit["near_tie"] > 0)[0].tolist())
    if not near:
        return near
    cl_of = {}
    for src in (ofit["hits"], gfollow):
        if src is None:
            continue
        for t in range(nt):
            for c in src[t][src[t] >= 0]:
                cl_of.setdefault(int(c), set()).add(t)
    ex = set(near)
    for t in near:
        for src in (ofit["hits"], gfollow):
            if src is None:
                continue
            for c in src[t][src[t] >= 0]:
                ex |= cl_of.get(int(c), set())
    return ex


def compare_fit(g, o, check_params=True):
    """Compares following, tracks and ownership; returns the number of exempt
    tracklets.  All violations are collected and printed before asserting."""
    ofit = o["fit"]
    gtr = g["tracks"]
    nt = len(o["tracklets"]["tl_start"])
    gf = gtr.get("follow_hits")
    ex = exempt_tracklets(ofit, gf)
    bad = []
    if gf is not None:
        for t in range(nt):
            if t in ex:
                continue
            oh = ofit["hits"][t] if ofit["follow_ok"][t] else np.full(NROW, -1)
            if not np.array_equal(gf[t], oh):
                bad.append(("follow", t, np.nonzero(gf[t] != oh)[0].tolist()))
    gidx = {int(t): j for j, t in enumerate(gtr["tracklet"])}
    okept = set(np.nonzero(ofit["kept"])[0].tolist())
    worst = 0.0
    n_ill = 0
    rels = []
    for t in range(nt):
        if t in ex:
            continue
        if (t in gidx) != (t in okept):
            bad.append(("kept", t, t in gidx, t in okept))
            continue
        if t not in okept:
            continue
        j = gidx[t]
        gh = gtr["hits"][gtr["hit_start"][j]:gtr["hit_start"][j + 1]]
        oh = np.sort(kept_hits_oracle(ofit, t))
        if not np.array_equal(np.sort(gh), oh):
            bad.append(("hits", t))
            continue
        if check_params:
            op = ofit["par"][t]
            gp = gtr["par"][j].astype(np.float64)
            if ill_conditioned(ofit, t):
                n_ill += 1
            else:
                r = np.abs(gp - op) / (PAR_RTOL * np.maximum(np.abs(op), FLOORS))
                rels.append(np.abs(gp - op) / np.maximum(np.abs(op), FLOORS))
                worst = max(worst, float(r.max()))
                if np.any(r > 1):
                    bad.append(("par", t, gp.tolist(), op.tolist(), r.round(3).tolist()))
            if gtr["row"][j] != ofit["row"][t] or gtr["ndf"][j] != 2 * ofit["nhits"][t] - 5:
                bad.append(("row/ndf", t))
    gct = gtr["cluster_track"]
    gtl = gtr["tracklet"]
    n_own = 0
    for c in range(len(ofit["cluster_owner"])):
        ot = ofit["cluster_owner"][c]
        gt = int(gtl[gct[c]]) if gct[c] >= 0 else -1
        if ot in ex or gt in ex:
            continue
        if ot != gt:
            n_own += 1
            if n_own <= 5:
                bad.append(("owner", c, ot, gt))
    print(f"fit parity: {nt} tracklets, {len(ex)} exempt, {len(gidx)} gpu tracks, "
          f"{n_ill} ill-conditioned refits (parameters not compared), "
          f"worst parameter deviation {worst:.3f} of tolerance, {len(bad)} violations, "
          f"{n_own} ownership differences")
    if rels:
        R = np.array(rels)
        q = np.percentile(R, [50, 99, 100], axis=0)
        print("  relative error vs FP64 oracle (|gpu - oracle| / max(|oracle|, floor)):")
        for i, name in enumerate(PAR_NAMES):
            print(f"    {name:4s} median {q[0][i]:.2e}  p99 {q[1][i]:.2e}  max {q[2][i]:.2e}")
    for v in bad[:20]:
        print("  ", v)
    assert not bad
    return len(ex)


def cov_pd(cov15):
    out = []
    iu = np.triu_indices(5)
    for c in cov15:
        M = np.zeros((5, 5))
        M[iu] = c
        M = M + M.T - np.diag(np.diag(M))
        out.append(bool(np.all(np.linalg.eigvalsh(M.astype(np.float64)) > 0)))
    return np.array(out, dtype=bool)

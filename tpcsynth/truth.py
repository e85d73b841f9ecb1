"""Generator-truth tools: cluster labels and tracking performance.

These run on reconstructed clusters and tracks (from either the oracle or the
GPU library) and compare them with the generator's deposits.  They are
analysis tools on the input side, not part of the reconstruction.

Cluster label: the deposit in the same (unit,row) whose centre cell lies in
the cluster's 5x5 window around the peak and whose expected charge in the
peak sample (Q * f_pad * f_time) is largest; ties go to the lower deposit id.

Segments: a truth segment is (track, unit, leg).  It is findable when at
least 20 clusters carry its label.  A reconstructed track is good when at
least 90% of its clusters carry its majority segment; otherwise it is fake.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erfc

NROW = 152


def _frac(mu: np.ndarray, cell: np.ndarray, sigma: float = 0.8) -> np.ndarray:
    s = sigma * math.sqrt(2.0)
    return 0.5 * (erfc(-(cell + 0.5 - mu) / s) - erfc(-(cell - 0.5 - mu) / s))


def cluster_labels(deposits: dict, clusters: dict, n_units: int) -> np.ndarray:
    """Deposit id of each cluster (or -1)."""
    crow = np.asarray(clusters["crow_start"], np.int64)
    nc = len(clusters["ppad"])
    ur_c = np.repeat(np.arange(n_units * NROW, dtype=np.int64), np.diff(crow))
    key_c = (ur_c * 65536 + clusters["ptime"].astype(np.int64)) * 256 + clusters["ppad"].astype(np.int64)
    labels = np.full(nc, -1, np.int64)
    if nc == 0 or len(deposits["mu_pad"]) == 0:
        return labels
    mu_p = deposits["mu_pad"]
    mu_t = deposits["mu_time"]
    pc = np.floor(mu_p + 0.5).astype(np.int64)
    tc = np.floor(mu_t + 0.5).astype(np.int64)
    ur_d = deposits["unit"].astype(np.int64) * NROW + deposits["row"]
    q = deposits["q"]
    did = deposits["id"].astype(np.int64)
    order = np.argsort(key_c)
    ks = key_c[order]
    cs, vs, ds = [], [], []
    for dt in range(-2, 3):
        ft = _frac(mu_t, tc + dt)
        for dp in range(-2, 3):
            pp = pc + dp
            tt = tc + dt
            ok = (pp >= 0) & (tt >= 0)
            key = (ur_d * 65536 + tt) * 256 + pp
            pos = np.searchsorted(ks, key)
            pos = np.minimum(pos, nc - 1)
            hit = ok & (ks[pos] == key)
            cs.append(order[pos[hit]])
            vs.append((q * _frac(mu_p, pp) * ft)[hit])
            ds.append(did[hit])
    c = np.concatenate(cs)
    v = np.concatenate(vs)
    d = np.concatenate(ds)
    if len(c):
        # per cluster: the largest expected charge, ties to the lower deposit id
        srt = np.lexsort((d, -v, c))
        first = np.ones(len(srt), bool)
        first[1:] = c[srt][1:] != c[srt][:-1]
        labels[c[srt][first]] = d[srt][first]
    return labels


def segment_ids(deposits: dict) -> np.ndarray:
    """Segment key (track, unit, leg) of every deposit, as one int64."""
    return (deposits["track"].astype(np.int64) * 64 + deposits["unit"]) * 2 + (deposits["leg"] > 0)


def performance(deposits: dict, tracks: dict, clusters: dict, n_units: int,
                track_hits: list, labels: np.ndarray = None) -> dict:
    """Efficiency, fake and clone rates of reconstructed tracks.

    track_hits: list of cluster-id arrays, one per reconstructed track.
    """
    if labels is None:
        labels = cluster_labels(deposits, clusters, n_units)
    seg_dep = segment_ids(deposits)
    seg_cl = np.where(labels >= 0, seg_dep[np.maximum(labels, 0)], -1)
    segs, counts = np.unique(seg_cl[seg_cl >= 0], return_counts=True)
    findable = set(segs[counts >= 20].tolist())
    matched = {}
    n_tr = len(track_hits)
    lens = np.array([len(h) for h in track_hits], dtype=np.int64)
    if n_tr and lens.sum():
        hits = np.concatenate([np.asarray(h, np.int64) for h in track_hits])
        tid = np.repeat(np.arange(n_tr, dtype=np.int64), lens)
        sg = seg_cl[hits]
        m = sg >= 0
        tid, sg = tid[m], sg[m]
        # per (track, segment) counts, then per track the largest count with
        # ties to the smaller segment id
        o = np.lexsort((sg, tid))
        tid, sg = tid[o], sg[o]
        new = np.ones(len(sg), bool)
        new[1:] = (tid[1:] != tid[:-1]) | (sg[1:] != sg[:-1])
        starts = np.nonzero(new)[0]
        cnt = np.diff(np.append(starts, len(sg)))
        t_run, s_run = tid[starts], sg[starts]
        o2 = np.lexsort((s_run, -cnt, t_run))
        first = np.ones(len(o2), bool)
        first[1:] = t_run[o2][1:] != t_run[o2][:-1]
        best_t, best_s, best_c = t_run[o2][first], s_run[o2][first], cnt[o2][first]
        good = best_c >= 0.9 * lens[best_t]
        gs, gc = np.unique(best_s[good], return_counts=True)
        matched = dict(zip(gs.tolist(), gc.tolist()))
        n_fake = n_tr - int(good.sum())
    else:
        n_fake = n_tr
    n_find = len(findable)
    n_match = sum(1 for s in findable if s in matched)
    clones = sum(max(0, matched[s] - 1) for s in findable if s in matched)
    # split by primary/secondary and pT bin
    trk = np.array([s // 128 for s in findable], dtype=np.int64)
    ok = np.array([s in matched for s in findable], dtype=bool)
    split = {}
    if len(trk):
        pt = tracks["pt"][trk]
        prim = tracks["primary"][trk]
        for name, m in (("primary", prim), ("secondary", ~prim), ("pt<0.2", pt < 0.2),
                        ("0.2<pt<1", (pt >= 0.2) & (pt < 1)), ("pt>1", pt >= 1)):
            if m.sum():
                split[name] = float(ok[m].mean())
    return dict(findable=n_find, matched=n_match,
                efficiency=n_match / n_find if n_find else float("nan"),
                fake_rate=n_fake / n_tr if n_tr else 0.0,
                clone_rate=clones / n_match if n_match else 0.0,
                n_tracks=n_tr, split=split)

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
    best = np.full(nc, -np.inf)
    mu_p = deposits["mu_pad"]
    mu_t = deposits["mu_time"]
    pc = np.floor(mu_p + 0.5).astype(np.int64)
    tc = np.floor(mu_t + 0.5).astype(np.int64)
    ur_d = deposits["unit"].astype(np.int64) * NROW + deposits["row"]
    q = deposits["q"]
    did = deposits["id"].astype(np.int64)
    order = np.argsort(key_c)
    ks = key_c[order]
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
            ci = order[pos[hit]]
            val = (q * _frac(mu_p, pp) * ft)[hit]
            d = did[hit]
            # process in deposit-id order so that ties keep the lower id
            for c, v, dd in zip(ci, val, d):
                if v > best[c] or (v == best[c] and dd < labels[c]):
                    best[c] = v
                    labels[c] = dd
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
    n_fake = 0
    for h in track_hits:
        s = seg_cl[np.asarray(h, np.int64)]
        s = s[s >= 0]
        if len(s) == 0:
            n_fake += 1
            continue
        vals, cnt = np.unique(s, return_counts=True)
        j = np.argmax(cnt)
        if cnt[j] >= 0.9 * len(h):
            matched[vals[j]] = matched.get(vals[j], 0) + 1
        else:
            n_fake += 1
    n_find = len(findable)
    n_match = sum(1 for s in findable if s in matched)
    clones = sum(max(0, matched[s] - 1) for s in findable if s in matched)
    n_tr = len(track_hits)
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

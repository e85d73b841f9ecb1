"""Per-unit views of a batched reconstruction, for sampled-unit parity at
full size: a unit (one sector of one frame) is reconstructed independently
of the others, so the oracle can be run on one unit alone and compared with
that unit's part of a call over many units."""
import numpy as np

import tpcsynth
from paper_2208_07412_amd import tpc

NROW = tpc.NROW


def unit_event(ev, u):
    s0, s1 = int(ev.row_start[u * NROW]), int(ev.row_start[(u + 1) * NROW])
    rs = (ev.row_start[u * NROW:(u + 1) * NROW + 1].astype(np.int64) - s0).astype(np.uint32)
    cfg = tpcsynth.config_small(0, n_time_bins=ev.n_time_bins)
    return tpcsynth.Event(cfg, ev.pad[s0:s1], ev.time[s0:s1], ev.adc[s0:s1], rs, 1,
                          ev.n_time_bins, {}, {}, None)


def unit_view(sl, u):
    """The slice's outputs restricted to unit u, indices rebased to the unit."""
    lu = u - sl["u0"]
    c, tr = sl["clusters"], sl["tracks"]
    crow = c["crow_start"].astype(np.int64)
    c0, c1 = int(crow[lu * NROW]), int(crow[(lu + 1) * NROW])
    cl = {k: v[c0:c1] for k, v in c.items() if isinstance(v, np.ndarray) and k != "crow_start"}
    cl["crow_start"] = (crow[lu * NROW:(lu + 1) * NROW + 1] - c0).astype(np.uint32)
    shift = lambda a: np.where(a >= 0, a - c0, a)
    links = {k: shift(sl["links"][k][c0:c1].astype(np.int64)) for k in ("down", "up", "downc", "upc")}
    ts = sl["tracklets"]["tl_start"].astype(np.int64)
    tsel = np.nonzero((ts >= c0) & (ts < c1))[0]
    t0 = int(tsel[0]) if len(tsel) else 0
    assert np.array_equal(tsel, np.arange(t0, t0 + len(tsel)))  # a unit's tracklets are contiguous
    tl = dict(tl_start=(ts[tsel] - c0).astype(np.uint32), tl_len=sl["tracklets"]["tl_len"][tsel])
    ttl = tr["tracklet"].astype(np.int64)
    jsel = np.nonzero((ttl >= t0) & (ttl < t0 + len(tsel)))[0]
    j0 = int(jsel[0]) if len(jsel) else 0
    hs = tr["hit_start"].astype(np.int64)
    h0 = int(hs[j0]) if len(jsel) else 0
    h1 = int(hs[j0 + len(jsel)]) if len(jsel) else 0
    ct = tr["cluster_track"][c0:c1].astype(np.int64)
    tracks = dict(tracklet=(ttl[jsel] - t0).astype(np.uint32), par=tr["par"][jsel],
                  cov=tr["cov"][jsel], chi2=tr["chi2"][jsel], ndf=tr["ndf"][jsel],
                  row=tr["row"][jsel], flags=tr["flags"][jsel],
                  hit_start=(hs[j0:j0 + len(jsel) + 1] - h0).astype(np.uint32),
                  hits=(tr["hits"][h0:h1].astype(np.int64) - c0).astype(np.uint32),
                  cluster_track=np.where(ct >= 0, ct - j0, -1))
    return dict(clusters=cl, links=links, tracklets=tl, tracks=tracks)

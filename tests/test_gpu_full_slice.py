"""Parity at the full size of the headline workload (the 2 ms slice: 100
collisions, 36 sectors x 152 rows, 10,500 bins, seed 303), in a launch
configuration the benchmark times (default launch shapes, the units in four
slices on concurrent streams, one graph replay; the other slicings give the
same outputs, which the pipeline tests check).  The oracle is run on sampled
units one by one (a unit is reconstructed independently of the others), and
properties that hold at any size are checked over the whole slice."""
import numpy as np
import pytest
import torch

import tpcsynth
from paper_2208_07412_amd import pipeline, tpc

from _parity import compare_clusters, compare_fit, run_oracle

pytestmark = pytest.mark.gpu

NROW = tpc.NROW
UNITS = (0, 17, 35)


@pytest.fixture(scope="module")
def slice_run():
    ev = tpcsynth.generate(tpcsynth.config_c3(303, 100), 303)
    print(f"slice: {ev.n_samples} samples", flush=True)
    zs = tpc.to_device_zs(ev.pad, ev.time, ev.adc, ev.row_start, ev.n_units, ev.n_time_bins)
    p = pipeline.Pipeline(zs, 4)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        p.enqueue()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        p.enqueue()
    with torch.cuda.stream(s):
        g.replay()
    torch.cuda.synchronize()
    counts = p.sync()
    out = []
    for sl in p.slices:
        n = int(sl.cl["n_clusters"].item())
        nu = sl.u1 - sl.u0
        out.append(dict(u0=sl.u0, u1=sl.u1,
                        clusters=tpc.clusters_to_host(sl.cl, nu),
                        links=tpc.links_to_host(sl.links, n),
                        tracklets=tpc.tracklets_to_host(sl.tl),
                        tracks=tpc.tracks_to_host(sl.tr, n)))
    del g
    p.close()
    return ev, counts, out


def _unit_event(ev, u):
    s0, s1 = int(ev.row_start[u * NROW]), int(ev.row_start[(u + 1) * NROW])
    rs = (ev.row_start[u * NROW:(u + 1) * NROW + 1].astype(np.int64) - s0).astype(np.uint32)
    cfg = tpcsynth.config_small(0, n_time_bins=ev.n_time_bins)
    return tpcsynth.Event(cfg, ev.pad[s0:s1], ev.time[s0:s1], ev.adc[s0:s1], rs, 1,
                          ev.n_time_bins, {}, {}, None)


def _unit_view(sl, u):
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


@pytest.mark.parametrize("u", UNITS)
def test_sampled_unit_equals_oracle(slice_run, u):
    ev, counts, out = slice_run
    sl = next(s for s in out if s["u0"] <= u < s["u1"])
    g = _unit_view(sl, u)
    o = run_oracle(_unit_event(ev, u))
    compare_clusters(g["clusters"], o["clusters"])
    assert np.array_equal(g["links"]["down"], o["down"])
    assert np.array_equal(g["links"]["up"], o["up"])
    assert np.array_equal(g["links"]["upc"], o["tracklets"]["upc"])
    assert np.array_equal(g["tracklets"]["tl_start"], o["tracklets"]["tl_start"])
    assert np.array_equal(g["tracklets"]["tl_len"], o["tracklets"]["tl_len"])
    compare_fit(g, o)


def test_whole_slice_properties(slice_run):
    ev, counts, out = slice_run
    n_cl = n_tr = n_hits = 0
    for sl in out:
        c, tr = sl["clusters"], sl["tracks"]
        nc = len(c["y_fx"])
        crow = c["crow_start"].astype(np.int64)
        assert crow[0] == 0 and crow[-1] == nc and np.all(np.diff(crow) >= 0)
        # clusters of a row in strictly ascending (peak time, peak pad) order
        ur = np.repeat(np.arange(len(crow) - 1), np.diff(crow))
        key = c["ptime"].astype(np.int64) * 512 + c["ppad"]
        same = ur[1:] == ur[:-1]
        assert np.all(np.diff(key)[same] > 0)
        # every kept hit is a cluster owned by its own track, one per row, rows ascending
        hs = tr["hit_start"].astype(np.int64)
        nk = np.diff(hs)
        assert np.all(nk >= 15)
        h = tr["hits"].astype(np.int64)
        owner = np.repeat(np.arange(len(nk)), nk)
        ct = tr["cluster_track"].astype(np.int64)
        assert np.all(ct[h] == owner)
        rows = np.searchsorted(crow, h, side="right") - 1
        same = owner[1:] == owner[:-1]
        assert np.all(np.diff(rows)[same] > 0)
        # each cluster owned by a track is one of that track's hits
        assert np.count_nonzero(ct >= 0) == len(h)
        assert np.all(np.isfinite(tr["par"])) and np.all(np.isfinite(tr["cov"]))
        n_cl += nc
        n_tr += len(tr["tracklet"])
        n_hits += len(tr["hits"])
    assert counts["n_clusters"] == n_cl and counts["n_tracks"] == n_tr
    assert n_cl > 1.5e7 and n_tr > 3e5

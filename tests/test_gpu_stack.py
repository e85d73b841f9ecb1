"""Many chunks in one launch sequence: three time-frame chunks of different
lengths stacked unit by unit (tpcsynth.stack) are reconstructed by one call,
captured once as a HIP graph and replayed; every chunk's part of the batch
equals that chunk reconstructed alone, on every replay.  Units are
independent, so the batch's index offsets are the only difference."""
import numpy as np
import pytest
import torch

import tpcsynth
from paper_2208_07412_amd import tpc

from _parity import run_gpu

pytestmark = pytest.mark.gpu

NROW = tpc.NROW


def _shift(a, off):
    a = np.asarray(a).astype(np.int64)
    return np.where(a >= 0, a + off, a)


def _check_part(bat, alone, u0, c_off, t_off, k_off, h_off):
    """Chunk `alone` equals the batch's unit-rows [u0, u0 + its unit-rows)
    shifted by the given cluster, tracklet, track and hit offsets; returns
    the sizes."""
    bc, ac = bat["clusters"], alone["clusters"]
    nu = len(ac["crow_start"]) - 1  # unit-rows of the chunk
    nc = len(ac["y_fx"])
    crow = bc["crow_start"][u0:u0 + nu + 1].astype(np.int64)
    assert crow[0] == c_off
    assert np.array_equal(crow - c_off, ac["crow_start"].astype(np.int64))
    for k in ("y_fx", "z_fx", "dpad", "dtime", "s2pad", "s2time", "qtot", "qmax", "ppad",
              "ptime", "flags"):
        assert np.array_equal(bc[k][c_off:c_off + nc], ac[k]), k
    for k in ("down", "up", "downc", "upc"):
        assert np.array_equal(bat["links"][k][c_off:c_off + nc], _shift(alone["links"][k], c_off)), k
    at = alone["tracklets"]
    nt = len(at["tl_start"])
    assert np.array_equal(bat["tracklets"]["tl_start"][t_off:t_off + nt].astype(np.int64),
                          at["tl_start"].astype(np.int64) + c_off)
    assert np.array_equal(bat["tracklets"]["tl_len"][t_off:t_off + nt], at["tl_len"])
    btr, atr = bat["tracks"], alone["tracks"]
    nk = len(atr["tracklet"])
    assert np.array_equal(btr["tracklet"][k_off:k_off + nk].astype(np.int64),
                          atr["tracklet"].astype(np.int64) + t_off)
    for k in ("par", "cov", "chi2", "ndf", "row", "flags"):
        assert np.array_equal(btr[k][k_off:k_off + nk], atr[k]), k
    nh = len(atr["hits"])
    assert np.array_equal(btr["hits"][h_off:h_off + nh].astype(np.int64),
                          atr["hits"].astype(np.int64) + c_off)
    assert np.array_equal(btr["hit_start"][k_off:k_off + nk + 1].astype(np.int64),
                          atr["hit_start"].astype(np.int64) + h_off)
    assert np.array_equal(btr["cluster_track"][c_off:c_off + nc],
                          _shift(atr["cluster_track"], k_off))
    return nu, nc, nt, nk, nh


def test_stacked_chunks_in_one_graph_equal_each_alone():
    chunks = [tpcsynth.generate(tpcsynth.config_chunk(404, i, n_coll=n), 4040 + i)
              for i, n in enumerate((3, 6, 2))]
    assert len({e.n_time_bins for e in chunks}) == 3
    alone = [run_gpu(e, moments=False, follow=False) for e in chunks]
    bat_ev = tpcsynth.stack(chunks)
    assert bat_ev.n_units == 3 * 36

    ns = bat_ev.n_samples
    mt = max(ns // 8, 1024)
    s = torch.cuda.Stream()
    reco = tpc.Reco(bat_ev.n_units, bat_ev.n_time_bins, ns, mt, stream=s)
    zs = tpc.to_device_zs(bat_ev.pad, bat_ev.time, bat_ev.adc, bat_ev.row_start, bat_ev.n_units,
                          bat_ev.n_time_bins)
    cl = reco.alloc_clusters(bat_ev.n_units, bat_ev.n_time_bins, ns)
    links = reco.alloc_links(ns)
    tl = reco.alloc_tracklets(mt)
    tr = reco.alloc_tracks(mt, ns, ns)
    with torch.cuda.stream(s):
        reco.process(zs, cl, links, tl, tr)  # first use outside the capture
    reco.sync()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        reco.process(zs, cl, links, tl, tr)
    torch.cuda.synchronize()
    try:
        for rep in range(3):
            tr["par"].fill_(0)  # a replay must rewrite every output
            cl["y_fx"].fill_(0)
            links["up"].fill_(-7)
            torch.cuda.synchronize()
            with torch.cuda.stream(s):
                g.replay()
            counts = reco.sync()
            n = counts["n_clusters"]
            bat = dict(clusters=tpc.clusters_to_host(cl, bat_ev.n_units),
                       links=tpc.links_to_host(links, n), tracklets=tpc.tracklets_to_host(tl),
                       tracks=tpc.tracks_to_host(tr, n))
            u0 = c_off = t_off = k_off = h_off = 0
            for a in alone:
                nu, nc, nt, nk, nh = _check_part(bat, a, u0, c_off, t_off, k_off, h_off)
                u0, c_off, t_off, k_off, h_off = (u0 + nu, c_off + nc, t_off + nt, k_off + nk,
                                                  h_off + nh)
            assert c_off == n and k_off == counts["n_tracks"]
            print(f"replay {rep}: {n} clusters, {counts['n_tracks']} tracks in "
                  f"{len(alone)} stacked chunks: each equals its own call")
    finally:
        del g
        reco.close()

"""Batched form over unit slices on concurrent streams: the slices' outputs,
put back together with their index offsets, are the outputs of one call over
the whole frame, eagerly and on every replay of a captured graph."""
import numpy as np
import pytest
import torch

import tpcsynth
from paper_2208_07412_amd import pipeline, tpc

from _parity import run_gpu

pytestmark = pytest.mark.gpu

NROW = tpc.NROW


@pytest.fixture(scope="module")
def frame():
    ev = tpcsynth.generate(tpcsynth.config_chunk(404, 3, n_coll=6), 4043)
    return ev, run_gpu(ev, moments=False, follow=False)


def _slice_host(sl):
    n = int(sl.cl["n_clusters"].item())
    nu = sl.u1 - sl.u0
    return dict(clusters=tpc.clusters_to_host(sl.cl, nu), links=tpc.links_to_host(sl.links, n),
                tracklets=tpc.tracklets_to_host(sl.tl), tracks=tpc.tracks_to_host(sl.tr, n))


def _shift(a, off):
    a = np.asarray(a).astype(np.int64)
    return np.where(a >= 0, a + off, a)


def _check(p, full):
    fc, ft, ftr = full["clusters"], full["tracklets"], full["tracks"]
    c_off = t_off = k_off = h_off = 0
    for sl in p.slices:
        g = _slice_host(sl)
        gc = g["clusters"]
        nc = len(gc["y_fx"])
        crow = fc["crow_start"][sl.u0 * NROW:sl.u1 * NROW + 1].astype(np.int64)
        assert crow[0] == c_off
        assert np.array_equal(gc["crow_start"].astype(np.int64), crow - c_off)
        for k in ("y_fx", "z_fx", "dpad", "dtime", "qtot", "qmax", "ppad", "ptime", "flags"):
            assert np.array_equal(gc[k], fc[k][c_off:c_off + nc]), k
        for k in ("down", "up", "downc", "upc"):
            assert np.array_equal(_shift(g["links"][k], c_off),
                                  full["links"][k][c_off:c_off + nc]), k
        ts = g["tracklets"]["tl_start"].astype(np.int64) + c_off
        nt = len(ts)
        assert np.array_equal(ts, ft["tl_start"][t_off:t_off + nt])
        gt = g["tracks"]
        nk = len(gt["tracklet"])
        assert np.array_equal(gt["tracklet"].astype(np.int64) + t_off,
                              ftr["tracklet"][k_off:k_off + nk])
        for k in ("par", "cov", "chi2", "ndf", "row", "flags"):
            assert np.array_equal(gt[k], ftr[k][k_off:k_off + nk]), k
        nh = len(gt["hits"])
        assert np.array_equal(gt["hits"].astype(np.int64) + c_off,
                              ftr["hits"][h_off:h_off + nh])
        assert np.array_equal(gt["hit_start"].astype(np.int64) + h_off,
                              ftr["hit_start"][k_off:k_off + nk + 1])
        assert np.array_equal(_shift(gt["cluster_track"], k_off),
                              ftr["cluster_track"][c_off:c_off + nc])
        c_off += nc
        t_off += nt
        k_off += nk
        h_off += nh
    assert c_off == len(fc["y_fx"]) and k_off == len(ftr["tracklet"])


@pytest.mark.parametrize("parts,stagger", [(1, "cluster"), (3, "cluster"), (4, "none"),
                                           (2, "tracklets")])
def test_slices_equal_one_call(frame, parts, stagger):
    ev, full = frame
    zs = tpc.to_device_zs(ev.pad, ev.time, ev.adc, ev.row_start, ev.n_units, ev.n_time_bins)
    p = pipeline.Pipeline(zs, parts, stagger=stagger)
    assert p.n_parts == parts and p.bounds[0] == 0 and p.bounds[-1] == ev.n_units
    p.enqueue()
    torch.cuda.synchronize()
    c = p.sync()
    assert c["n_clusters"] == full["counts"]["n_clusters"]
    assert c["n_tracks"] == full["counts"]["n_tracks"]
    _check(p, full)
    p.close()


def test_graph_replays(frame):
    ev, full = frame
    zs = tpc.to_device_zs(ev.pad, ev.time, ev.adc, ev.row_start, ev.n_units, ev.n_time_bins)
    p = pipeline.Pipeline(zs, 2)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        p.enqueue()  # first use outside the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        p.enqueue()
    torch.cuda.synchronize()
    for _ in range(3):
        for sl in p.slices:  # clear what a replay must rewrite
            sl.tr["par"].fill_(0)
            sl.cl["y_fx"].fill_(0)
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            g.replay()
        torch.cuda.synchronize()
        assert p.sync()["n_tracks"] == full["counts"]["n_tracks"]
        _check(p, full)
    del g
    p.close()

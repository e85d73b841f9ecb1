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
from _units import unit_event, unit_view

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


@pytest.mark.parametrize("u", UNITS)
def test_sampled_unit_equals_oracle(slice_run, u):
    ev, counts, out = slice_run
    sl = next(s for s in out if s["u0"] <= u < s["u1"])
    g = unit_view(sl, u)
    o = run_oracle(unit_event(ev, u))
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

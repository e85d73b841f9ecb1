"""Tracking efficiency and fake rate of the GPU tracks against generator
truth, beside the FP64 oracle's on the same input: the two must agree within
0.2 percentage points (the acceptance rule for physics performance).

Truth: each cluster carries the label of the deposit that dominates its peak
sample; a segment (track, sector, leg) is findable with at least 20 labelled
clusters; a track is good when at least 90% of its clusters carry its
majority segment, otherwise it is a fake.  Both sides are scored with the
same labels (clusters are bit-exact, so the labels are shared).  Inputs: one
central collision, and four sectors of the 2 ms slice (pile-up of about five
collisions per drift window)."""
import numpy as np
import pytest

import tpcsynth
from tpcsynth import truth

from _parity import run_gpu, run_oracle

pytestmark = pytest.mark.gpu

TOL = 0.002  # 0.2 percentage points


def _score(ev):
    g = run_gpu(ev)
    o = run_oracle(ev)
    gc, oc = g["clusters"], o["clusters"]
    assert np.array_equal(gc["y_fx"], oc["y_fx"]) and np.array_equal(gc["z_fx"], oc["z_fx"])
    labels = truth.cluster_labels(ev.deposits, oc, ev.n_units)
    gt = g["tracks"]
    hs = gt["hit_start"].astype(np.int64)
    g_hits = [gt["hits"][hs[j]:hs[j + 1]].astype(np.int64) for j in range(len(gt["tracklet"]))]
    fit = o["fit"]
    owner = fit["cluster_owner"]
    o_hits = []
    for t in np.nonzero(fit["kept"])[0]:
        h = fit["hits"][t]
        h = h[h >= 0]
        o_hits.append(h[owner[h] == t].astype(np.int64))
    pg = truth.performance(ev.deposits, ev.tracks, oc, ev.n_units, g_hits, labels)
    po = truth.performance(ev.deposits, ev.tracks, oc, ev.n_units, o_hits, labels)
    return pg, po


def _check(pg, po, name):
    print(f"{name}: findable {po['findable']}; "
          f"efficiency gpu {pg['efficiency']:.5f} oracle {po['efficiency']:.5f}; "
          f"fake gpu {pg['fake_rate']:.5f} oracle {po['fake_rate']:.5f}; "
          f"clone gpu {pg['clone_rate']:.5f} oracle {po['clone_rate']:.5f}; "
          f"tracks gpu {pg['n_tracks']} oracle {po['n_tracks']}")
    print(f"  split gpu {pg['split']}\n  split oracle {po['split']}")
    assert po["findable"] > 1000
    assert abs(pg["efficiency"] - po["efficiency"]) <= TOL
    assert abs(pg["fake_rate"] - po["fake_rate"]) <= TOL
    for k in po["split"]:  # every split bin present on both sides
        assert k in pg["split"], k
    # sanity of the reading, not a parity rule: most primaries above 0.2 GeV/c found
    assert po["split"].get("0.2<pt<1", 1.0) > 0.9


def test_efficiency_central_collision():
    ev = tpcsynth.generate(tpcsynth.config_c2(), 202)
    pg, po = _score(ev)
    _check(pg, po, "central collision")


def test_efficiency_slice_sectors():
    full = tpcsynth.generate(tpcsynth.config_c3(303, 100), 303)
    ev = tpcsynth.select_units(full, [0, 12, 24, 35])
    del full
    pg, po = _score(ev)
    _check(pg, po, "2 ms slice, sectors 0, 12, 24, 35")

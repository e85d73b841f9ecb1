"""GPU decoding of raw zero-suppressed pages against the oracle's decoder
(integer work: bit-exact), and the clusterizer fed from decoded pages
against the oracle's clusters of the original samples.

Cases: the hand-assembled example (tests/golden), generated events at the
sizes of one sector, one central collision and the full 2 ms slice (there
the decoded arrays are compared with the packed samples as a whole), a page
filled to its end, an empty page, no pages at all, every malformed field the
format forbids (always checked, or only in validate mode), and an output
capacity that is too small."""
import numpy as np
import pytest
import torch

import oracle
import tpcsynth
from paper_2208_07412_amd import tpc

from _parity import compare_clusters
from _zspages import load_example, page

pytestmark = pytest.mark.gpu


def _decode(pages, n_units, T, capacity=None, validate=0, reco=None):
    pages = np.asarray(pages, np.uint32).reshape(-1, 2048)
    cap = capacity if capacity is not None else max(pages.shape[0] * 6600, 1)
    own = reco is None
    if own:
        reco = tpc.Reco(n_units, T, 1 << 16, 1024, param_overrides=dict(validate=validate),
                        max_samples=max(cap, 1))
    soa = reco.alloc_zs_soa(n_units, T, cap)
    dev = tpc.pages_to_device(pages) if pages.shape[0] else torch.zeros(1, dtype=torch.int32,
                                                                        device="cuda")
    reco.decode_zs_pages(dev, soa, n_pages=pages.shape[0])
    c = reco.sync(raise_on_error=False)
    out = tpc.zs_soa_to_host(soa) if c["status"] == 0 else None
    if own:
        reco.close()
    return c, out, soa


def test_hand_assembled_example():
    pages, nu, T, exp = load_example()
    for v in (0, 1):
        c, d, _ = _decode(pages, nu, T, validate=v)
        assert c["status"] == 0 and d["n_samples"] == 6
        for k in ("pad", "time", "adc", "row_start"):
            assert np.array_equal(d[k], exp[k]), k


@pytest.mark.parametrize("which", ["c1", "c2"])
def test_generated_pages_and_clusters(which):
    cfg, seed = {"c1": (tpcsynth.config_c1(), 101), "c2": (tpcsynth.config_c2(), 202)}[which]
    ev = tpcsynth.generate(cfg, seed)
    pages = tpcsynth.zs_pages(ev)
    od = oracle.decode_zs_pages(pages, ev.n_units, ev.n_time_bins, validate=True)
    assert od["status"] == 0
    ns = ev.n_samples
    reco = tpc.Reco(ev.n_units, ev.n_time_bins, ns, max(ns // 8, 1024),
                    param_overrides=dict(validate=1), max_samples=ns + 64)
    try:
        soa = reco.alloc_zs_soa(ev.n_units, ev.n_time_bins, ns + 64)
        reco.decode_zs_pages(tpc.pages_to_device(pages), soa)
        cl = reco.alloc_clusters(ev.n_units, ev.n_time_bins, ns, n_samples=ns + 64, moments=True)
        reco.cluster(tpc.zs_from_soa(soa), cl)  # same stream: after the decoder
        c = reco.sync()
        d = tpc.zs_soa_to_host(soa)
        assert d["n_samples"] == ns
        for k in ("pad", "time", "adc", "row_start"):
            assert np.array_equal(d[k], od[k]), k
        o = oracle.cluster(ev.pad, ev.time, ev.adc, ev.row_start, ev.n_units, ev.n_time_bins,
                           n_threads=8)
        assert c["n_clusters"] == len(o["y_fx"])
        compare_clusters(tpc.clusters_to_host(cl, ev.n_units), o)
    finally:
        reco.close()


def test_full_slice_pages():
    ev = tpcsynth.generate(tpcsynth.config_c3(303, 100), 303)
    pages = tpcsynth.zs_pages(ev)
    print(f"slice: {ev.n_samples} samples in {pages.shape[0]} pages "
          f"({pages.nbytes / ev.n_samples:.2f} B/sample)", flush=True)
    ns = ev.n_samples
    reco = tpc.Reco(ev.n_units, ev.n_time_bins, 1 << 16, 1024, max_samples=ns)
    try:
        soa = reco.alloc_zs_soa(ev.n_units, ev.n_time_bins, ns)
        dev = tpc.pages_to_device(pages)
        del pages
        for _ in range(2):  # the second call overwrites the first's outputs alike
            reco.decode_zs_pages(dev, soa)
            c = reco.sync()
        d = tpc.zs_soa_to_host(soa)
        assert d["n_samples"] == ns
        for k in ("pad", "time", "adc", "row_start"):
            assert np.array_equal(d[k], getattr(ev, k)), k
    finally:
        reco.close()


def test_full_page_empty_page_and_no_pages():
    rng = np.random.default_rng(3)
    runs = [(t, 0, rng.integers(1, 1024, 128).tolist()) for t in range(49)]
    empty = np.zeros(2048, np.uint32)
    empty[0] = 0x5A53 | (1 << 16)
    empty[1] = 151 << 16
    pages = np.stack([page(0, 151, runs), empty])
    od = oracle.decode_zs_pages(pages, 1, 64, validate=True)
    c, d, _ = _decode(pages, 1, 64, validate=1)
    assert c["status"] == 0 and d["n_samples"] == 6272
    for k in ("pad", "time", "adc", "row_start"):
        assert np.array_equal(d[k], od[k]), k
    c, d, soa = _decode(np.zeros((0, 2048), np.uint32), 2, 64, capacity=16)
    assert c["status"] == 0 and d["n_samples"] == 0 and not d["row_start"].any()


def test_malformed_pages_reported():
    good = page(1, 4, [(7, 3, [1, 2, 3])])
    reco = tpc.Reco(2, 16, 1 << 12, 1024, max_samples=1 << 14)
    reco_v = tpc.Reco(2, 16, 1 << 12, 1024, param_overrides=dict(validate=1),
                      max_samples=1 << 14)
    always = [[page(1, 4, [(7, 3, [1])], header={0: 0x5A54 | 1 << 16})],
              [page(2, 4, [(7, 3, [1])])],
              [page(1, 152, [(7, 3, [1])])],
              [page(1, 4, [(7, 66, [1, 2, 3])])],
              [page(1, 4, [(16, 3, [1])])],
              [page(1, 4, [(7, 3, [1, 2])], header={2: 1 | 3 << 16})],
              [page(1, 4, [(7, 3, [1])], header={3: 1})],
              [page(1, 4, [], header={2: 1})],
              [page(1, 5, [(7, 3, [1])]), page(1, 4, [(7, 3, [1])])],
              [page(1, 4, [(7, 3, [1])], header={2: 1 | 6540 << 16})]]
    validate_only = [[page(1, 4, [(7, 3, [1, 0, 3])])],
                     [page(1, 4, [(7, 3, [1]), (6, 9, [1])])],
                     [page(1, 4, [(7, 3, [1, 1]), (7, 4, [1])])],
                     [page(1, 4, [(7, 3, [1])]), page(1, 4, [(7, 3, [1])])]]
    try:
        c, d, _ = _decode([good], 2, 16, reco=reco_v)
        assert c["status"] == 0 and d["n_samples"] == 3
        for i, pages in enumerate(always):
            assert oracle.decode_zs_pages(np.stack(pages), 2, 16)["status"] == -3, i
            assert _decode(pages, 2, 16, reco=reco)[0]["status"] == -3, i
        for i, pages in enumerate(validate_only):
            assert _decode(pages, 2, 16, reco=reco)[0]["status"] == 0, i
            assert _decode(pages, 2, 16, reco=reco_v)[0]["status"] == -3, i
        # the context works normally after the reported errors
        c, d, _ = _decode([good], 2, 16, reco=reco)
        assert c["status"] == 0 and d["n_samples"] == 3
    finally:
        reco.close()
        reco_v.close()


def test_misaligned_pages_rejected():
    # pages are loaded in 16-byte words: a pointer off that alignment is an
    # argument error, raised before anything is launched
    reco = tpc.Reco(1, 500, 4096, 64)
    words = torch.zeros(2 * tpc.ZS_PAGE_WORDS + 1, dtype=torch.int32, device="cuda")
    soa = reco.alloc_zs_soa(1, 500, 4096)
    with pytest.raises(tpc.TpcError):
        reco.decode_zs_pages(words[1:], soa, n_pages=2)
    reco.close()


def test_capacity_overflow_reported():
    pages, nu, T, exp = load_example()
    c, _, _ = _decode(pages, nu, T, capacity=5)
    assert c["status"] == -2 and c["required"] == 6
    c, d, _ = _decode(pages, nu, T, capacity=6)
    assert c["status"] == 0 and np.array_equal(d["adc"], exp["adc"])

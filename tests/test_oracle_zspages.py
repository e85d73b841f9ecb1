"""Pins of the oracle's raw ZS page decoder.

The paper places zero suppression on the readout FPGA (section "Hardware and
data flow") and fixes no format; the library defines its own (stated with
tpc_decode_zs_pages).  The decoder is pinned by
* a hand-assembled example whose every bit field is worked out in the
  fixture's comments (tests/golden/zs_pages_example.txt), including a 10-bit
  field that straddles two words and a row continued on a second page;
* round trips through the generator's page packer (separate code, written
  from the format statement) on generated events: decoding returns exactly
  the samples that were packed;
* the error rules: every malformed field the format forbids is rejected, and
  the validate-only rules only in validate mode.
"""
import numpy as np
import pytest

import oracle
import tpcsynth

from _zspages import load_example, page


def test_hand_assembled_example():
    pages, nu, T, exp = load_example()
    d = oracle.decode_zs_pages(pages, nu, T, validate=True)
    assert d["status"] == 0 and d["n_samples"] == len(exp["pad"])
    for k in ("pad", "time", "adc", "row_start"):
        assert np.array_equal(d[k], exp[k]), k


@pytest.mark.parametrize("which", ["c1", "small36", "pileup"])
def test_round_trip_through_generator_packer(which):
    cfg, seed = {"c1": (tpcsynth.config_c1(), 101),
                 "small36": (tpcsynth.config_small(400, sector_mode=0, n_sec=80), 11),
                 "pileup": (tpcsynth.config_chunk(404, 1, n_coll=25), 4041)}[which]
    ev = tpcsynth.generate(cfg, seed)
    pages = tpcsynth.zs_pages(ev)
    # some rows span several pages at this occupancy
    if which == "pileup":
        ur = (pages[:, 1] & 0xFFFF).astype(np.int64) * 152 + ((pages[:, 1] >> 16) & 0xFF)
        assert (np.diff(ur) == 0).any()
    d = oracle.decode_zs_pages(pages, ev.n_units, ev.n_time_bins, validate=True)
    assert d["status"] == 0
    for k in ("pad", "time", "adc", "row_start"):
        assert np.array_equal(d[k], getattr(ev, k)), k


def test_full_page_and_empty_page():
    # 49 runs of 128 pads: 4 + 49 + 1960 words, close to the page's 2048
    rng = np.random.default_rng(3)
    runs = [(t, 0, rng.integers(1, 1024, 128).tolist()) for t in range(49)]
    pg = page(0, 151, runs)
    assert 2000 < 4 + 49 + (10 * 6272 + 31) // 32 <= 2048
    empty = np.zeros(2048, np.uint32)
    empty[0] = 0x5A53 | (1 << 16)
    empty[1] = 0 | (152 - 1) << 16  # unit 0, row 151, no runs, no samples
    d = oracle.decode_zs_pages(np.stack([pg, empty]), 1, 64, validate=True)
    assert d["status"] == 0 and d["n_samples"] == 6272
    exp_adc = np.concatenate([np.array(a) for _, _, a in runs])
    assert np.array_equal(d["adc"], exp_adc)
    assert np.array_equal(d["pad"], np.tile(np.arange(128), 49))
    assert np.array_equal(d["time"], np.repeat(np.arange(49), 128))
    assert d["row_start"][151] == 0 and d["row_start"][152] == 6272


def test_no_pages():
    d = oracle.decode_zs_pages(np.zeros((0, 2048), np.uint32), 3, 100)
    assert d["status"] == 0 and d["n_samples"] == 0 and not d["row_start"].any()


def _bad(pages, validate=False, n_units=2, T=16):
    return oracle.decode_zs_pages(np.stack(pages), n_units, T, validate=validate)["status"]


def test_malformed_pages_rejected():
    good = page(1, 4, [(7, 3, [1, 2, 3])])
    assert _bad([good]) == 0
    assert _bad([page(1, 4, [(7, 3, [1])], header={0: 0x5A54 | 1 << 16})]) == -3  # magic
    assert _bad([page(1, 4, [(7, 3, [1])], header={0: 0x5A53 | 2 << 16})]) == -3  # version
    assert _bad([page(2, 4, [(7, 3, [1])])]) == -3                       # unit beyond frame
    assert _bad([page(1, 152, [(7, 3, [1])])]) == -3                     # row beyond 151
    assert _bad([page(1, 4, [(7, 66, [1, 2, 3])])]) == -3                # pads 66-68 of 68
    assert _bad([page(1, 4, [(7, 65, [1, 2, 3])])]) == 0                 # pads 65-67 fit
    assert _bad([page(1, 4, [(16, 3, [1])])]) == -3                      # time beyond 16 bins
    assert _bad([page(1, 4, [(7, 3, [1, 2])], header={2: 1 | 3 << 16})]) == -3  # run sum
    assert _bad([page(1, 4, [(7, 3, [1])], header={3: 1})]) == -3        # reserved word
    assert _bad([page(1, 4, [(7, 3, [1])], header={2: 0 | 1 << 16})]) == -3  # samples, no runs
    assert _bad([page(1, 4, [], header={2: 1})]) == -3                   # a run, no samples
    assert _bad([page(1, 5, [(7, 3, [1])]), page(1, 4, [(7, 3, [1])])]) == -3  # row order
    # a page claiming more fields than it holds
    assert _bad([page(1, 4, [(7, 3, [1])], header={2: 1 | 6540 << 16})]) == -3


def test_validate_only_rules():
    zero = page(1, 4, [(7, 3, [1, 0, 3])])
    back = page(1, 4, [(7, 3, [1]), (6, 9, [1])])         # time steps back
    overlap = page(1, 4, [(7, 3, [1, 1]), (7, 4, [1])])   # pad 4 twice
    across = [page(1, 4, [(7, 3, [1])]), page(1, 4, [(7, 3, [1])])]  # continuation repeats
    for pages in ([zero], [back], [overlap], across):
        assert _bad(pages) == 0
        assert _bad(pages, validate=True) == -3


def test_capacity_overflow():
    pages, nu, T, exp = load_example()
    d = oracle.decode_zs_pages(pages, nu, T, capacity=5)
    assert d["status"] == -2 and d["n_samples"] == 6
    assert np.array_equal(d["pad"], exp["pad"][:5])

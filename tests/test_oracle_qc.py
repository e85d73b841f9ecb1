"""Pins of the oracle's quality-control histograms (plain definition, numpy
bincount) against brute-force counting loops and a hand-counted fixture."""
import numpy as np

import oracle

NROW = 152


def _brute(qtot, qmax, ct, hs):
    h = [0] * oracle.QC_BINS
    for q in qtot:
        h[oracle.QC_QTOT + min(int(q) // 8, 255)] += 1
    for q in qmax:
        h[oracle.QC_QMAX + min(int(q) // 4, 255)] += 1
    for j in range(len(hs) - 1):
        h[oracle.QC_NHITS + min(int(hs[j + 1]) - int(hs[j]), NROW)] += 1
    for t in ct:
        h[oracle.QC_ATTACH + (1 if t >= 0 else 0)] += 1
    return np.array(h, np.int64)


def test_hand_counted():
    # qtot bins 0, 1, 255, 255; qmax bins 0, 1, 255, 0; tracks of 5, 0, 152
    # hits; two clusters on a track, two off
    h = oracle.qc_histograms([0, 8, 2047, 40000], [3, 4, 1023, 0], [-1, 2, 0, -1],
                             [0, 5, 5, 157])
    exp = np.zeros(oracle.QC_BINS, np.int64)
    exp[[0, 1]] = 1
    exp[255] = 2
    exp[256] = 2
    exp[257] = 1
    exp[511] = 1
    exp[512 + 0] = exp[512 + 5] = exp[512 + 152] = 1
    exp[665] = exp[666] = 2
    assert np.array_equal(h, exp)


def test_against_brute_force():
    rng = np.random.default_rng(7)
    for n, m in ((0, 0), (1, 1), (37, 5), (500, 60)):
        qtot = rng.integers(0, 1 << 15, n)
        qmax = rng.integers(0, 1024, n)
        ct = rng.integers(-1, 3, n)
        hs = np.concatenate([[0], np.cumsum(rng.integers(0, 160, m))])
        assert np.array_equal(oracle.qc_histograms(qtot, qmax, ct, hs), _brute(qtot, qmax, ct, hs))


def test_totals():
    rng = np.random.default_rng(3)
    qtot = rng.integers(0, 5000, 300)
    qmax = rng.integers(0, 1024, 300)
    ct = rng.integers(-1, 10, 300)
    hs = np.concatenate([[0], np.cumsum(rng.integers(3, 153, 40))])
    h = oracle.qc_histograms(qtot, qmax, ct, hs)
    assert h[0:256].sum() == h[256:512].sum() == h[665:667].sum() == 300
    assert h[512:665].sum() == 40

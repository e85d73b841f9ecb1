"""Pins of the oracle clusterizer and its fixed-point positions.

* an independent dense-grid brute force of the clusterizer definition on tiny
  random grids (peaks = strict key maxima with ADC >= threshold; each sample
  joins the peak it reaches in at most two uphill steps; integer moments);
* hand-worked special cases (lone sample, symmetric 3x3, plateau, two-sample
  centroid, saturation and edge flags);
* invariants (charge conservation, one cluster per sample);
* y_fx / z_fx against exact rational rounding.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle

NPADS, XFX, PFX = oracle.geometry()


def make_input(samples_per_ur, n_units=1):
    """samples_per_ur: dict (unit,row) -> list of (time, pad, adc)."""
    pad, time, adc = [], [], []
    rs = [0]
    for u in range(n_units):
        for r in range(152):
            lst = sorted(samples_per_ur.get((u, r), []))
            for t, p, a in lst:
                time.append(t)
                pad.append(p)
                adc.append(a)
            rs.append(len(pad))
    return (np.array(pad, np.uint16), np.array(time, np.uint16), np.array(adc, np.uint16),
            np.array(rs, np.uint32))


def brute_clusters(grid, qmin):
    """Dense-grid brute force on one row.  grid[t][p] = adc (0 = absent).
    Returns a list of dicts in (time, pad) peak order and the owner map."""
    T, P = grid.shape
    present = grid > 0

    def key(t, p):
        return (int(grid[t, p]), t, p)

    up = {}
    for t in range(T):
        for p in range(P):
            if not present[t, p]:
                continue
            best = (t, p)
            for dt in (-1, 0, 1):
                for dp in (-1, 0, 1):
                    tt, pp = t + dt, p + dp
                    if 0 <= tt < T and 0 <= pp < P and present[tt, pp] and key(tt, pp) > key(*best):
                        best = (tt, pp)
            up[(t, p)] = best
    peaks = {s for s, u in up.items() if u == s and grid[s] >= qmin}
    owner = {}
    for s, u in up.items():
        if u in peaks:
            owner[s] = u
        elif up[u] in peaks:
            owner[s] = up[u]
    out = []
    for (t, p) in sorted(peaks):
        mem = [s for s, o in owner.items() if o == (t, p)]
        q = sum(int(grid[s]) for s in mem)
        sp = sum(int(grid[s]) * (s[1] - p) for s in mem)
        st = sum(int(grid[s]) * (s[0] - t) for s in mem)
        spp = sum(int(grid[s]) * (s[1] - p) ** 2 for s in mem)
        stt = sum(int(grid[s]) * (s[0] - t) ** 2 for s in mem)
        sat = any(int(grid[s]) >= 1023 for s in mem)
        out.append(dict(ptime=t, ppad=p, qtot=q, qmax=int(grid[t, p]), sp=sp, st=st, spp=spp,
                        stt=stt, nsamp=len(mem), sat=sat))
    return out, owner


def exact_fx(ppad, ptime, q, sp, st, r):
    n = int(NPADS[r])
    y = Fraction((2 * (ppad * q + sp) - (n - 1) * q) * int(PFX[r]), 2 * q)
    z = Fraction(65536 * (ptime * q + st), 2 * q)
    return math.floor(y + Fraction(1, 2)), math.floor(z + Fraction(1, 2))


@pytest.mark.parametrize("seed", range(12))
def test_clusterizer_matches_dense_bruteforce(seed):
    rng = np.random.default_rng(seed)
    rows = [0, 5, 151] if seed % 2 else [3, 77]
    T = 24
    samples = {}
    grids = {}
    for r in rows:
        P = int(NPADS[r])
        g = np.zeros((T, P), np.int64)
        # a few Gaussian blobs plus sparse noise; some saturated values
        for _ in range(rng.integers(1, 6)):
            mt, mp = rng.uniform(0, T), rng.uniform(0, min(P, 12))
            amp = rng.choice([20.0, 150.0, 3000.0])
            for t in range(T):
                for p in range(min(P, 14)):
                    g[t, p] += int(amp * math.exp(-((t - mt) ** 2 + (p - mp) ** 2) / 1.5))
        g += (rng.random(g.shape) < 0.05) * rng.integers(3, 9, g.shape)
        g = np.minimum(g, 1023)
        g[g < 3] = 0
        grids[r] = g
        samples[(0, r)] = [(t, p, int(g[t, p])) for t in range(T) for p in range(P) if g[t, p]]
    pad, time, adc, rs = make_input(samples)
    res = oracle.cluster(pad, time, adc, rs, 1, T, labels=True)
    k = 0
    for r in range(152):
        a, b = int(res["crow_start"][r]), int(res["crow_start"][r + 1])
        if r not in grids:
            assert a == b
            continue
        exp, owner = brute_clusters(grids[r], 5)
        assert b - a == len(exp)
        for j, e in enumerate(exp):
            i = a + j
            for f in ("ptime", "ppad", "qtot", "qmax", "sp", "st", "spp", "stt", "nsamp"):
                assert int(res[f][i]) == e[f], (r, j, f)
            assert bool(res["flags"][i] & 2) == e["sat"]
            edge = e["ppad"] <= 1 or e["ppad"] >= NPADS[r] - 2
            assert bool(res["flags"][i] & 1) == edge
            yfx, zfx = exact_fx(e["ppad"], e["ptime"], e["qtot"], e["sp"], e["st"], r)
            assert res["y_fx"][i] == yfx and res["z_fx"][i] == zfx
            assert abs(res["pad"][i] - (e["ppad"] + e["sp"] / e["qtot"])) < 1e-12
        # labels: each sample -> its cluster
        s0 = int(rs[r])
        peak_index = {(e["ptime"], e["ppad"]): a + j for j, e in enumerate(exp)}
        for s in range(int(rs[r]), int(rs[r + 1])):
            key = (int(time[s]), int(pad[s]))
            want = peak_index[owner[key]] if key in owner else -1
            assert res["sample_label"][s] == want
        k += 1
    assert k == len(rows)


def _single_row(sample_list, row=10, T=20, qmin=None):
    pad, time, adc, rs = make_input({(0, row): sample_list})
    params = oracle.default_params()
    if qmin is not None:
        params["qmax_min"] = qmin
    return oracle.cluster(pad, time, adc, rs, 1, T, params=params, labels=True)


def test_lone_sample_centroid_exact():
    res = _single_row([(7, 30, 50)])
    assert len(res["qtot"]) == 1
    assert res["pad"][0] == 30.0 and res["time"][0] == 7.0
    assert res["s2pad"][0] == 0.0 and res["s2time"][0] == 0.0
    assert res["qtot"][0] == 50 and res["nsamp"][0] == 1


def test_lone_sample_below_threshold_is_no_cluster():
    res = _single_row([(7, 30, 4)])
    assert len(res["qtot"]) == 0
    assert res["sample_label"][0] == -1


def test_symmetric_3x3_centroid_at_centre():
    s = [(t, p, 10) for t in (4, 6) for p in (20, 22)]
    s += [(5, 20, 30), (5, 22, 30), (4, 21, 30), (6, 21, 30), (5, 21, 100)]
    res = _single_row(s)
    assert len(res["qtot"]) == 1
    assert res["pad"][0] == 21.0 and res["time"][0] == 5.0
    assert res["qtot"][0] == 4 * 10 + 4 * 30 + 100
    # second moments: Spp = 2*10*2 (corners) + 2*30 (pad neighbours) = 100
    assert res["spp"][0] == 100 and res["stt"][0] == 100


def test_two_sample_centroid():
    res = _single_row([(3, 40, 10), (3, 41, 5)])
    assert len(res["qtot"]) == 1
    assert res["ppad"][0] == 40
    assert abs(res["pad"][0] - (40 + 5 / 15)) < 1e-15
    assert abs(res["s2pad"][0] - (5 / 15 - (5 / 15) ** 2)) < 1e-15


def test_plateau_single_peak_at_max_time_then_pad():
    # equal ADC on a 2x2 block: the peak is the larger time, then larger pad
    s = [(t, p, 40) for t in (8, 9) for p in (15, 16)]
    res = _single_row(s)
    assert len(res["qtot"]) == 1
    assert (res["ptime"][0], res["ppad"][0]) == (9, 16)
    assert res["qtot"][0] == 160


def test_two_step_assignment_bounds_cluster():
    # a monotone ramp along pads: samples 3 steps downhill are not assigned
    s = [(5, 10 + k, 100 - 10 * k) for k in range(6)]
    res = _single_row(s)
    assert len(res["qtot"]) == 1 and res["ppad"][0] == 10
    assert res["nsamp"][0] == 3
    assert list(res["sample_label"]) == [0, 0, 0, -1, -1, -1]


def test_saturation_and_edge_flags():
    res = _single_row([(5, 0, 1023), (5, 1, 500)], row=0)
    assert res["flags"][0] == 3  # EDGE | SAT


def test_charge_conservation_invariant():
    import tpcsynth

    ev = tpcsynth.generate(tpcsynth.config_small(30), 9)
    res = oracle.cluster(ev.pad, ev.time, ev.adc, ev.row_start, ev.n_units, ev.n_time_bins,
                         labels=True)
    lab = res["sample_label"]
    assigned = ev.adc[lab >= 0].astype(np.int64).sum()
    assert int(res["qtot"].astype(np.int64).sum()) == int(assigned)
    # per cluster: charge of its samples equals Q
    q = np.bincount(lab[lab >= 0], weights=ev.adc[lab >= 0].astype(np.float64),
                    minlength=len(res["qtot"]))
    assert np.array_equal(q.astype(np.int64), res["qtot"].astype(np.int64))
    # peaks are strict key maxima: every cluster's qmax is the max ADC of its samples
    mx = np.zeros(len(res["qtot"]), np.int64)
    np.maximum.at(mx, lab[lab >= 0], ev.adc[lab >= 0].astype(np.int64))
    assert np.array_equal(mx, res["qmax"].astype(np.int64))


def test_unsorted_input_rejected():
    pad = np.array([5, 4], np.uint16)
    time = np.array([3, 3], np.uint16)
    adc = np.array([10, 10], np.uint16)
    rs = np.zeros(153, np.uint32)
    rs[1:] = 2
    with pytest.raises(ValueError):
        oracle.cluster(pad, time, adc, rs, 1, 10)


@pytest.mark.parametrize("bad_adc", [0, 1024, 4095])
def test_adc_outside_ten_bits_rejected(bad_adc):
    # a stored zero-suppressed sample has a 10-bit ADC above zero
    pad = np.array([4, 5], np.uint16)
    time = np.array([3, 3], np.uint16)
    rs = np.zeros(153, np.uint32)
    rs[1:] = 2
    ok = oracle.cluster(pad, time, np.array([10, 1023], np.uint16), rs, 1, 10)
    assert ok["qtot"].tolist() == [1033]
    with pytest.raises(ValueError):
        oracle.cluster(pad, time, np.array([10, bad_adc], np.uint16), rs, 1, 10)


def test_empty_input():
    rs = np.zeros(153, np.uint32)
    e = np.zeros(0, np.uint16)
    res = oracle.cluster(e, e, e, rs, 1, 10)
    assert len(res["qtot"]) == 0 and res["crow_start"][-1] == 0

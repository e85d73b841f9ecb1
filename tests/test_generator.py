"""Pins of the synthetic generator against textbook physics and closed forms.

* helix / row-plane crossings vs an RK4 integration of the Lorentz force;
* pT power law and Landau charge vs their CDFs (KS test);
* zero-suppression and ordering contract of the generated samples;
* determinism under a seed.
"""
import math

import numpy as np
import pytest
import scipy.stats as st

import tpcsynth

B = tpcsynth.BZ_B


def _lorentz_rk4(v0, d0, curv, tgl, s_end, h=0.02):
    """Integrate dr/ds = t, dt/ds = C * (t x z_hat) projected on the transverse
    plane (dz/ds = tgl), by classical RK4 in the 2-D arc length s."""

    def f(state):
        x, y, z, tx, ty = state
        return np.array([tx, ty, tgl, curv * -ty, curv * tx])

    state = np.array([v0[0], v0[1], v0[2], d0[0], d0[1]], dtype=np.float64)
    out = [(0.0, state.copy())]
    s = 0.0
    while s < s_end:
        k1 = f(state)
        k2 = f(state + 0.5 * h * k1)
        k3 = f(state + 0.5 * h * k2)
        k4 = f(state + h * k3)
        state = state + h / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)
        s += h
        out.append((s, state.copy()))
    return out


def test_crossings_match_rk4_lorentz():
    rng = np.random.default_rng(7)
    n = 6
    tr = dict(vx=np.zeros(n), vy=np.zeros(n), vz=np.zeros(n),
              phi0=rng.uniform(0, 2 * math.pi, n), tgl=rng.uniform(-0.8, 0.8, n),
              t0=np.zeros(n))
    pt = np.array([0.15, 0.3, 0.7, 1.5, 4.0, 0.25])
    q = np.array([1, -1, 1, -1, 1, -1], dtype=float)
    tr["curv"] = -q * B / pt
    cr = tpcsynth.crossings(tr, 0, 500)
    x_r, _, _ = tpcsynth.geometry()
    checked = 0
    for i in range(n):
        sel = np.nonzero(cr["track"] == i)[0][:12]
        if len(sel) == 0:
            continue
        s_end = cr["s"][sel].max() + 1.0
        d0 = (math.cos(tr["phi0"][i]), math.sin(tr["phi0"][i]))
        traj = _lorentz_rk4((0, 0, 0), d0, tr["curv"][i], tr["tgl"][i], s_end)
        ss = np.array([t[0] for t in traj])
        sv = np.array([t[1] for t in traj])
        for j in sel:
            unit, row = cr["unit"][j], cr["row"][j]
            alpha = math.radians((unit % 18 + 0.5) * 20.0)
            lx = sv[:, 0] * math.cos(alpha) + sv[:, 1] * math.sin(alpha) - x_r[row]
            # the RK4 step bracketing the crossing closest to the generator's arc
            k = int(np.argmin(np.abs(ss - cr["s"][j])))
            lo = max(k - 2, 0)
            seg = slice(lo, min(k + 3, len(ss)))
            idx = np.nonzero(np.diff(np.sign(lx[seg])) != 0)[0]
            assert len(idx) >= 1
            a = lo + idx[0]
            # refine inside the step with fine RK4 from the bracketing state
            sub = _lorentz_rk4(sv[a][:3], sv[a][3:], tr["curv"][i], tr["tgl"][i], 0.021, h=1e-4)
            sx = np.array([t[1] for t in sub])
            lxs = sx[:, 0] * math.cos(alpha) + sx[:, 1] * math.sin(alpha) - x_r[row]
            b = np.nonzero(np.diff(np.sign(lxs)) != 0)[0][0]
            w = lxs[b] / (lxs[b] - lxs[b + 1])
            p = sx[b] + w * (sx[b + 1] - sx[b])
            ly = -p[0] * math.sin(alpha) + p[1] * math.cos(alpha)
            assert abs(ly - cr["y"][j]) < 1e-6
            assert abs(p[2] - cr["z"][j]) < 1e-6
            checked += 1
    assert checked >= 30


def test_pt_power_law_ks():
    rng = np.random.default_rng(11)
    pt = tpcsynth.sample_pt_powerlaw(rng, 20000)
    a, b = 0.1, 10.0
    cdf = lambda x: (a ** -2 - np.asarray(x) ** -2) / (a ** -2 - b ** -2)
    assert st.kstest(pt, cdf).pvalue > 1e-3
    assert 0.74 < np.mean(pt < 0.2) < 0.76  # 75% below 0.2 GeV/c


def test_landau_charge_ks():
    rng = np.random.default_rng(12)
    q = tpcsynth.landau_charge(rng, 20000)
    ref = st.landau(loc=100 + 0.22278 * 10, scale=10)
    sel = q < 5000
    assert st.kstest(q[sel], lambda x: ref.cdf(x) / ref.cdf(5000)).pvalue > 1e-3
    # most probable value near 100 ADC
    hist, edges = np.histogram(q, bins=np.arange(50, 200, 2))
    assert 90 < edges[np.argmax(hist)] < 110


def test_zs_contract_and_determinism():
    ev = tpcsynth.generate(tpcsynth.config_small(20, n_time_bins=300), 5)
    assert ev.adc.min() >= 3 and ev.adc.max() <= 1023
    x, pitch, npads = tpcsynth.geometry()
    rs = ev.row_start.astype(np.int64)
    for ur in range(ev.n_units * 152):
        a, b = rs[ur], rs[ur + 1]
        assert np.all(ev.pad[a:b] < npads[ur % 152])
        key = ev.time[a:b].astype(np.int64) * 256 + ev.pad[a:b]
        assert np.all(np.diff(key) > 0)
    ev2 = tpcsynth.generate(tpcsynth.config_small(20, n_time_bins=300), 5)
    assert np.array_equal(ev.adc, ev2.adc) and np.array_equal(ev.pad, ev2.pad)


def test_noise_occupancy_matches_tail_probability():
    # no tracks: every sample is noise; occupancy = P(N(0,1) >= 2.5)
    cfg = tpcsynth.config_small(0, n_time_bins=2000)
    ev = tpcsynth.generate(cfg, 3)
    occ = ev.n_samples / (15504 * 2000)
    p = 0.5 * math.erfc(2.5 / math.sqrt(2))
    assert abs(occ - p) < 5 * math.sqrt(p / (15504 * 2000))

"""Pins of the oracle's Kalman primitives against closed forms.

* propagation vs an analytic helix written in angle form (y from the centre
  of curvature, z from the turning angle);
* the Jacobian vs central finite differences of the propagation;
* the 3-point seed vs the circle through the three points (perpendicular
  bisectors) and the dip from the turning angle;
* a fit of exact helix points returns the helix;
* with no process noise the Kalman fit equals the batch weighted least-squares
  solution with the same Gaussian prior (scipy);
* pulls of smeared helices are standard normal; covariances are PD.
"""
import math

import mpmath
import numpy as np
import pytest
from scipy.optimize import least_squares

import oracle

PAR = oracle.default_params()
B = PAR["bz_b"]
NPADS, XFX, PFX = oracle.geometry()
XR = XFX / 65536.0


def helix_at(p0, x0, x):
    """State (y, z, snp, tgl, qpt) at x of the helix with state p0 at x0,
    evaluated in 50-digit arithmetic (mpmath) so that the reference has no
    cancellation even for nearly straight tracks."""
    with mpmath.workdps(50):
        y0, z0, s0, t, q = [mpmath.mpf(float(v)) for v in p0]
        C = -mpmath.mpf(B) * q
        s = s0 + C * (mpmath.mpf(float(x)) - mpmath.mpf(float(x0)))
        if abs(s) >= 1:
            return None
        phi0, phi = mpmath.asin(s0), mpmath.asin(s)
        if C == 0:
            y = y0 + mpmath.tan(phi0) * (x - x0)
            z = z0 + t * (x - x0) / mpmath.cos(phi0)
        else:
            y = y0 + (mpmath.cos(phi0) - mpmath.cos(phi)) / C
            z = z0 + t * (phi - phi0) / C
        return np.array([float(y), float(z), float(s), float(t), float(q)])


CASES = [
    ([1.0, 2.0, 0.3, 0.5, 2.0], 100.0, 112.0),
    ([-3.0, 0.0, -0.6, -0.9, -8.0], 150.0, 131.0),
    ([10.0, -5.0, 0.0, 0.1, 0.05], 200.0, 240.0),
    ([0.5, 1.0, 0.85, 0.3, 6.0], 90.0, 91.06),
    ([0.0, 0.0, -0.2, 1.0, -15.0], 120.0, 121.06),
    ([0.0, 0.0, 0.4, -0.4, 1e-6], 100.0, 180.0),
]


@pytest.mark.parametrize("p0,x1,x2", CASES)
def test_propagation_matches_analytic_helix(p0, x1, x2):
    rc, p = oracle.helix_propagate(p0, x1, x2)
    assert rc == 0
    ref = helix_at(p0, x1, x2)
    assert np.allclose(p, ref, rtol=0, atol=1e-10)


def test_propagation_stops_at_snp_limit():
    p0 = [0.0, 0.0, 0.9, 0.0, 20.0]  # C = -0.03/cm -> s falls... use positive C
    rc, _ = oracle.helix_propagate([0.0, 0.0, 0.9, 0.0, -20.0], 100.0, 102.0)
    assert rc == 1  # s2 = 0.9 + 0.02998*2 > 0.95
    rc, _ = oracle.helix_propagate(p0, 100.0, 102.0)
    assert rc == 0


@pytest.mark.parametrize("p0,x1,x2", CASES)
def test_jacobian_matches_finite_differences(p0, x1, x2):
    rc, p, J = oracle.helix_propagate(p0, x1, x2, jacobian=True)
    assert rc == 0
    Jfd = np.zeros((5, 5))
    for j in range(5):
        h = 1e-6 * max(1.0, abs(p0[j]))
        a = list(p0)
        b = list(p0)
        a[j] += h
        b[j] -= h
        pa = helix_at(a, x1, x2)
        pb = helix_at(b, x1, x2)
        Jfd[:, j] = (pa - pb) / (2 * h)
    assert np.allclose(J, Jfd, rtol=1e-6, atol=1e-7)


def circle_through(a, m, e):
    """Centre and radius of the circle through three points."""
    (x1, y1), (x2, y2), (x3, y3) = a, m, e
    A = np.array([[x2 - x1, y2 - y1], [x3 - x1, y3 - y1]], dtype=np.float64)
    rhs = 0.5 * np.array([x2 ** 2 - x1 ** 2 + y2 ** 2 - y1 ** 2, x3 ** 2 - x1 ** 2 + y3 ** 2 - y1 ** 2])
    c = np.linalg.solve(A, rhs)
    return c, math.hypot(x1 - c[0], y1 - c[1])


@pytest.mark.parametrize("q,s0,t,L", [(2.0, 0.2, 0.4, 9), (-5.0, -0.5, -1.0, 5), (0.3, 0.7, 0.1, 30),
                                      (-12.0, 0.1, 0.8, 12)])
def test_seed_matches_circle_through_three_points(q, s0, t, L):
    r1 = 20
    p0 = [3.0, 7.0, s0, t, q]
    ys, zs = [], []
    for i in range(L):
        st = helix_at(p0, XR[r1], XR[r1 + i])
        ys.append(int(round(st[0] * 65536)))
        zs.append(int(round((st[1] + 100.0) * 65536)))
    rc, p = oracle.seed(ys, zs, r1)
    assert rc == 0
    iA, iM, iE = 0, (L + 1) // 2 - 1, L - 1
    pts = [(XR[r1 + i], ys[i] / 65536.0) for i in (iA, iM, iE)]
    c, R = circle_through(*pts)
    # orientation: counter-clockwise (left turn) means positive curvature
    (ax, ay), (mx, my), (ex, ey) = pts
    orient = np.sign((mx - ax) * (ey - ay) - (my - ay) * (ex - ax))
    C = orient / R
    assert abs(p[4] - (-C / B)) <= 1e-9 * max(1, abs(C / B))
    # tangent at A is perpendicular to the radius, oriented towards +x
    rx, ry = ax - c[0], ay - c[1]
    tx, ty = (-ry, rx) if orient > 0 else (ry, -rx)
    nrm = math.hypot(tx, ty)
    assert abs(p[2] - ty / nrm) < 1e-9
    # dip: dz over the arc from A to E (turning angle times radius)
    ang = math.atan2(ey - c[1], ex - c[0]) - math.atan2(ay - c[1], ax - c[0])
    ang = (ang + math.pi) % (2 * math.pi) - math.pi
    arc = abs(ang) * R
    assert abs(p[3] - (zs[iE] - zs[iA]) / 65536.0 / arc) < 1e-9
    assert p[0] == ys[0] / 65536.0 and p[1] == 0.0
    # and it is close to the generating helix (fixed-point rounding only)
    assert abs(p[4] - q) < 0.02 * max(1.0, abs(q)) + 0.05


def _c0(row):
    return np.diag([PAR["sigma_y"][row] ** 2, PAR["sigma_z"][row] ** 2, 0.1 ** 2, 0.1 ** 2, 10.0 ** 2])


def _track_points(truth_last, rows, rng=None, sy=0.06, sz=0.05):
    my, mz = [], []
    for r in rows:
        st = helix_at(truth_last, XR[rows[-1]], XR[r])
        my.append(st[0] + (rng.normal(0, sy) if rng is not None else 0.0))
        mz.append(st[1] + (rng.normal(0, sz) if rng is not None else 0.0))
    return np.array(my), np.array(mz)


def test_fit_of_exact_helix_returns_helix():
    rows = list(range(140, 20, -1))
    truth = np.array([4.0, -3.0, 0.25, 0.6, 1.5])  # at the last (innermost) row
    my, mz = _track_points(truth, rows)
    start = helix_at(truth, XR[rows[-1]], XR[rows[0]])
    start = start + np.array([0.05, 0.05, 0.01, 0.01, 0.2])
    n = len(rows)
    # a prior much broader than the measurements, so that its offset from the
    # helix does not bias the result
    broad = np.diag([10.0 ** 2, 10.0 ** 2, 1.0, 1.0, 100.0 ** 2])
    rc, p, C, chi2 = oracle.kalman_fit(rows, my, mz, [0.06 ** 2] * n, [0.05 ** 2] * n, start,
                                       broad)
    assert rc == 0
    # second pass from the first result, covariance reset, as in the refit
    p1 = helix_at(p, XR[rows[-1]], XR[rows[0]])
    rc, p2, C2, chi2 = oracle.kalman_fit(rows, my, mz, [0.06 ** 2] * n, [0.05 ** 2] * n, p1,
                                         broad)
    assert rc == 0
    assert np.allclose(p2, truth, rtol=0, atol=1e-7)
    assert chi2 < 1e-8


def _ls_solution(rows, my, mz, p_start, C0):
    xr, x0 = XR[rows[-1]], XR[rows[0]]
    w0 = 1.0 / np.sqrt(np.diag(C0))

    def resid(q):
        out = []
        for r, a, b in zip(rows, my, mz):
            st = helix_at(q, xr, XR[r])
            out += [(a - st[0]) / 0.06, (b - st[1]) / 0.05]
        pf = helix_at(q, xr, x0)
        out += list((pf - p_start) * w0)
        return np.array(out)

    q0 = helix_at(p_start, x0, xr)
    sol = least_squares(resid, q0, xtol=1e-15, ftol=1e-15, gtol=1e-15, method="lm")
    return sol.x


@pytest.mark.parametrize("seed", range(4))
def test_kalman_equals_batch_least_squares(seed):
    rng = np.random.default_rng(300 + seed)
    rows = list(range(150, 40, -1))
    truth = np.array([rng.uniform(-5, 5), rng.uniform(-5, 5), rng.uniform(-0.5, 0.5),
                      rng.uniform(-1, 1), rng.uniform(-3, 3)])
    my, mz = _track_points(truth, rows, rng)
    # The extended filter linearises each step around its running estimate,
    # so it equals the batch optimum only while that estimate stays near it.
    # A prior centred on the helix and about as tight as the data keeps it
    # there from the first hit on; the prior is the same in both solutions.
    start = helix_at(truth, XR[rows[-1]], XR[rows[0]])
    C0 = np.diag([0.06 ** 2, 0.05 ** 2, 0.002 ** 2, 0.002 ** 2, 0.02 ** 2])
    n = len(rows)
    rc, p, C, _ = oracle.kalman_fit(rows, my, mz, [0.06 ** 2] * n, [0.05 ** 2] * n, start, C0)
    assert rc == 0
    q = _ls_solution(rows, my, mz, start, C0)
    sig = np.sqrt(np.diag(C))
    # the extended Kalman filter linearises around its running estimate; it
    # agrees with the exact least-squares optimum to a small fraction of sigma
    assert np.all(np.abs(p - q) <= 1e-2 * sig)


def test_pulls_are_standard_normal():
    rng = np.random.default_rng(400)
    N = 2000
    pulls = []
    rows = list(range(151, 0, -2))
    for _ in range(N):
        truth = np.array([rng.uniform(-5, 5), rng.uniform(-5, 5), rng.uniform(-0.4, 0.4),
                          rng.uniform(-1, 1), rng.uniform(-2, 2)])
        my, mz = _track_points(truth, rows, rng)
        start = helix_at(truth, XR[rows[-1]], XR[rows[0]])
        n = len(rows)
        rc, p, C, _ = oracle.kalman_fit(rows, my, mz, [0.06 ** 2] * n, [0.05 ** 2] * n, start,
                                        _c0(rows[0]))
        assert rc == 0
        assert oracle.is_pd(C)
        pulls.append((p - truth) / np.sqrt(np.diag(C)))
    pulls = np.array(pulls)
    m = pulls.mean(axis=0)
    s = pulls.std(axis=0)
    assert np.all(np.abs(m) < 3 / math.sqrt(N)), m
    assert np.all(np.abs(s - 1) < 0.05), s


def test_is_pd():
    assert oracle.is_pd(np.eye(5))
    M = np.eye(5)
    M[0, 1] = M[1, 0] = 1.0
    assert not oracle.is_pd(M)

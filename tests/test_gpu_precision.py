"""Precision stress: 30% low-pT loopers (0.05-0.2 GeV/c), noise sigma 2 ADC
(peak threshold 10) and 10% dead pads.  The FP32 following and refit (the
refit with UD-factorised covariance; FP64 only for a low-pT track whose FP32
pivots fail), against the FP64 oracle: integer outputs bit-exact,
parameters within tolerance.  Prints the FP64 refit rate and the error of
each parameter against the oracle."""
import numpy as np
import pytest

import oracle
import tpcsynth

from _parity import (FLOORS, compare_clusters, compare_fit, cov_pd, exempt_tracklets,
                     ill_conditioned, run_gpu, run_oracle)

pytestmark = pytest.mark.gpu

PAR = oracle.default_params(2.0)  # peak threshold 10 at noise 2
NAMES = ("y", "z", "snp", "tgl", "qpt")


@pytest.fixture(scope="module")
def c5():
    ev = tpcsynth.generate(tpcsynth.config_chunk(505, 0, stress=True, n_coll=3), 505)
    return ev, run_gpu(ev, params=PAR), run_oracle(ev, params=PAR)


def test_stress_clusters_links_tracklets(c5):
    ev, g, o = c5
    compare_clusters(g["clusters"], o["clusters"])
    assert np.array_equal(g["links"]["down"], o["down"])
    assert np.array_equal(g["links"]["up"], o["up"])
    assert np.array_equal(g["tracklets"]["tl_start"], o["tracklets"]["tl_start"])


def test_stress_fit_precision(c5):
    ev, g, o = c5
    compare_fit(g, o)
    gtr, ofit = g["tracks"], o["fit"]
    ex = exempt_tracklets(ofit, gtr.get("follow_hits"))
    rel, sig = [], []
    for j, t in enumerate(gtr["tracklet"]):
        t = int(t)
        if t in ex or ill_conditioned(ofit, t):
            continue
        op = ofit["par"][t]
        gp = gtr["par"][j].astype(np.float64)
        rel.append(np.abs(gp - op) / np.maximum(np.abs(op), FLOORS))
        iu = np.triu_indices(5)
        C = np.zeros((5, 5))
        C[iu] = ofit["cov"][t]
        sig.append(np.abs(gp - op) / np.sqrt(np.diag(C)))
    rel, sig = np.array(rel), np.array(sig)
    n = len(gtr["tracklet"])
    c = g["counts"]
    fb = c["n_fallback"] / max(n, 1)
    print(f"precision stress: {ev.n_samples} samples, {c['n_clusters']} clusters, {n} tracks, "
          f"{len(ex)} exempt tracklets; FP64 refits {c['n_fallback']} ({100 * fb:.2f}%), "
          f"FP32 tracks flagged not PD {c['n_not_pd']}; FP64 still not PD {c['n_fallback_fail']}")
    for i, nm in enumerate(NAMES):
        print(f"  {nm:4s} relative error: median {np.median(rel[:, i]):.2e} "
              f"p99 {np.percentile(rel[:, i], 99):.2e} max {rel[:, i].max():.2e}; "
              f"in oracle sigma: p99 {np.percentile(sig[:, i], 99):.2e} max {sig[:, i].max():.2e}")
    assert rel.max() <= 1e-4
    assert c["n_fallback_fail"] == 0
    assert np.all(cov_pd(gtr["cov"]))
    assert fb < 0.25

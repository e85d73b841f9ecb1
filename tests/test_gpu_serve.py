"""Serving loop on the GPU: chunks of uneven size run concurrently on several
slots (one stream each) give exactly the results they give alone, including a
chunk rerun after its output estimate proved too small."""
import numpy as np
import pytest

import tpcsynth
from paper_2208_07412_amd import serve, tpc

from _parity import run_gpu

pytestmark = pytest.mark.gpu

NCOLL = [3, 6, 2, 8, 4, 5, 1, 7]


@pytest.fixture(scope="module")
def chunks():
    return [tpcsynth.generate(tpcsynth.config_chunk(404, i, n_coll=n), 4040 + i)
            for i, n in enumerate(NCOLL)]


def _host(job):
    o = job.outputs
    n = job.counts["n_clusters"]
    return dict(clusters=tpc.clusters_to_host(o["clusters"], job.n_units),
                links=tpc.links_to_host(o["links"], n),
                tracklets=tpc.tracklets_to_host(o["tracklets"]),
                tracks=tpc.tracks_to_host(o["tracks"], n))


def test_same_alone_and_in_mix(chunks):
    alone = [run_gpu(ev, moments=False, follow=False) for ev in chunks]
    T = max(ev.n_time_bins for ev in chunks)
    ns = max(ev.n_samples for ev in chunks)
    ex = serve.GpuExecutor(3, 36, T, ns, ns // 4, keep_outputs=True)
    jobs = [serve.make_job(i, ev) for i, ev in enumerate(chunks)]
    jobs[2].cl_cap = 1024  # too small: the device reports the need, the chunk reruns
    sched = serve.Scheduler(ex, 3, budget_bytes=64 << 30)
    arrivals = np.array([0.0, 0.0, 0.0, 0.0, 0.002, 0.004, 0.004, 0.01])
    done = serve.run_stream(sched, jobs, arrivals)
    assert len(done) == len(jobs)
    assert sched.max_concurrent == 3
    assert jobs[2].retries == 1
    for j, a in zip(jobs, alone):
        assert j.error is None, j.error
        g = _host(j)
        for k in ("crow_start", "y_fx", "z_fx", "dpad", "dtime", "qtot", "qmax", "flags"):
            assert np.array_equal(g["clusters"][k], a["clusters"][k]), (j.id, k)
        n = j.counts["n_clusters"]
        for k in ("down", "up", "upc", "downc"):
            assert np.array_equal(g["links"][k], a["links"][k][:n]), (j.id, k)
        assert np.array_equal(g["tracklets"]["tl_start"], a["tracklets"]["tl_start"])
        for k in ("tracklet", "par", "cov", "chi2", "hits", "hit_start", "cluster_track", "flags"):
            assert np.array_equal(g["tracks"][k], a["tracks"][k]), (j.id, k)
        assert j.latency > 0
    ex.close()

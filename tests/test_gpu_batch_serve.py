"""Batched and served forms: every job's result equals its result alone.

A batch runs all its jobs through one fused counting launch and one set of
job-aware scan / agglomeration / filter launches replayed from a HIP graph;
the server runs batches of whatever has arrived on several streams at once.
Neither may change any job's result: rows, counts and labels are compared
bit for bit with the plain single-job call and with the oracle.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import assert_same, dev, same_result

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU test run without a GPU"
    return t


@pytest.fixture(scope="module")
def raster(torch):
    import paper_1907_03620_amd as r
    r.load()
    r.set_tuning(None)
    yield r
    r.set_tuning(None)


def _say(msg):
    print(msg, flush=True)


def _jobs(n_jobs=24, scale=0.02, seed=4):
    specs = synth.batch_jobs(seed=seed, n_jobs=n_jobs, size_scale=scale)
    out = []
    for k, sp in enumerate(specs):
        dt = "f32" if k % 5 == 3 else "f64"
        sp = synth.JobSpec(seed=sp.seed, n=sp.n, precision=sp.precision, tau=sp.tau, mu=sp.mu, dtype=dt)
        out.append((sp, synth.job_points(sp)))
    return out


@pytest.fixture(scope="module")
def batch24(torch):
    jobs = _jobs()
    # an empty job and a one-point job ride along
    jobs.append((synth.JobSpec(seed=0, n=0, precision=2, tau=1, mu=1), np.zeros((0, 2))))
    jobs.append((synth.JobSpec(seed=0, n=1, precision=1, tau=1, mu=1), np.array([[1.25, 2.5]])))
    return [(sp, pts, dev(pts, torch)) for sp, pts in jobs]


def _batch_args(batch):
    return [dict(points=d, precision=sp.precision, tau=sp.tau, mu=sp.mu) for sp, _, d in batch]


@pytest.mark.parametrize("mode", [0, 1])
def test_batch_matches_alone_and_oracle(raster, torch, batch24, mode):
    _say(f"batch of {len(batch24)} jobs, {sum(sp.n for sp, _, _ in batch24)} points, mode {mode}")
    raster.set_tuning(mode=mode)
    try:
        res = raster.cluster_batch(_batch_args(batch24))
    finally:
        raster.set_tuning(None)
    assert len(res) == len(batch24)
    for k, ((sp, pts, d), r) in enumerate(zip(batch24, res)):
        alone = raster.cluster(d, precision=sp.precision, tau=sp.tau, mu=sp.mu)
        same_result(r, alone, f"job {k} batch vs alone")
        o = oracle.cluster(pts, tau=sp.tau, mu=sp.mu, precision=sp.precision)
        assert_same(r, o, f"job {k} batch vs oracle")


def test_batch_graph_replay_and_recapture(raster, torch, batch24):
    first = raster.cluster_batch(_batch_args(batch24))
    again = raster.cluster_batch(_batch_args(batch24))          # replay of the captured graph
    smaller = raster.cluster_batch(_batch_args(batch24[3:11]))  # fits the same buffers: replay
    for k in range(len(batch24)):
        same_result(first[k], again[k], f"replay job {k}")
    for k in range(8):
        same_result(first[k + 3], smaller[k], f"sub-batch job {k}")
    for tuning in (dict(block=512, items=2, mode=1), dict(preagg_slots=2048, mode=1),
                   dict(block=128, items=16, load_factor=0.3), dict(mode=1, load_factor=0.8)):
        raster.set_tuning(**tuning)
        try:
            other = raster.cluster_batch(_batch_args(batch24))
        finally:
            raster.set_tuning(None)
        for k in range(len(batch24)):
            same_result(first[k], other[k], f"tuning {tuning} job {k}")


def test_batch_spilled_job_is_redone(raster, torch):
    # uniform noise: nearly every point its own tile, far more than the table
    # sized for n/8 tiles can hold, so the job spills and is redone alone
    rng = np.random.default_rng(9)
    noise = rng.uniform(0.0, 1000.0, size=(400_000, 2))
    small = synth.plain_small(1)[:50_000]
    d1, d2 = dev(noise, torch), dev(small, torch)
    for mode in (0, 1):
        raster.set_tuning(mode=mode)
        try:
            res = raster.cluster_batch([dict(points=d1, precision=2, tau=1, mu=1),
                                        dict(points=d2, precision=1, tau=5, mu=4)])
        finally:
            raster.set_tuning(None)
        assert_same(res[0], oracle.cluster(noise, tau=1, mu=1, precision=2), f"spilled job, mode {mode}")
        assert_same(res[1], oracle.cluster(small, tau=5, mu=4, precision=1), f"neighbour of spilled job, mode {mode}")


def test_batch_range_error_fails_whole_batch(raster, torch, batch24):
    bad = np.array([[0.5, 0.5], [np.inf, 0.0]])
    args = _batch_args(batch24[:4]) + [dict(points=dev(bad, torch), precision=1, tau=1, mu=1)]
    with pytest.raises(raster.RasterError) as e:
        raster.cluster_batch(args)
    assert e.value.code == raster.E_RANGE
    # the engine still works afterwards
    ok = raster.cluster_batch(_batch_args(batch24[:4]))
    for k in range(4):
        sp, _, d = batch24[k]
        same_result(ok[k], raster.cluster(d, precision=sp.precision, tau=sp.tau, mu=sp.mu), f"after error {k}")


def test_batch_invalid_job(raster, torch, batch24):
    args = _batch_args(batch24[:2])
    args[1]["tau"] = 0
    with pytest.raises(raster.RasterError) as e:
        raster.cluster_batch(args)
    assert e.value.code == raster.E_INVAL


def test_server_mix_matches_alone(raster, torch, batch24):
    srv = raster.Server(budget_bytes=8 << 30, max_slots=3)
    try:
        tickets = [(k, srv.submit(d, tau=sp.tau, mu=sp.mu, precision=sp.precision))
                   for k, (sp, _, d) in enumerate(batch24)]
        # a second wave while the first is still running
        tickets += [(k, srv.submit(batch24[k][2], tau=batch24[k][0].tau, mu=batch24[k][0].mu,
                                   precision=batch24[k][0].precision))
                    for k in range(0, len(batch24), 2)]
        lats = []
        for k, t in tickets:
            r, lat = srv.wait(t)
            lats.append(lat)
            sp, _, d = batch24[k]
            alone = raster.cluster(d, precision=sp.precision, tau=sp.tau, mu=sp.mu)
            same_result(r, alone, f"served job {k}")
        assert min(lats) > 0.0
    finally:
        srv.close()


def test_server_tight_budget_queues(raster, torch, batch24):
    # a budget that holds about one job at a time: jobs queue, none fails
    from paper_1907_03620_amd import RasterError
    srv = raster.Server(budget_bytes=16 << 20, max_slots=2)
    try:
        big = dev(synth.zipf_hot(2, n=2_000_000, block=1_000_000), torch)
        with pytest.raises(RasterError) as e:
            srv.submit(big, tau=5, mu=4, precision=2)
        assert e.value.code == raster.E_BUDGET
        tickets = [(k, srv.submit(d, tau=sp.tau, mu=sp.mu, precision=sp.precision))
                   for k, (sp, _, d) in enumerate(batch24[:10])]
        for k, t in tickets:
            r, _ = srv.wait(t)
            sp, _, d = batch24[k]
            same_result(r, raster.cluster(d, precision=sp.precision, tau=sp.tau, mu=sp.mu), f"queued job {k}")
    finally:
        srv.close()


def test_autotuner_choice_gives_same_results(raster, torch, batch24, tmp_path, monkeypatch):
    monkeypatch.setenv("RASTER_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    from paper_1907_03620_amd import autotune
    args = _batch_args(batch24)
    points = sum(sp.n for sp, _, _ in batch24)
    base = raster.cluster_batch(args)
    best = autotune.tune("batch", lambda: raster.cluster_batch(args), points=points, reps=1, use_cache=False,
                         sweeps={"block": [128, 512], "preagg_slots": [0, 1024], "load_factor": [0.4, 0.8]})
    assert autotune.cached("batch", points) == best
    raster.set_tuning(best)
    try:
        res = raster.cluster_batch(args)
    finally:
        raster.set_tuning(None)
    for k in range(len(batch24)):
        same_result(base[k], res[k], f"autotuned job {k}")

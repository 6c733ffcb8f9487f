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


def _lowbias32(x):
    """C. Wellons' 32-bit mixer, as the library hashes tiles (test-local)."""
    x = np.asarray(x, dtype=np.uint32)
    x = x ^ (x >> np.uint32(16))
    x = x * np.uint32(0x7FEB352D)
    x = x ^ (x >> np.uint32(15))
    x = x * np.uint32(0x846CA68B)
    return x ^ (x >> np.uint32(16))


def _unsketched_noise(n, precision, seed):
    """Uniform noise with every point removed whose tile falls in the fixed
    1/64 hash sample that the batch's distinct-tile sketch reads: the sketch
    sees almost no tile, the job's batch table gets its smallest size and
    overflows, and the job must be redone alone."""
    rng = np.random.default_rng(seed)
    pts = rng.uniform(0.0, 1000.0, size=(3 * n // 2, 2))
    s = 10.0 ** precision
    kx = np.trunc(pts[:, 0] * s).astype(np.int64)
    ky = np.trunc(pts[:, 1] * s).astype(np.int64)
    bx = (kx + (1 << 31)).astype(np.uint64).astype(np.uint32)
    by = (ky + (1 << 31)).astype(np.uint64).astype(np.uint32)
    with np.errstate(over="ignore"):
        h = _lowbias32(bx * np.uint32(0x9E3779B9) + by)
    return np.ascontiguousarray(pts[(h & np.uint32(63)) != 0][:n])


def test_batch_spilled_job_is_redone(raster, torch):
    noise = _unsketched_noise(400_000, 2, seed=9)
    small = synth.plain_small(1)[:50_000]
    d1, d2 = dev(noise, torch), dev(small, torch)
    for mode in (0, 1):
        raster.set_tuning(mode=mode)
        try:
            res = raster.cluster_batch([dict(points=d1, precision=2, tau=1, mu=1),
                                        dict(points=d2, precision=1, tau=5, mu=4)])
        finally:
            raster.set_tuning(None)
        assert res[0].stats["redone"] == 1, f"mode {mode}: the job fit its batch table"
        assert res[1].stats["redone"] == 0
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


def test_server_orders_after_producer(raster, torch):
    """Points still being written on the submitter's stream are read only
    once that stream has written them."""
    pts = synth.plain_small(1)
    base = dev(pts, torch)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        out = torch.full_like(base, 1.0e6)   # until the copy lands: every point on one far tile
        torch.cuda._sleep(20_000_000)        # the producer is still busy when the job is submitted
        out.copy_(base)
        srv = raster.Server(budget_bytes=1 << 30, max_slots=2)
        try:
            t = srv.submit(out, tau=5, mu=4, precision=1)
            r, _ = srv.wait(t)
        finally:
            srv.close()
    torch.cuda.synchronize()
    same_result(r, raster.cluster(base, precision=1, tau=5, mu=4), "job submitted behind its producer")
    assert_same(r, oracle.cluster(pts, tau=5, mu=4, precision=1), "job submitted behind its producer")


def test_server_budget_bounds_device_memory(raster, torch):
    """Noise-heavy jobs (p=3: almost every point its own tile, tables many
    times an n/8 guess) under a budget that holds about two of them: the
    library's in-use device bytes stay within the budget."""
    specs = [synth.JobSpec(seed=7000 + k, n=300_000 + 60_000 * k, precision=3, tau=3, mu=2) for k in range(8)]
    host = [synth.job_points(sp) for sp in specs]
    devs = [dev(h, torch) for h in host]
    plain = [raster.cluster(d, precision=sp.precision, tau=sp.tau, mu=sp.mu) for sp, d in zip(specs, devs)]
    budget = 192 << 20
    torch.cuda.synchronize()
    srv = raster.Server(budget_bytes=budget, max_slots=3)
    try:
        used0, _, _ = raster.memory_stats(reset_peak=True)
        tickets = [srv.submit(d, tau=sp.tau, mu=sp.mu, precision=sp.precision) for sp, d in zip(specs, devs)]
        results = [srv.wait(t)[0] for t in tickets]
        _, _, peak = raster.memory_stats()
        _, charged = srv.memory()
    finally:
        srv.close()
    _say(f"budget {budget >> 20} MiB: peak in-use {(peak - used0) >> 20} MiB above the start, "
         f"largest charge {charged >> 20} MiB")
    assert charged <= budget
    assert peak - used0 <= budget, f"in-use device bytes rose by {peak - used0}, budget {budget}"
    for k, (r, p) in enumerate(zip(results, plain)):
        same_result(r, p, f"budgeted job {k}")

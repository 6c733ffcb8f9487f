"""Full-size parity: every row of the full-size workloads against the oracle.

The oracle's results on these workloads were computed once, by
tests/golden/make_full_size_digests.py (which calls only the seeded
generators and the CPU oracle), and stored as canonical digests of their rows
with their statistics (tests/golden/full_size_digests.json).  Each test here
regenerates the same inputs, checks their digests (so a change of the
generators is reported as such), runs the GPU path at full size and compares
the digest of every row (tile, count, label) and every statistic.

* paper-500M: the benchmark's workload and launch shape -- 500M FP64 points
  streamed in ten 50M chunks through begin / feed_chunk / finish, p=2, tau=5,
  mu=4 (Algorithm 1; Section 3.6 chunked input);
* batch-256: all 256 jobs of the batched workload (sizes log-uniform in
  [1e4, 5e6], p, tau and mu drawn per job) in one batch, under the default
  and the benchmark's autotuned settings; each job also against its plain
  call;
* served-slice: the served workload's first half second of arrivals plus
  its largest job (sizes up to about 20M, FP32 and FP64, the two-million-point
  solo path), replayed in real time into the server; each job against the
  oracle and against its plain call.

On a mismatch the test reruns the oracle on the failing input and reports the
first differing rows.
"""
import json
import os
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
import synth
from digest import STAT_KEYS, points_digest, rows_digest, unbias_label
from gpu_util import assert_same, dev

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "full_size_digests.json")
GPU_STAT = {"n": "n_points", "distinct": "distinct_tiles", "significant": "significant_tiles",
            "components": "components", "clusters": "clusters", "tiles": "tiles"}


@pytest.fixture(scope="module")
def golden():
    with open(GOLDEN) as f:
        return json.load(f)


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


def gpu_summary(res):
    kx, ky, cnt, lab = res.numpy(sort=False)
    lx, ly = unbias_label(lab)
    d = {k: int(res.stats[v]) for k, v in GPU_STAT.items()}
    d["rows"] = rows_digest(kx.astype(np.int64), ky.astype(np.int64), cnt.astype(np.uint64), lx, ly)
    return d


def check(res, want, what, oracle_fn):
    got = gpu_summary(res)
    bad = [k for k in STAT_KEYS + ("rows",) if got[k] != want[k]]
    if bad:
        _say(f"{what}: {bad} differ; rerunning the oracle for detail")
        assert_same(res, oracle_fn(), what)
    assert not bad, f"{what}: {bad} differ: {[(got[k], want[k]) for k in bad]}"


def test_paper_500M_every_row(raster, torch, golden):
    cfg = synth.PAPER_SCALE
    want = golden["paper"]
    centres = synth.paper_scale_centres(cfg["seed"])

    def chunk(c):
        return synth.paper_scale_chunk(c, seed=cfg["seed"], chunk=cfg["chunk"], n_chunks=cfg["chunks"],
                                       centres=centres)

    _say("paper-500M: generating")
    with ThreadPoolExecutor(10) as ex:
        host = list(ex.map(chunk, range(cfg["chunks"])))
    with ThreadPoolExecutor(10) as ex:
        assert list(ex.map(points_digest, host)) == want["inputs"], "the generator no longer gives the stored input"
    devs = [dev(h, torch) for h in host]
    _say("paper-500M: GPU stream, as the benchmark runs it")
    st = raster.Stream(tau=cfg["tau"], mu=cfg["mu"], precision=cfg["precision"])
    for d in devs:
        st.feed(d)
    res = st.finish()
    st.close()
    del devs
    torch.cuda.empty_cache()
    check(res, want, "paper-500M",
          lambda: oracle.cluster_chunks(host, tau=cfg["tau"], mu=cfg["mu"], precision=cfg["precision"]))


def _gen(specs, want):
    with ThreadPoolExecutor(16) as ex:
        host = list(ex.map(synth.job_points, specs))
    for sp, h, w in zip(specs, host, want):
        assert (w["seed"], w["n"], w["dtype"]) == (sp.seed, sp.n, sp.dtype)
    with ThreadPoolExecutor(16) as ex:
        digests = list(ex.map(points_digest, host))
    assert digests == [w["input"] for w in want], "the generator no longer gives the stored input"
    return host


# the autotuned choice the benchmark recorded for this batch, and the defaults
BATCH_TUNINGS = [None, dict(block=512, items=2, preagg_slots=1024, load_factor=0.6, mode=0)]


@pytest.mark.parametrize("tuning", BATCH_TUNINGS, ids=["default", "bench-autotuned"])
def test_batch_256_full_size(raster, torch, golden, tuning):
    specs = synth.batch_jobs(4)
    want = golden["batch"]["jobs"]
    _say(f"batch-256: generating {sum(s.n for s in specs)} points")
    host = _gen(specs, want)
    devs = [dev(h, torch) for h in host]
    args = [dict(points=d, precision=sp.precision, tau=sp.tau, mu=sp.mu) for sp, d in zip(specs, devs)]
    if tuning:
        raster.set_tuning(**tuning)
    try:
        _say("batch-256: one batch")
        res = raster.cluster_batch(args)
    finally:
        raster.set_tuning(None)
    assert len(res) == len(specs)
    plain_checked = 0
    for k, (sp, h, r, w) in enumerate(zip(specs, host, res, want)):
        check(r, w, f"batch job {k} (n={sp.n}, p={sp.precision})",
              lambda: oracle.cluster(h, tau=sp.tau, mu=sp.mu, precision=sp.precision))
        if tuning is None:
            alone = raster.cluster(devs[k], precision=sp.precision, tau=sp.tau, mu=sp.mu)
            assert gpu_summary(alone) == gpu_summary(r), f"job {k}: batch and plain call differ"
            plain_checked += 1
    _say(f"batch-256: {len(specs)} jobs match the oracle ({plain_checked} also their plain call)")
    del res, devs, args
    torch.cuda.empty_cache()


def test_served_slice_full_size(raster, torch, golden):
    specs = synth.served_parity_slice(5)
    want = golden["served"]["jobs"]
    assert max(s.n for s in specs) > 15_000_000 and sum(s.n >= 2_000_000 for s in specs) > 10
    assert {s.dtype for s in specs} == {"f32", "f64"}
    _say(f"served slice: generating {len(specs)} jobs, {sum(s.n for s in specs)} points")
    host = _gen(specs, want)
    devs = [dev(h, torch) for h in host]
    torch.cuda.synchronize()
    srv = raster.Server(budget_bytes=64 << 30, max_slots=4)
    tickets = []
    t0 = time.perf_counter()
    for sp, d in zip(specs, devs):
        delay = t0 + min(sp.arrival_s, 0.5) - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        tickets.append(srv.submit(d, tau=sp.tau, mu=sp.mu, precision=sp.precision))
    results = [srv.wait(t)[0] for t in tickets]
    srv.close()
    _say("served slice: comparing")
    for k, (sp, h, r, w) in enumerate(zip(specs, host, results, want)):
        check(r, w, f"served job {k} (n={sp.n}, {sp.dtype}, p={sp.precision})",
              lambda: oracle.cluster(h, tau=sp.tau, mu=sp.mu, precision=sp.precision))
        alone = raster.cluster(devs[k], precision=sp.precision, tau=sp.tau, mu=sp.mu)
        assert gpu_summary(alone) == gpu_summary(r), f"served job {k}: server and plain call differ"
    del results, devs
    torch.cuda.empty_cache()

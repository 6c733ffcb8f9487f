"""The 2x2 post-step of Section 3.6 on the GPU against the oracle.

With the step, a tile below tau is also significant when a 2x2 square of tiles
containing it holds at least tau points together (Figure 4's points spread
around a grid corner).  Compared row by row with the oracle on the paper's
corner case, tiny inputs, the plain, binned and streaming paths, range-edge
tiles and together with a wider neighbourhood.
"""
import ctypes
import json
import os

import numpy as np
import pytest

import oracle
import synth
from gpu_util import assert_same, dev

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


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


def test_fig4_corner(raster, torch):
    g = json.load(open(os.path.join(GOLDEN, "fig4_grid_corner.json")))
    pts = dev(np.array(g["points"]), torch)
    assert raster.cluster(pts, precision=0, tau=4, mu=1).stats["significant_tiles"] == 0
    r = raster.cluster(pts, precision=0, tau=4, mu=1, square=True)
    assert r.stats["significant_tiles"] == g["tau4_with_2x2_step_significant"] and r.num_clusters == 1
    kx, ky, cnt, lab = r.numpy()
    assert sorted(zip(kx.tolist(), ky.tolist())) == [tuple(t) for t in g["tiles"]]
    assert cnt.tolist() == [1, 1, 1, 1]


def _tiny(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(0, 400))
    centre = rng.uniform(-1.0, 1.0, size=2)
    pts = centre + rng.normal(0.0, float(rng.choice([0.1, 0.3, 0.6])), size=(n, 2))
    dtype = np.float32 if rng.random() < 0.25 else np.float64
    return pts.astype(dtype), int(rng.integers(0, 3)), int(rng.integers(2, 7)), int(rng.integers(1, 5))


@pytest.mark.parametrize("metric,delta", [("chebyshev", 1), ("manhattan", 2)])
def test_tiny_corpus(raster, torch, metric, delta):
    for seed in range(5000, 5100):
        pts, p, tau, mu = _tiny(seed)
        o = oracle.cluster(pts, tau=tau, mu=mu, precision=p, metric=metric, delta=delta, window=True)
        g = raster.cluster(dev(pts, torch), precision=p, tau=tau, mu=mu, metric=metric, delta=delta, square=True)
        assert_same(g, o, f"tiny seed {seed} {metric} {delta}")


def test_plain_small(raster, torch):
    pts = synth.plain_small(1)
    o = oracle.cluster(pts, tau=8, mu=4, precision=1, window=True)
    base = oracle.cluster(pts, tau=8, mu=4, precision=1)
    assert o.stats["significant"] > base.stats["significant"]
    g = raster.cluster(dev(pts, torch), precision=1, tau=8, mu=4, square=True)
    assert_same(g, o, "plain-200k with the 2x2 step")


@pytest.mark.parametrize("mode", [2, 1])
def test_mid_counting_paths(raster, torch, mode):
    pts = synth.zipf_hot(2, n=3_000_000, block=1_000_000)
    o = oracle.cluster(pts, tau=6, mu=4, precision=2, window=True)
    raster.set_tuning(mode=mode)
    try:
        g = raster.cluster(dev(pts, torch), precision=2, tau=6, mu=4, square=True)
    finally:
        raster.set_tuning(None)
    assert_same(g, o, f"zipf 3M with the 2x2 step, mode {mode}")


def test_dense_uniform_grid(raster, torch):
    # mostly light tiles: most of the table goes through the square test
    rng = synth.rng_for(13)
    pts = rng.uniform(0.0, 100.0, size=(1_000_000, 2))
    _say("dense uniform grid with the 2x2 step")
    o = oracle.cluster(pts, tau=3, mu=4, precision=1, window=True)
    g = raster.cluster(dev(pts, torch), precision=1, tau=3, mu=4, square=True)
    assert_same(g, o, "dense uniform grid with the 2x2 step")


def test_stream(raster, torch):
    centres = synth.paper_scale_centres(3)
    chunks = [synth.paper_scale_chunk(c, centres=centres, chunk=300_000) for c in range(4)]
    st = raster.Stream(tau=3, mu=2, precision=2, square=True)
    for c in chunks:
        st.feed(dev(c, torch))
    g = st.finish()
    st.close()
    assert_same(g, oracle.cluster_chunks(chunks, tau=3, mu=2, precision=2, window=True), "stream with the 2x2 step")


def test_extreme_tiles(raster, torch):
    lim = 2 ** 31 - 2
    tiles = [(lim, lim), (lim - 1, lim), (-lim, -lim), (-lim + 1, -lim + 1), (lim, -lim), (5, 5), (6, 6)]
    pts = np.array([[x + 0.5 if x >= 0 else x - 0.5, y + 0.5 if y >= 0 else y - 0.5] for x, y in tiles])
    o = oracle.cluster(pts, tau=2, mu=1, precision=0, window=True)
    g = raster.cluster(dev(pts, torch), precision=0, tau=2, mu=1, square=True)
    assert_same(g, o, "extreme tiles with the 2x2 step")


def test_invalid_options(raster, torch):
    lib = raster.load()
    pts = dev(np.array([[0.5, 0.5]]), torch)
    out = ctypes.c_void_p()
    for o in (raster._Options(0, 1, 2, 0), raster._Options(0, 1, 0, 1), raster._Options(3, 1, 0, 0),
              raster._Options(0, 0, 1, 0)):
        rc = lib.raster_cluster_opts(ctypes.c_void_p(pts.data_ptr()), 1, 2, 10.0, 1, 1, ctypes.byref(o), None,
                                     ctypes.byref(out))
        assert rc == raster.E_INVAL and not out.value
    # NULL options are the defaults
    rc = lib.raster_cluster_opts(ctypes.c_void_p(pts.data_ptr()), 1, 2, 10.0, 1, 1, None, None, ctypes.byref(out))
    assert rc == 0 and out.value
    lib.raster_result_free(out)


def test_batch_and_server_with_the_step(raster, torch):
    # jobs with and without the step (and with another neighbourhood) in one
    # batch call and through the server; each equals the oracle
    specs = synth.batch_jobs(seed=31, n_jobs=10, size_scale=0.02)
    variants = [dict(), dict(square=True), dict(square=True, metric="manhattan", delta=2), dict(metric="chebyshev",
                                                                                               delta=2)]
    jobs = [(sp, synth.job_points(sp), variants[k % len(variants)]) for k, sp in enumerate(specs)]
    args = [dict(points=dev(p, torch), precision=sp.precision, tau=sp.tau, mu=sp.mu, **v) for sp, p, v in jobs]

    def want(sp, p, v):
        return oracle.cluster(p, tau=sp.tau, mu=sp.mu, precision=sp.precision, metric=v.get("metric", "chebyshev"),
                              delta=v.get("delta", 1), window=v.get("square", False))

    res = raster.cluster_batch(args)
    for k, ((sp, p, v), g) in enumerate(zip(jobs, res)):
        assert_same(g, want(sp, p, v), f"batch job {k} {v}")
    # a larger job with the step: the square pass runs over a whole batch arena
    fig = np.array(json.load(open(os.path.join(GOLDEN, "fig4_grid_corner.json")))["points"])
    res = raster.cluster_batch([dict(points=dev(fig, torch), precision=0, tau=4, mu=1, square=True),
                                dict(points=args[0]["points"], precision=jobs[0][0].precision, tau=jobs[0][0].tau,
                                     mu=jobs[0][0].mu, square=True)])
    assert res[0].num_clusters == 1 and res[0].num_tiles == 4
    assert_same(res[1], want(jobs[0][0], jobs[0][1], dict(square=True)), "second job of a square batch")
    srv = raster.Server(budget_bytes=8 << 30, max_slots=2)
    try:
        tickets = [srv.submit(a["points"], a["tau"], a["mu"], precision=a["precision"],
                              metric=a.get("metric", "chebyshev"), delta=a.get("delta", 1),
                              square=a.get("square", False)) for a in args]
        for k, (t, (sp, p, v)) in enumerate(zip(tickets, jobs)):
            g, _ = srv.wait(t)
            assert_same(g, want(sp, p, v), f"served job {k} {v}")
    finally:
        srv.close()

"""Per-point labels on the GPU against the oracle, element by element.

Every point gets the label of its tile's cluster (Section 4.1's per-point
variant) or -1.  The lookup table the library builds from a result is reused
by later calls; points that were not part of the clustering, empty inputs,
results without tiles and range errors are covered as well as plain, chunked
and batched results.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import dev

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


def _check(got, want, what):
    got = got.cpu().numpy()
    assert got.dtype == np.int64 and got.shape == want.shape, what
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, f"{what}: {bad.size} labels differ, first at {bad[:5]}: {got[bad[:5]]} vs {want[bad[:5]]}"


@pytest.fixture(scope="module")
def small():
    return synth.plain_small(1)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_plain_small(raster, torch, small, dtype):
    pts = small.astype(dtype)
    _say(f"point labels plain-200k {np.dtype(dtype).name}")
    o = oracle.cluster(pts, tau=5, mu=4, precision=1)
    want = oracle.point_labels(pts, o, precision=1)
    assert (want != -1).sum() > 0 and (want == -1).sum() > 0
    d = dev(pts, torch)
    g = raster.cluster(d, precision=1, tau=5, mu=4)
    _check(g.point_labels(d), want, "plain-200k")
    # the cached lookup table gives the same answer on a second call, on another stream
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        again = g.point_labels(d, stream=s)
    s.synchronize()
    _check(again, want, "plain-200k, second call")


def test_points_outside_the_clustering(raster, torch, small):
    # labels of points that were not clustered: a shifted copy and fresh noise
    o = oracle.cluster(small, tau=5, mu=4, precision=1)
    g = raster.cluster(dev(small, torch), precision=1, tau=5, mu=4)
    rng = synth.rng_for(77)
    other = np.concatenate([small[::3] + 0.05, rng.uniform(-50, 150, size=(50_001, 2))])
    _check(g.point_labels(dev(other, torch)), oracle.point_labels(other, o, precision=1), "other points")


def test_mid_binned_and_ragged(raster, torch):
    pts = synth.zipf_hot(2, n=3_000_000, block=1_000_000)
    o = oracle.cluster(pts, tau=5, mu=4, precision=2)
    want = oracle.point_labels(pts, o, precision=2)
    d = dev(pts, torch)
    g = raster.cluster(d, precision=2, tau=5, mu=4)
    _say("point labels zipf 3M")
    _check(g.point_labels(d), want, "zipf 3M")
    for n in (1, 2047, 2048, 2049, 777_777):   # ragged tails of the 2048-point step
        _check(g.point_labels(d[:n]), want[:n], f"zipf 3M prefix {n}")


def test_stream_result(raster, torch):
    centres = synth.paper_scale_centres(3)
    chunks = [synth.paper_scale_chunk(c, centres=centres, chunk=500_000) for c in range(4)]
    st = raster.Stream(tau=5, mu=4, precision=2)
    for c in chunks:
        st.feed(dev(c, torch))
    g = st.finish()
    st.close()
    o = oracle.cluster_chunks(chunks, tau=5, mu=4, precision=2)
    for k, c in enumerate(chunks):
        _check(g.point_labels(dev(c, torch)), oracle.point_labels(c, o, precision=2), f"stream chunk {k}")


def test_batch_results(raster, torch):
    specs = synth.batch_jobs(seed=4, n_jobs=8, size_scale=0.02)
    jobs = [(sp, synth.job_points(sp)) for sp in specs]
    devs = [dev(p, torch) for _, p in jobs]
    res = raster.cluster_batch([dict(points=d, precision=sp.precision, tau=sp.tau, mu=sp.mu)
                                for (sp, _), d in zip(jobs, devs)])
    for k, ((sp, p), d, g) in enumerate(zip(jobs, devs, res)):
        o = oracle.cluster(p, tau=sp.tau, mu=sp.mu, precision=sp.precision)
        _check(g.point_labels(d), oracle.point_labels(p, o, precision=sp.precision), f"batch job {k}")


def test_non_integer_scale(raster, torch, small):
    s = 10.0 ** 0.5
    o = oracle.cluster(small, tau=5, mu=2, scale=s)
    d = dev(small, torch)
    g = raster.cluster(d, scale=s, tau=5, mu=2)
    _check(g.point_labels(d), oracle.point_labels(small, o, scale=s), "scale 10^0.5")


def test_empty_and_tileless(raster, torch, small):
    d = dev(small, torch)
    g = raster.cluster(d, precision=1, tau=5, mu=4)
    assert g.point_labels(d[:0]).shape == (0,)
    none = raster.cluster(d, precision=1, tau=1_000_000, mu=1)   # no significant tile
    assert none.num_tiles == 0
    lab = none.point_labels(d).cpu().numpy()
    assert lab.shape == (small.shape[0],) and (lab == -1).all()
    e = raster.cluster(d[:0], precision=1, tau=1, mu=1)
    assert (e.point_labels(d[:1000]).cpu().numpy() == -1).all()


def test_range_error_then_recovery(raster, torch, small):
    d = dev(small, torch)
    g = raster.cluster(d, precision=1, tau=5, mu=4)
    bad = small[:10_000].copy()
    bad[5_432, 0] = np.inf
    with pytest.raises(raster.RasterError) as e:
        g.point_labels(dev(bad, torch))
    assert e.value.code == raster.E_RANGE
    big = small[:10_000].copy()
    big[17, 1] = 1e9   # 1e10 after scaling: outside the tile range
    with pytest.raises(raster.RasterError) as e:
        g.point_labels(dev(big, torch))
    assert e.value.code == raster.E_RANGE
    # the error flag is cleared for the next call
    o = oracle.cluster(small, tau=5, mu=4, precision=1)
    _check(g.point_labels(d), oracle.point_labels(small, o, precision=1), "after range errors")

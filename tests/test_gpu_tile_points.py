"""Per-tile point lists (RASTER', Section 3.4) on the GPU against the oracle.

The GPU lists each kept tile's points under the result's rows, in compaction
order and unordered within a row; the oracle lists them ascending under its
own rows.  Compared per tile as sorted lists (a tile's points form a set),
plus the row offsets, the number of listed points and the errors.
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


def _gpu_lists(g, d):
    start, index = g.tile_points(d)
    start, index = start.cpu().numpy(), index.cpu().numpy()
    kx, ky = (a.cpu().numpy() for a in g.tensors()[:2])
    assert start.shape == (g.num_tiles + 1,) and start[0] == 0 and np.all(np.diff(start) >= 0)
    assert start[-1] == index.shape[0]
    return {(int(kx[j]), int(ky[j])): np.sort(index[start[j]:start[j + 1]]) for j in range(g.num_tiles)}


def _oracle_lists(pts, o, **kw):
    start, index = oracle.tile_points(pts, o, **kw)
    return {(int(o.kx[j]), int(o.ky[j])): index[start[j]:start[j + 1]] for j in range(o.num_tiles)}


def _check(got, want, what):
    assert got.keys() == want.keys(), what
    bad = [t for t in want if not np.array_equal(got[t], want[t])]
    assert not bad, f"{what}: {len(bad)} tiles differ, first {bad[:3]}"


@pytest.fixture(scope="module")
def small():
    return synth.plain_small(1)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_plain_small(raster, torch, small, dtype):
    pts = small.astype(dtype)
    o = oracle.cluster(pts, tau=5, mu=4, precision=1)
    d = dev(pts, torch)
    g = raster.cluster(d, precision=1, tau=5, mu=4)
    _check(_gpu_lists(g, d), _oracle_lists(pts, o, precision=1), "plain-200k")
    # counts of the rows equal the listed points per row
    start, _ = g.tile_points(d)
    cnt = g.tensors()[2].cpu().numpy().astype(np.int64)
    assert np.array_equal(np.diff(start.cpu().numpy()), cnt)


def test_hot_tiles_3M(raster, torch):
    # zipf-weighted centres: tiles with up to ~10^5 points in one row
    pts = synth.zipf_hot(2, n=3_000_000, block=1_000_000)
    o = oracle.cluster(pts, tau=5, mu=4, precision=2)
    d = dev(pts, torch)
    g = raster.cluster(d, precision=2, tau=5, mu=4)
    _say("tile points zipf 3M")
    _check(_gpu_lists(g, d), _oracle_lists(pts, o, precision=2), "zipf 3M")
    for n in (1, 2047, 2049, 100_001):
        _check(_gpu_lists(g, d[:n]), _oracle_lists(pts[:n], o, precision=2), f"zipf 3M prefix {n}")


def test_stream_and_other_points(raster, torch):
    centres = synth.paper_scale_centres(3)
    chunks = [synth.paper_scale_chunk(c, centres=centres, chunk=300_000) for c in range(3)]
    st = raster.Stream(tau=5, mu=4, precision=2)
    for c in chunks:
        st.feed(dev(c, torch))
    g = st.finish()
    st.close()
    o = oracle.cluster_chunks(chunks, tau=5, mu=4, precision=2)
    for k, c in enumerate(chunks):
        _check(_gpu_lists(g, dev(c, torch)), _oracle_lists(c, o, precision=2), f"stream chunk {k}")


def test_batch_results(raster, torch):
    specs = synth.batch_jobs(seed=4, n_jobs=6, size_scale=0.02)
    jobs = [(sp, synth.job_points(sp)) for sp in specs]
    devs = [dev(p, torch) for _, p in jobs]
    res = raster.cluster_batch([dict(points=d, precision=sp.precision, tau=sp.tau, mu=sp.mu)
                                for (sp, _), d in zip(jobs, devs)])
    for k, ((sp, p), d, g) in enumerate(zip(jobs, devs, res)):
        o = oracle.cluster(p, tau=sp.tau, mu=sp.mu, precision=sp.precision)
        _check(_gpu_lists(g, d), _oracle_lists(p, o, precision=sp.precision), f"batch job {k}")


def test_empty_tileless_and_errors(raster, torch, small):
    d = dev(small, torch)
    g = raster.cluster(d, precision=1, tau=5, mu=4)
    start, index = g.tile_points(d[:0])
    assert index.shape == (0,) and (start.cpu().numpy() == 0).all()
    none = raster.cluster(d, precision=1, tau=1_000_000, mu=1)
    start, index = none.tile_points(d)
    assert start.cpu().numpy().tolist() == [0] and index.shape == (0,)
    bad = small[:5000].copy()
    bad[123, 1] = np.nan
    with pytest.raises(raster.RasterError) as e:
        g.tile_points(dev(bad, torch))
    assert e.value.code == raster.E_RANGE
    # an index buffer that is too small: E_INVAL, n_kept still reported
    import ctypes
    import torch as t
    lib = raster.load()
    st = t.empty(g.num_tiles + 1, dtype=t.int64, device="cuda")
    idx = t.empty(10, dtype=t.int64, device="cuda")
    kept = ctypes.c_int64()
    rc = lib.raster_result_tile_points(g._h, ctypes.c_void_p(d.data_ptr()), small.shape[0], 2,
                                       ctypes.c_void_p(st.data_ptr()), ctypes.c_void_p(idx.data_ptr()), 10,
                                       ctypes.byref(kept), None)
    assert rc == raster.E_INVAL
    o = oracle.cluster(small, tau=5, mu=4, precision=1)
    assert kept.value == int(o.count.sum())
    # and a good call afterwards
    _check(_gpu_lists(g, d), _oracle_lists(small, o, precision=1), "after errors")

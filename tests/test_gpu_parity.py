"""HIP path against the oracle, element by element (all integers: bit-exact).

Sizes here run in seconds; they still span many scan tiles (4096 slots),
counting workgroups and a ragged tail.  Full-size workloads are in
test_gpu_large.py.
"""
import json
import os

import numpy as np
import pytest

import oracle
import synth
from digest import biased
from gpu_util import assert_same, decode_keys, dev, same_result

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


def test_projection_pins(raster, torch):
    g = json.load(open(os.path.join(GOLDEN, "projection_pins.json")))
    for kind, dtype in (("f64", np.float64), ("f32", np.float32)):
        for case in g[kind]:
            pts = np.array([[case["x"], 0.0], [0.0, case["x"]]], dtype)
            st = raster.Stream(tau=1, mu=1, precision=case["p"])
            st.feed(dev(pts, torch))
            keys, cnts = st.tiles()
            kx, ky = decode_keys(keys.cpu().numpy())
            got = sorted(zip(kx.tolist(), ky.tolist()))
            want = sorted({(case["k"], 0), (0, case["k"])})
            assert got == want, (kind, case, got)
            st.close()


def test_worked_example_and_fig4(raster, torch):
    g = json.load(open(os.path.join(GOLDEN, "worked_example.json")))
    pts = dev(np.array(g["points"]), torch)
    r = raster.cluster(pts, precision=2, tau=3, mu=1)
    kx, ky, cnt, lab = r.numpy()
    assert (kx.tolist(), ky.tolist(), cnt.tolist()) == ([100], [100], [3])
    assert raster.cluster(pts, precision=2, tau=4, mu=1).num_tiles == 0
    f = json.load(open(os.path.join(GOLDEN, "fig4_grid_corner.json")))
    pts = dev(np.array(f["points"]), torch)
    assert raster.cluster(pts, precision=0, tau=4, mu=1).stats["significant_tiles"] == 0
    r = raster.cluster(pts, precision=0, tau=1, mu=4)
    kx, ky, cnt, lab = r.numpy()
    assert sorted(zip(kx.tolist(), ky.tolist())) == [tuple(t) for t in f["tiles"]]
    assert set(lab.tolist()) == {int(biased([0], [0])[0])}


def test_range_errors(raster, torch):
    g = json.load(open(os.path.join(GOLDEN, "projection_pins.json")))
    for case in g["range_errors"]:
        x = float(case["x"])
        for pts in (np.array([[0.5, 0.5], [x, 0.0]]), np.array([[0.0, x], [0.5, 0.5]])):
            with pytest.raises(raster.RasterError) as e:
                raster.cluster(dev(pts, torch), precision=case["p"], tau=1, mu=1)
            assert e.value.code == raster.E_RANGE
            st = raster.Stream(tau=1, mu=1, precision=case["p"])
            st.feed(dev(np.zeros((3, 2)), torch))
            with pytest.raises(raster.RasterError) as e:
                st.feed(dev(pts, torch))
                st.finish()
            assert e.value.code == raster.E_RANGE
            with pytest.raises(raster.RasterError):
                st.finish()
            st.close()


def test_stream_state_errors(raster, torch):
    st = raster.Stream(tau=1, mu=1, precision=1)
    st.feed(dev(np.ones((10, 2)), torch))
    st.finish()
    with pytest.raises(raster.RasterError) as e:
        st.feed(dev(np.ones((10, 2)), torch))
    assert e.value.code == raster.E_STATE
    with pytest.raises(raster.RasterError) as e:
        st.finish()
    assert e.value.code == raster.E_STATE
    st.close()
    st = raster.Stream(tau=1, mu=1, precision=1)
    st.feed(dev(np.ones((10, 2)), torch))
    st.close()  # destroy without finish


def _tiny_case(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(0, 400))
    span = float(rng.choice([0.3, 0.6, 1.0, 2.0]))
    centre = rng.uniform(-1.0, 1.0, size=2)
    kind = int(rng.integers(0, 3))
    if kind == 0:
        pts = centre + rng.uniform(-span, span, size=(n, 2))
    elif kind == 1:
        pts = centre + rng.normal(0.0, span / 3, size=(n, 2))
    else:
        pts = np.round((centre + rng.uniform(-span, span, size=(n, 2))) * 20) / 20
    dtype = np.float32 if rng.random() < 0.25 else np.float64
    return pts.astype(dtype), int(rng.integers(0, 3)), int(rng.integers(1, 6)), int(rng.integers(1, 6))


def test_tiny_corpus(raster, torch):
    for seed in range(300):
        pts, p, tau, mu = _tiny_case(seed)
        o = oracle.cluster(pts, tau=tau, mu=mu, precision=p)
        g = raster.cluster(dev(pts, torch), precision=p, tau=tau, mu=mu)
        assert_same(g, o, f"tiny seed {seed}")


@pytest.fixture(scope="module")
def small():
    return synth.plain_small(1)


@pytest.fixture(scope="module")
def small_oracle(small):
    return oracle.cluster(small, tau=5, mu=4, precision=1)


def test_plain_small_f64(raster, torch, small, small_oracle):
    _say("plain-200k f64")
    g = raster.cluster(dev(small, torch), precision=1, tau=5, mu=4)
    assert_same(g, small_oracle, "plain-200k f64")
    assert 90 <= g.num_clusters <= 110


def test_plain_small_f32(raster, torch, small):
    pts = small.astype(np.float32)
    o = oracle.cluster(pts, tau=5, mu=4, precision=1)
    g = raster.cluster(dev(pts, torch), precision=1, tau=5, mu=4)
    assert_same(g, o, "plain-200k f32")


def test_contraction_counts_match(raster, torch, small):
    # every (tile, count) of the device table against the oracle's accumulator
    st = raster.Stream(tau=5, mu=4, precision=1)
    st.feed(dev(small, torch))
    keys, cnts = st.tiles()
    kx, ky = decode_keys(keys.cpu().numpy())
    c = cnts.cpu().numpy().astype(np.uint64)
    order = np.lexsort((ky, kx))
    os_ = oracle.OracleStream(oracle.scale_for_precision(1), 5, 4)
    os_.feed(small)
    okx, oky, oc = os_.tile_counts()
    assert np.array_equal(kx[order], okx) and np.array_equal(ky[order], oky) and np.array_equal(c[order], oc)
    assert int(c.sum()) == small.shape[0]
    st.close()


@pytest.mark.parametrize("block,items,preagg,lf", [
    (64, 1, 0, 0.5), (256, 16, 0, 0.25), (1024, 4, 0, 0.9), (256, 4, 1024, 0.5), (512, 8, 4096, 0.7),
    (128, 2, 256, 0.1),
])
def test_launch_configs_agree(raster, torch, small, small_oracle, block, items, preagg, lf):
    raster.set_tuning(block=block, items=items, preagg_slots=preagg, load_factor=lf)
    try:
        g = raster.cluster(dev(small, torch), precision=1, tau=5, mu=4)
    finally:
        raster.set_tuning(None)
    assert_same(g, small_oracle, f"tuning {block},{items},{preagg},{lf}")


def test_table_growth(raster, torch, small, small_oracle):
    # a tiny table forces spills, growth and rehashing, across several chunks
    st = raster.Stream(tau=5, mu=4, precision=1, tile_hint=1)
    for c in np.array_split(small, 5):
        st.feed(dev(c, torch))
    g = st.finish()
    assert g.stats["grow_events"] >= 1
    assert_same(g, small_oracle, "grown table")
    st.close()


@pytest.mark.parametrize("k", [1, 2, 7, 10])
def test_chunk_and_order_invariance(raster, torch, small, small_oracle, k):
    rng = np.random.default_rng(100 + k)
    cuts = np.sort(rng.choice(np.arange(1, small.shape[0]), size=k - 1, replace=False))
    chunks = np.split(small, cuts)
    st = raster.Stream(tau=5, mu=4, precision=1, tile_hint=20000)
    for i in rng.permutation(len(chunks)):
        st.feed(dev(chunks[i], torch))
    g = st.finish()
    assert_same(g, small_oracle, f"{k} chunks")
    st.close()


def test_repeatable(raster, torch, small):
    a = raster.cluster(dev(small, torch), precision=1, tau=5, mu=4)
    b = raster.cluster(dev(small, torch), precision=1, tau=5, mu=4)
    same_result(a, b, "repeat")


def test_empty_inputs(raster, torch):
    r = raster.cluster(dev(np.zeros((0, 2)), torch), precision=2, tau=1, mu=1)
    assert r.num_tiles == 0 and r.stats["distinct_tiles"] == 0
    st = raster.Stream(tau=1, mu=1, precision=2)
    r = st.finish()
    assert r.num_tiles == 0
    st.close()


def test_one_hot_tile(raster, torch):
    # every point on one tile: contended atomics on a single slot
    n = 3_000_000
    rng = np.random.default_rng(7)
    pts = 5.0 + rng.uniform(0.0, 0.99, size=(n, 2))
    for preagg in (0, 2048):
        raster.set_tuning(preagg_slots=preagg)
        try:
            r = raster.cluster(dev(pts, torch), precision=0, tau=n, mu=1)
        finally:
            raster.set_tuning(None)
        kx, ky, cnt, lab = r.numpy()
        assert (kx.tolist(), ky.tolist(), cnt.tolist()) == ([5], [5], [n])


def test_extreme_tiles(raster, torch):
    # tiles at the edge of the valid range, where neighbour lookups must be
    # skipped rather than wrap around, plus a cluster straddling the origin
    big = 2147483646.5
    pts = []
    for x, y in [(big, big), (big - 1, big), (big, big - 1), (-big, -big), (-big + 1, -big),
                 (big, -big), (-big, big), (0.5, 0.5), (-0.5, 0.5), (-1.5, -1.5)]:
        pts += [[x, y]] * 3
    pts = np.array(pts)
    o = oracle.cluster(pts, tau=3, mu=1, precision=0)
    g = raster.cluster(dev(pts, torch), precision=0, tau=3, mu=1)
    assert_same(g, o, "extreme tiles")


def test_non_integer_scale(raster, torch, small):
    s = 10.0 ** 0.5
    o = oracle.cluster(small, tau=5, mu=2, scale=s)
    g = raster.cluster(dev(small, torch), scale=s, tau=5, mu=2)
    assert_same(g, o, "scale 10^0.5")


@pytest.fixture(scope="module")
def mid():
    # 3M points with hot tiles and noise: large enough for the binned path
    return synth.zipf_hot(2, n=3_000_000, block=1_000_000)


@pytest.fixture(scope="module")
def mid_oracle(mid):
    return oracle.cluster(mid, tau=5, mu=4, precision=2)


@pytest.mark.parametrize("mode,group,hint,chunks", [
    (2, 1, 2_000_000, 1),    # binned, three flushes of one million points
    (2, 1, 2_000_000, 7),    # binned, uneven chunks straddling flushes
    (2, 1, 300_000, 3),      # binned into a table that must grow with keys in flight
    (2, 2, 0, 5),            # binned, table sized from the first chunk
    (1, 256, 0, 3),          # direct
    (0, 256, 0, 1),          # automatic choice
])
def test_counting_paths_agree(raster, torch, mid, mid_oracle, mode, group, hint, chunks):
    raster.set_tuning(mode=mode, group_mpoints=group)
    try:
        st = raster.Stream(tau=5, mu=4, precision=2, tile_hint=hint)
        for c in np.array_split(mid, chunks):
            st.feed(dev(c, torch))
        g = st.finish()
        st.close()
    finally:
        raster.set_tuning(None)
    assert_same(g, mid_oracle, f"mode {mode} group {group} hint {hint} chunks {chunks}")
    if mode == 2 and hint >= 2_000_000:
        assert g.stats["flushes"] >= 3
    if mode == 1:
        assert g.stats["flushes"] == 0


def test_plain_binned_auto(raster, torch, mid, mid_oracle):
    g = raster.cluster(dev(mid, torch), precision=2, tau=5, mu=4)
    assert g.stats["flushes"] >= 1
    assert_same(g, mid_oracle, "plain 3M auto")


def test_binned_f32(raster, torch, mid):
    pts = mid.astype(np.float32)
    o = oracle.cluster(pts, tau=5, mu=4, precision=2)
    raster.set_tuning(mode=2)
    try:
        g = raster.cluster(dev(pts, torch), precision=2, tau=5, mu=4)
    finally:
        raster.set_tuning(None)
    assert g.stats["flushes"] >= 1
    assert_same(g, o, "binned f32")


def test_binned_range_error(raster, torch, mid):
    bad = mid[:1_000_000].copy()
    bad[777_777, 1] = np.nan
    raster.set_tuning(mode=2)
    try:
        with pytest.raises(raster.RasterError) as e:
            raster.cluster(dev(bad, torch), precision=2, tau=5, mu=4)
    finally:
        raster.set_tuning(None)
    assert e.value.code == raster.E_RANGE


def test_stream_range_error_in_a_middle_chunk(raster, torch, mid):
    # binned chunks go in without waiting for the previous chunk's counters;
    # a bad coordinate in a middle chunk must still fail the stream, by
    # finish at the latest, and every later call must report it
    chunks = [c.copy() for c in np.array_split(mid[:1_200_000], 6)]
    chunks[2][1234, 0] = np.nan
    raster.set_tuning(mode=2)
    try:
        st = raster.Stream(tau=5, mu=4, precision=2, tile_hint=500_000)
        with pytest.raises(raster.RasterError) as e:
            for c in chunks:
                st.feed(dev(c, torch))
            st.finish()
        assert e.value.code == raster.E_RANGE
        with pytest.raises(raster.RasterError):
            st.finish()
        st.close()
    finally:
        raster.set_tuning(None)


def test_stream_whose_tiles_keep_growing(raster, torch):
    # every chunk covers its own region, so the distinct tiles grow with each
    # chunk far past the first chunk's guess; the sketch taken while binning
    # sizes the table at the flush (no spill-and-grow), and the result is the
    # oracle's
    chunks = []
    for c in range(8):
        rng = synth.rng_for(300 + c)
        centres = rng.uniform(0.0, 100.0, size=(2000, 2)) + np.array([200.0 * c, 0.0])
        pts = centres[rng.integers(0, 2000, size=500_000)] + rng.normal(0.0, 0.05, size=(500_000, 2))
        chunks.append(np.ascontiguousarray(pts))
    raster.set_tuning(mode=2)
    try:
        st = raster.Stream(tau=3, mu=2, precision=2)
        for c in chunks:
            st.feed(dev(c, torch))
        g = st.finish()
        st.close()
    finally:
        raster.set_tuning(None)
    o = oracle.cluster_chunks(chunks, tau=3, mu=2, precision=2)
    assert g.stats["distinct_tiles"] > 4 * 250_000
    assert g.stats["grow_events"] <= 1, g.stats
    assert_same(g, o, "stream with growing tiles")


def test_repeated_runs_identical(raster, torch, mid, mid_oracle):
    # races in the union-find passes show up as run-to-run differences
    d = dev(mid, torch)
    for rep in range(6):
        g = raster.cluster(d, precision=2, tau=5, mu=4)
        assert_same(g, mid_oracle, f"repeat {rep}")


def test_dense_uniform_grid(raster, torch):
    """Mostly-singleton tiles: 3M uniform points over 1000 x 1000 tiles (p = 1).
    The table-size guess (n/8 distinct) is far too small, so the binned path
    spills, grows and re-inserts; results must not change."""
    rng = synth.rng_for(11)
    pts = rng.uniform(0.0, 100.0, size=(3_000_000, 2))
    _say(f"dense uniform grid: {pts.shape[0]} points")
    for mode in (0, 2):
        raster.set_tuning(mode=mode)
        try:
            r = raster.cluster(dev(pts, torch), precision=1, tau=3, mu=4)
        finally:
            raster.set_tuning(None)
        assert r.stats["distinct_tiles"] > 900_000
        assert_same(r, oracle.cluster(pts, tau=3, mu=4, precision=1), f"dense uniform grid, mode {mode}")

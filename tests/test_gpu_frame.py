"""The key frame of a two-dimensional table, against the oracle.

When a sample of the first binned chunk shows the tiles within a window of
2^20 x 2^20, the table places its keys by their position in that window and
the binned contraction moves 4-byte entries that give the keys back.  Keys
outside the frame go into the table directly and stay where an unframed
table would put them.  None of this may change a result (Algorithm 1;
Section 3.6: chunks in any order give the same clusters):

* streams whose later chunks lie far outside the frame (keys placed both
  ways in one table), with several flushes, so that partitions holding
  foreign keys are read back and updated;
* the framed fallback that inserts entries directly (tables whose partition
  count is outside the framed binning's range), and growth by rehashing;
* frames clamped at both ends of the tile range;
* FP32 chunks;
* framed and unframed (tuning mode 3) binning on the same input;
* inputs too wide for a frame;
* the census of significant tiles at table sizes below, at and above one
  partition per census block.
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


def run_stream(raster, torch, chunks, precision, tau, mu, tile_hint=0, **tuning):
    if tuning:
        raster.set_tuning(**tuning)
    try:
        st = raster.Stream(tau=tau, mu=mu, precision=precision, tile_hint=tile_hint)
        for c in chunks:
            st.feed(dev(c, torch))
        res = st.finish()
        st.close()
    finally:
        raster.set_tuning(None)
    return res


def blob_box(seed, n, lo, hi, n_centres=200, sigma=0.02, noise=0.05, dtype=np.float64):
    rng = synth.rng_for(seed)
    pts = synth.blobs(rng, n, n_centres, hi - lo, sigma, noise) + lo
    return np.ascontiguousarray(pts.astype(dtype))


def test_paper_like_stream_framed(raster, torch):
    centres = synth.paper_scale_centres(3)
    chunks = [synth.paper_scale_chunk(c, centres=centres, chunk=1_000_000) for c in range(6)]
    chunks[3] = np.ascontiguousarray(chunks[3].astype(np.float32))
    _say("frame: paper-like stream 6 x 1M (one chunk FP32)")
    res = run_stream(raster, torch, chunks, 2, 5, 4)
    assert res.stats["key_frame"] == 1 and res.stats["flushes"] >= 1
    ref = oracle.cluster_chunks(chunks, tau=5, mu=4, precision=2)
    assert_same(res, ref, "paper-like framed")
    unframed = run_stream(raster, torch, chunks, 2, 5, 4, mode=3)
    assert unframed.stats["key_frame"] == 0
    same_result(res, unframed, "framed vs unframed binning")


def _near_far_chunks():
    near = [blob_box(7200 + i, 600_000, 0.0, 100.0) for i in range(3)]
    # 20000 at p=2 is tile 2,000,000: far outside any frame around [0, 100]
    far = [blob_box(7300 + i, 600_000, 20_000.0, 20_100.0) for i in range(2)]
    return [near[0], far[0], near[1], far[1], near[2]]


@pytest.mark.parametrize("order", ["near-first", "far-first"])
def test_keys_outside_the_frame_and_several_flushes(raster, torch, order):
    chunks = _near_far_chunks()
    if order == "far-first":
        chunks = chunks[::-1][1:] + chunks[-1:]  # starts with a far chunk
    ref = oracle.cluster_chunks(chunks, tau=5, mu=4, precision=2)
    # one million points per flush: later flushes read back partitions that
    # hold keys placed outside the frame.  The table is filled only when first
    # needed, so the first keys outside the frame wait in the spill buffer;
    # without a hint the first chunk's guess sizes the table, and then one
    # group holds the whole stream (one flush, the final update)
    for hint, group, flushes in ((600_000, 1, 3), (0, 0, 1)):
        _say(f"frame: near/far stream ({order}), tile hint {hint}")
        tuning = dict(mode=2, group_mpoints=group) if group else dict(mode=2)
        res = run_stream(raster, torch, chunks, 2, 5, 4, tile_hint=hint, **tuning)
        assert res.stats["key_frame"] == 1
        assert res.stats["flushes"] >= flushes
        assert_same(res, ref, f"near/far {order}, hint {hint}")


def test_framed_direct_fallback_and_growth(raster, torch):
    # a table of 2^19 slots has 128 partitions: too few for the framed
    # binning (256 coarse buckets), so the entries are inserted directly
    pts = blob_box(7400, 300_000, 0.0, 50.0)
    _say("frame: direct fallback")
    res = run_stream(raster, torch, [pts[:150_000], pts[150_000:]], 2, 3, 2, tile_hint=200_000, mode=2)
    assert res.stats["key_frame"] == 1 and res.stats["table_capacity"] == 1 << 19
    assert_same(res, oracle.cluster(pts, tau=3, mu=2, precision=2), "framed fallback")
    # growth: a clustered first chunk sizes the table, then a chunk of
    # mostly distinct tiles inside the same box makes it grow by rehashing
    a = blob_box(7401, 1_200_000, 0.0, 1000.0, n_centres=300, sigma=0.01, noise=0.0)
    b = blob_box(7402, 3_000_000, 0.0, 1000.0, n_centres=10, sigma=0.01, noise=0.9)
    _say("frame: growth")
    # one million points per flush: the table holds keys when it has to grow
    res = run_stream(raster, torch, [a, b, a[:500_000]], 2, 4, 3, group_mpoints=1)
    assert res.stats["key_frame"] == 1 and res.stats["grow_events"] >= 1
    assert_same(res, oracle.cluster_chunks([a, b, a[:500_000]], tau=4, mu=3, precision=2), "framed growth")


@pytest.mark.parametrize("side", ["top", "bottom"])
def test_frame_at_the_ends_of_the_tile_range(raster, torch, side):
    # tiles up to 2^31 - 10 (or down to -(2^31 - 10)) at p=2
    edge = (2 ** 31 - 10) / 100.0
    lo, hi = (edge - 60.0, edge) if side == "top" else (-edge, -edge + 60.0)
    pts = blob_box(7500 + (side == "top"), 1_500_000, lo, hi, n_centres=100)
    pts = np.clip(pts, -edge, edge)
    _say(f"frame: {side} of the tile range")
    res = run_stream(raster, torch, [pts[:700_000], pts[700_000:]], 2, 5, 4, tile_hint=700_000, mode=2)
    assert res.stats["key_frame"] == 1
    assert_same(res, oracle.cluster(pts, tau=5, mu=4, precision=2), f"frame {side}")


def test_too_wide_for_a_frame(raster, torch):
    # 5000 units at p=3 span 5M tiles per axis
    pts = blob_box(7600, 2_000_000, 0.0, 5000.0, n_centres=400, sigma=0.002, noise=0.02)
    _say("frame: too wide")
    res = raster.cluster(dev(pts, torch), precision=3, tau=5, mu=4)
    assert res.stats["key_frame"] == 0
    assert_same(res, oracle.cluster(pts, tau=5, mu=4, precision=3), "unframed wide input")
    framed_size = blob_box(7601, 2_000_000, 0.0, 500.0, n_centres=400, sigma=0.002, noise=0.02)
    res = raster.cluster(dev(framed_size, torch), precision=3, tau=5, mu=4)
    assert res.stats["key_frame"] == 1
    assert_same(res, oracle.cluster(framed_size, tau=5, mu=4, precision=3), "framed plain call")


def test_partition_overflow_at_high_load(raster, torch):
    """A stream kept at about 80% table load (a stream keeps its table until
    the sketch shows it 85% full): partitions overflow in the LDS update,
    whose spilled entries make the table grow and are inserted again.
    Results must not change."""
    rng = synth.rng_for(7700)
    # about 800K distinct tiles of 1 x 1 (p=0) in a 2^20-slot table
    pts = rng.uniform(0.0, 2000.0, size=(900_000, 2))
    chunks = [np.ascontiguousarray(pts[i::3]) for i in range(3)]
    _say("frame: final update at high load")
    res = run_stream(raster, torch, chunks, 0, 2, 2, tile_hint=600_000, mode=2)
    assert res.stats["key_frame"] == 1
    assert res.stats["distinct_tiles"] > 700_000
    assert_same(res, oracle.cluster_chunks(chunks, tau=2, mu=2, precision=0), "high-load final update")


@pytest.mark.parametrize("square", [False, True])
def test_census_table_sizes(raster, torch, square):
    """Framed tables of 512 partitions and more find their significant tiles
    by a census counted in blocks of whole partitions (one partition or
    fewer per block below 2048 partitions, several above).  Tables of 2^21,
    2^23 and 2^24 slots hold the same points; every result must equal the
    oracle's (Algorithm 1; with the 2x2 post-step of Section 3.3 too)."""
    pts = blob_box(7800, 400_000, 0.0, 80.0, n_centres=150, sigma=0.03, noise=0.1)
    chunks = [pts[:250_000], pts[250_000:]]
    ref = oracle.cluster_chunks(chunks, tau=4, mu=3, precision=2, window=square)
    for hint in (1_000_000, 4_000_000, 9_000_000):
        _say(f"frame: census, tile hint {hint}, square {square}")
        raster.set_tuning(mode=2)  # binned chunks (the frame is chosen by the first one)
        try:
            st = raster.Stream(tau=4, mu=3, precision=2, tile_hint=hint, square=square)
            for c in chunks:
                st.feed(dev(c, torch))
            res = st.finish()
            st.close()
        finally:
            raster.set_tuning(None)
        assert res.stats["key_frame"] == 1
        assert res.stats["table_capacity"] >= 1 << 21
        assert_same(res, ref, f"census, {res.stats['table_capacity']} slots, square {square}")


def test_final_update_image_then_growth(raster, torch):
    """The final update of a table of 512+ partitions writes a slice image
    instead of the table.  When it spills at high load, the table is rebuilt
    from the image before it grows; results must not change (Algorithm 1)."""
    rng = synth.rng_for(7900)
    # about 1.6M distinct tiles of 1 x 1 (p=0) in a table of 2^21 slots
    pts = rng.uniform(0.0, 2200.0, size=(1_900_000, 2))
    chunks = [np.ascontiguousarray(pts[i::3]) for i in range(3)]
    _say("frame: final update image, then growth")
    res = run_stream(raster, torch, chunks, 0, 2, 2, tile_hint=1_200_000, mode=2)
    assert res.stats["key_frame"] == 1
    assert res.stats["grow_events"] >= 1, "the final update did not spill"
    assert_same(res, oracle.cluster_chunks(chunks, tau=2, mu=2, precision=0), "image, then growth")

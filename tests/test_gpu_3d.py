"""Three-dimensional points on the GPU against the oracle (Section 3.6).

Section 3.6 generalises RASTER to d dimensions: tiles are d-tuples and a tile
has 3^d - 1 neighbours (2d at Manhattan distance 1).  In 3-D the GPU packs the
three biased coordinates into one 64-bit key (21 bits each); every case is
compared row by row (kx, ky, kz, count, label) and by statistics with the
oracle.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import dev

pytestmark = pytest.mark.gpu

B3 = 1 << 20


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


def _label3(lx, ly, lz):
    lx, ly, lz = (np.asarray(a, dtype=np.int64) + B3 for a in (lx, ly, lz))
    return ((lx.astype(np.uint64) << np.uint64(42)) | (ly.astype(np.uint64) << np.uint64(21))
            | lz.astype(np.uint64))


def _same3(g, o, what):
    kx, ky, kz, cnt, lab = g.numpy(sort=True)
    assert kx.shape[0] == o.num_tiles, f"{what}: {kx.shape[0]} rows vs {o.num_tiles}"
    for name, a, b in (("kx", kx, o.kx), ("ky", ky, o.ky), ("kz", kz, o.kz), ("count", cnt, o.count),
                       ("label", lab.astype(np.uint64), _label3(o.label_x, o.label_y, o.label_z))):
        a = np.asarray(a).astype(np.int64 if name != "label" else np.uint64)
        b = np.asarray(b).astype(np.int64 if name != "label" else np.uint64)
        bad = np.nonzero(a != b)[0]
        assert bad.size == 0, f"{what}: {name} differs at {bad.size} rows, first {bad[:5]}"
    st = g.stats
    for k_g, k_o in (("distinct_tiles", "distinct"), ("significant_tiles", "significant"),
                     ("clusters", "clusters"), ("tiles", "tiles"), ("n_points", "n")):
        assert int(st[k_g]) == int(o.stats[k_o]), f"{what}: {k_g} {st[k_g]} vs {o.stats[k_o]}"


def _tiny3(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(0, 300))
    centre = rng.uniform(-1.0, 1.0, size=3)
    pts = centre + rng.normal(0.0, float(rng.choice([0.2, 0.4, 0.8])), size=(n, 3))
    dtype = np.float32 if rng.random() < 0.25 else np.float64
    return pts.astype(dtype), int(rng.integers(0, 2)), int(rng.integers(1, 4)), int(rng.integers(1, 5))


@pytest.mark.parametrize("metric,delta", [("chebyshev", 1), ("manhattan", 1), ("chebyshev", 2), ("manhattan", 3)])
def test_tiny_corpus(raster, torch, metric, delta):
    for seed in range(7000, 7060):
        pts, p, tau, mu = _tiny3(seed)
        o = oracle.cluster(pts, tau=tau, mu=mu, precision=p, metric=metric, delta=delta, dims=3)
        g = raster.cluster(dev(pts, torch), precision=p, tau=tau, mu=mu, metric=metric, delta=delta)
        _same3(g, o, f"tiny 3-D seed {seed} {metric} {delta}")


@pytest.mark.parametrize("metric,delta", [("chebyshev", 4), ("manhattan", 8), ("chebyshev", 8)])
def test_wide_neighbourhoods(raster, torch, metric, delta):
    # many link groups (Chebyshev 8 in 3-D: 2456 backward offsets, 154 groups)
    for seed in range(7200, 7206):
        pts, p, tau, mu = _tiny3(seed)
        o = oracle.cluster(pts, tau=tau, mu=mu, precision=p, metric=metric, delta=delta, dims=3)
        g = raster.cluster(dev(pts, torch), precision=p, tau=tau, mu=mu, metric=metric, delta=delta)
        _same3(g, o, f"tiny 3-D seed {seed} {metric} {delta}")


def test_neighbour_counts_section_3_6(raster, torch):
    units = [(dx, dy, dz) for dx in (-1, 0, 1) for dy in (-1, 0, 1) for dz in (-1, 0, 1) if (dx, dy, dz) != (0, 0, 0)]
    for metric, want in (("chebyshev", 26), ("manhattan", 6)):
        joined = 0
        for dx, dy, dz in units:
            pts = np.array([[5.05, 5.05, 5.05], [5.05 + dx / 10, 5.05 + dy / 10, 5.05 + dz / 10]])
            joined += raster.cluster(dev(pts, torch), precision=1, tau=1, mu=1, metric=metric).num_clusters == 1
        assert joined == want, metric


@pytest.fixture(scope="module")
def mid3():
    return synth.blobs3d(21, n=3_000_000, n_centres=3000, box=100.0, sigma=0.15, noise_frac=0.05)


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_blobs_3M_counting_paths(raster, torch, mid3, mode):
    o = oracle.cluster(mid3, tau=4, mu=3, precision=1)
    raster.set_tuning(mode=mode)
    try:
        g = raster.cluster(dev(mid3, torch), precision=1, tau=4, mu=3)
    finally:
        raster.set_tuning(None)
    _say(f"3-D blobs 3M mode {mode}: {g.num_clusters} clusters")
    assert g.num_clusters > 1000
    _same3(g, o, f"3-D blobs 3M mode {mode}")


def test_f32_and_manhattan(raster, torch, mid3):
    pts = mid3[:500_000].astype(np.float32)
    o = oracle.cluster(pts, tau=2, mu=2, precision=1, metric="manhattan", delta=2)
    g = raster.cluster(dev(pts, torch), precision=1, tau=2, mu=2, metric="manhattan", delta=2)
    _same3(g, o, "3-D f32 manhattan 2")


def test_stream(raster, torch, mid3):
    chunks = np.array_split(mid3[:1_200_000], 5)
    st = raster.Stream(tau=3, mu=3, precision=1, dims=3)
    for c in chunks:
        st.feed(dev(np.ascontiguousarray(c), torch))
    g = st.finish()
    st.close()
    _same3(g, oracle.cluster_chunks(chunks, tau=3, mu=3, precision=1, dims=3), "3-D stream")


@pytest.mark.parametrize("mode,group,hint,chunks", [
    (2, 1, 50_000, 3),     # binned, flushes of one million points into a table that must grow with keys in it
    (2, 1, 0, 7),          # binned, uneven chunks straddling flushes
    (1, 256, 20_000, 4),   # direct counting, growth by spills
])
def test_stream_growth_paths(raster, torch, mid3, mode, group, hint, chunks):
    # growing a 3-D table rehashes its keys: home slots and partitions must
    # follow the 3-D placement there too
    pts = mid3[:2_500_000]
    raster.set_tuning(mode=mode, group_mpoints=group)
    try:
        st = raster.Stream(tau=3, mu=3, precision=1, dims=3, tile_hint=hint)
        for c in np.array_split(pts, chunks):
            st.feed(dev(np.ascontiguousarray(c), torch))
        g = st.finish()
        st.close()
    finally:
        raster.set_tuning(None)
    _say(f"3-D stream mode {mode} group {group} hint {hint}: {g.stats['grow_events']} growths, "
         f"{g.stats['flushes']} flushes")
    if hint:
        assert g.stats["grow_events"] >= 1
    _same3(g, oracle.cluster(pts, tau=3, mu=3, precision=1), f"3-D stream mode {mode} group {group} hint {hint}")


def test_range_edges_and_errors(raster, torch):
    lim = B3 - 2
    tiles = [(lim, lim, lim), (lim - 1, lim, lim), (-lim, -lim, -lim), (-lim + 1, -lim + 1, -lim + 1),
             (lim, -lim, 0), (0, 0, 0), (1, 1, 1)]
    pts = np.array([[c + 0.5 if c >= 0 else c - 0.5 for c in t] for t in tiles])
    for metric, delta in (("chebyshev", 1), ("chebyshev", 2), ("manhattan", 3)):
        o = oracle.cluster(pts, tau=1, mu=1, precision=0, metric=metric, delta=delta)
        g = raster.cluster(dev(pts, torch), precision=0, tau=1, mu=1, metric=metric, delta=delta)
        _same3(g, o, f"3-D range edges {metric} {delta}")
    for bad in ([[0.5, 0.5, B3 - 0.5]], [[-(B3 - 0.5), 0.5, 0.5]], [[0.5, np.inf, 0.5]]):
        with pytest.raises(raster.RasterError) as e:
            raster.cluster(dev(np.array(bad), torch), precision=0, tau=1, mu=1)
        assert e.value.code == raster.E_RANGE


def test_unsupported_combinations(raster, torch):
    pts = dev(np.array([[0.5, 0.5, 0.5]] * 4), torch)
    with pytest.raises(raster.RasterError) as e:
        raster.cluster(pts, precision=1, tau=1, mu=1, square=True)
    assert e.value.code == raster.E_INVAL
    g = raster.cluster(pts, precision=1, tau=1, mu=1)
    assert g.dims == 3 and g.num_tiles == 1
    # the points of a 3-D result's lookups have three coordinates
    with pytest.raises(ValueError):
        g.point_labels(dev(np.array([[0.5, 0.5]]), torch))
    with pytest.raises(ValueError):
        g.tile_points(dev(np.array([[0.5, 0.5]]), torch))


# ---- per-point labels (Section 4.1) and per-tile point lists (Section 3.4) in 3-D

def _lists3(g, d):
    start, index = g.tile_points(d)
    start, index = start.cpu().numpy(), index.cpu().numpy()
    kx, ky, cnt, _ = (a.cpu().numpy() for a in g.tensors())
    kz = g.kz().cpu().numpy()
    assert start.shape == (g.num_tiles + 1,) and start[0] == 0 and start[-1] == index.shape[0]
    return {(int(kx[j]), int(ky[j]), int(kz[j])): np.sort(index[start[j]:start[j + 1]]) for j in range(g.num_tiles)}


def _oracle_lists3(pts, o, **kw):
    start, index = oracle.tile_points(pts, o, **kw)
    return {(int(o.kx[j]), int(o.ky[j]), int(o.kz[j])): index[start[j]:start[j + 1]] for j in range(o.num_tiles)}


def _check_lists(got, want, what):
    assert got.keys() == want.keys(), what
    bad = [t for t in want if not np.array_equal(got[t], want[t])]
    assert not bad, f"{what}: {len(bad)} tiles differ, first {bad[:3]}"


def test_point_labels_and_lists_tiny(raster, torch):
    for seed in range(7100, 7140):
        pts, p, tau, mu = _tiny3(seed)
        o = oracle.cluster(pts, tau=tau, mu=mu, precision=p, dims=3)
        d = dev(pts, torch)
        g = raster.cluster(d, precision=p, tau=tau, mu=mu)
        want = oracle.point_labels(pts, o, precision=p)
        assert np.array_equal(g.point_labels(d).cpu().numpy(), want), seed
        _check_lists(_lists3(g, d), _oracle_lists3(pts, o, precision=p), f"tiny 3-D seed {seed}")


def test_point_labels_blobs_3M(raster, torch, mid3):
    o = oracle.cluster(mid3, tau=4, mu=3, precision=1)
    d = dev(mid3, torch)
    g = raster.cluster(d, precision=1, tau=4, mu=3)
    got = g.point_labels(d).cpu().numpy()
    want = oracle.point_labels(mid3, o, precision=1)
    _say(f"3-D labels 3M: {(want != -1).sum()} labelled")
    assert (want != -1).sum() > 1_000_000 and (want == -1).sum() > 10_000
    assert np.array_equal(got, want)
    # labels agree with the rows' labels
    _, _, _, _, lab = g.numpy()
    assert set(np.unique(got[got != -1]).tolist()) == set(np.unique(lab.astype(np.int64)).tolist())
    # points that were not clustered, in FP32: a prefix and shifted copies
    other = (mid3[:400_000] + np.array([0.05, -0.05, 0.1])).astype(np.float32)
    assert np.array_equal(g.point_labels(dev(other, torch)).cpu().numpy(),
                          oracle.point_labels(other, o, precision=1))


def test_tile_points_blobs_3M(raster, torch, mid3):
    pts = mid3[:1_500_000]
    o = oracle.cluster(pts, tau=4, mu=3, precision=1)
    d = dev(pts, torch)
    g = raster.cluster(d, precision=1, tau=4, mu=3)
    _check_lists(_lists3(g, d), _oracle_lists3(pts, o, precision=1), "3-D tile points 1.5M")
    start, _ = g.tile_points(d)
    assert np.array_equal(np.diff(start.cpu().numpy()), g.tensors()[2].cpu().numpy().astype(np.int64))


def test_stream_labels_and_range_errors(raster, torch, mid3):
    chunks = [np.ascontiguousarray(c) for c in np.array_split(mid3[:900_000], 3)]
    st = raster.Stream(tau=3, mu=3, precision=1, dims=3)
    for c in chunks:
        st.feed(dev(c, torch))
    g = st.finish()
    st.close()
    o = oracle.cluster_chunks(chunks, tau=3, mu=3, precision=1, dims=3)
    for k, c in enumerate(chunks):
        assert np.array_equal(g.point_labels(dev(c, torch)).cpu().numpy(), oracle.point_labels(c, o, precision=1)), k
    for bad in ([[0.5, 0.5, (B3 - 0.5) / 10]], [[np.nan, 0.5, 0.5]]):
        pts = np.concatenate([chunks[0][:1000], np.array(bad)])
        with pytest.raises(raster.RasterError) as e:
            g.point_labels(dev(pts, torch))
        assert e.value.code == raster.E_RANGE
        with pytest.raises(raster.RasterError) as e:
            g.tile_points(dev(pts, torch))
        assert e.value.code == raster.E_RANGE
    # a tile at the edge of the range is fine
    edge = np.array([[0.05, 0.05, (B3 - 2.5) / 10]])
    assert g.point_labels(dev(edge, torch)).cpu().numpy().tolist() == [-1]

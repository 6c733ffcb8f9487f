"""Full-size workloads on the GPU.

* zipf-50M (50M FP64 points, hot tiles) is compared with the oracle in full.
* The paper-scale stream (500M FP64 points in ten 50M chunks, as timed by the
  benchmark) is too large for the full oracle within a test, so it is checked
  through properties that hold at any size and through sampled clusters: for
  each sampled cluster the oracle counts, one by one, the points on the
  cluster's tiles and on every tile around them, and the test checks that the
  cluster is exactly a connected component of significant tiles with the
  right counts, size and label.
* A scaled-down copy of the same stream (ten 2M chunks) is compared in full.
"""
import numpy as np
import pytest

import oracle
import synth
from digest import biased
from gpu_util import assert_same, dev

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
    return r


def _say(msg):
    print(msg, flush=True)


def test_zipf_50M_full(raster, torch):
    _say("zipf-50M: generating")
    pts = synth.zipf_hot(2)
    d = dev(pts, torch)
    _say("zipf-50M: GPU")
    g = raster.cluster(d, precision=2, tau=5, mu=4)
    _say("zipf-50M: oracle")
    o = oracle.cluster(pts, tau=5, mu=4, precision=2)
    assert_same(g, o, "zipf-50M")
    del d
    torch.cuda.empty_cache()


def test_paper_stream_scaled_full(raster, torch):
    centres = synth.paper_scale_centres(3)
    chunks = [synth.paper_scale_chunk(c, centres=centres, chunk=2_000_000) for c in range(10)]
    _say("paper-stream 10x2M: GPU")
    st = raster.Stream(tau=5, mu=4, precision=2)
    for c in chunks:
        st.feed(dev(c, torch))
    g = st.finish()
    st.close()
    _say("paper-stream 10x2M: oracle")
    o = oracle.cluster_chunks(chunks, tau=5, mu=4, precision=2)
    assert_same(g, o, "paper-stream 10x2M")


def _components(tiles):
    """Connected components (Chebyshev 1) of a small set of (x, y) tiles."""
    tiles = set(tiles)
    seen, comps = set(), []
    for t in tiles:
        if t in seen:
            continue
        stack, comp = [t], []
        seen.add(t)
        while stack:
            u = stack.pop()
            comp.append(u)
            for dx in (-1, 0, 1):
                for dy in (-1, 0, 1):
                    v = (u[0] + dx, u[1] + dy)
                    if v in tiles and v not in seen:
                        seen.add(v)
                        stack.append(v)
        comps.append(comp)
    return comps


def test_paper_stream_full_size_sampled(raster, torch):
    n_chunks, chunk, tau, mu = 10, 50_000_000, 5, 4
    centres = synth.paper_scale_centres(3)
    host, devs = [], []
    for c in range(n_chunks):
        _say(f"paper-500M: chunk {c}")
        h = synth.paper_scale_chunk(c, centres=centres, chunk=chunk)
        host.append(h)
        devs.append(dev(h, torch))
    _say("paper-500M: GPU stream")
    st = raster.Stream(tau=tau, mu=mu, precision=2, tile_hint=40_000_000)
    for d in devs:
        st.feed(d)
    g = st.finish()
    st.close()
    del devs
    torch.cuda.empty_cache()
    stats = g.stats
    assert stats["n_points"] == n_chunks * chunk
    assert stats["distinct_tiles"] <= stats["n_points"]
    kx, ky, cnt, lab = g.numpy(sort=True)
    kx, ky, cnt = kx.astype(np.int64), ky.astype(np.int64), cnt.astype(np.int64)
    assert kx.shape[0] == stats["tiles"] and stats["clusters"] > 900_000
    # every output tile meets tau; clusters meet mu and carry their min key
    assert cnt.min() >= tau
    keys = biased(kx, ky)
    order = np.argsort(lab, kind="stable")
    lab_s, keys_s = lab[order], keys[order]
    starts = np.r_[0, np.nonzero(np.diff(lab_s))[0] + 1]
    sizes = np.diff(np.r_[starts, lab_s.shape[0]])
    assert starts.shape[0] == stats["clusters"]
    assert sizes.min() >= mu
    assert np.array_equal(np.minimum.reduceat(keys_s, starts), lab_s[starts])
    # sampled clusters against the definition, with oracle counts
    rng = np.random.default_rng(0)
    pick = rng.choice(starts.shape[0], size=200, replace=False)
    members = {}
    for c in pick:
        rows = order[starts[c]:starts[c] + sizes[c]]
        members[int(lab_s[starts[c]])] = [(int(kx[r]), int(ky[r]), int(cnt[r])) for r in rows]
    query = set()
    for ts in members.values():
        for x, y, _ in ts:
            for dx in (-1, 0, 1):
                for dy in (-1, 0, 1):
                    query.add((x + dx, y + dy))
    query = sorted(query)
    qx = np.array([q[0] for q in query], np.int64)
    qy = np.array([q[1] for q in query], np.int64)
    _say(f"paper-500M: oracle counts for {len(query)} tiles")
    counts = np.zeros(len(query), np.uint64)
    s = oracle.scale_for_precision(2)
    for h in host:
        oracle.count_tiles(h, s, qx, qy, out=counts)
    exact = dict(zip(query, counts.tolist()))
    for label, ts in members.items():
        tiles = {(x, y) for x, y, _ in ts}
        for x, y, c in ts:
            assert exact[(x, y)] == c, (label, x, y, c, exact[(x, y)])
        ring = {(x + dx, y + dy) for x, y in tiles for dx in (-1, 0, 1) for dy in (-1, 0, 1)} - tiles
        assert all(exact[t] < tau for t in ring), label
        assert len(_components(tiles)) == 1, label
        assert int(biased([min(tiles)[0]], [min(tiles)[1]])[0]) == label
    # per-point labels over all 500M points: each cluster holds exactly the
    # points its tiles counted, the rest are noise, and sampled points carry
    # the label of their tile as the oracle projects and looks it up
    _say("paper-500M: per-point labels")
    lab_i = lab.astype(np.uint64).view(np.int64)
    labs_u, inv = np.unique(lab_i, return_inverse=True)
    want_pts = np.bincount(inv, weights=cnt.astype(np.float64)).astype(np.int64)
    lab_u = lab.astype(np.uint64)
    rows = oracle.OracleResult(kx, ky, cnt.astype(np.uint64),
                               (lab_u >> np.uint64(32)).astype(np.int64) - (1 << 31),
                               (lab_u & np.uint64(0xFFFFFFFF)).astype(np.int64) - (1 << 31))
    got_pts = np.zeros(labs_u.shape[0], np.int64)
    noise = 0
    for c, h in enumerate(host):
        d = dev(h, torch)
        pl = g.point_labels(d)
        u, n_u = torch.unique(pl, return_counts=True)
        u, n_u = u.cpu().numpy(), n_u.cpu().numpy()
        noise += int(n_u[u == -1].sum())
        keep = u != -1
        pos = np.searchsorted(labs_u, u[keep])
        assert (pos < labs_u.shape[0]).all() and np.array_equal(labs_u[pos], u[keep]), c
        got_pts[pos] += n_u[keep]
        sample = rng.choice(h.shape[0], size=20_000, replace=False)
        want = oracle.point_labels(h[sample], rows, precision=2)
        assert np.array_equal(pl[torch.from_numpy(sample).to(pl.device)].cpu().numpy(), want), c
        del d, pl
    assert np.array_equal(got_pts, want_pts)
    assert noise == n_chunks * chunk - int(want_pts.sum())

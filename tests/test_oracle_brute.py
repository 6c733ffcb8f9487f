"""The oracle against an independent brute force on many tiny inputs.

Inputs are small (n <= 300) and packed into a few tiles, with negative
coordinates, so that counts cross tau, components touch diagonally and
clusters land on both sides of mu.  Compared exactly: every output row
(tile, count, label) and the number of kept clusters.
"""
import numpy as np
import pytest

from brute import brute_cluster, brute_tile_counts


def _case(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(0, 300))
    span = float(rng.choice([0.3, 0.6, 1.0, 2.0]))
    centre = rng.uniform(-1.0, 1.0, size=2)
    kind = int(rng.integers(0, 3))
    if kind == 0:
        pts = centre + rng.uniform(-span, span, size=(n, 2))
    elif kind == 1:
        pts = centre + rng.normal(0.0, span / 3, size=(n, 2))
    else:  # points snapped to a coarse lattice: many exact duplicates
        pts = np.round((centre + rng.uniform(-span, span, size=(n, 2))) * 20) / 20
    dtype = np.float32 if rng.random() < 0.25 else np.float64
    p = int(rng.integers(0, 3))
    tau = int(rng.integers(1, 6))
    mu = int(rng.integers(1, 6))
    return pts.astype(dtype), p, tau, mu


@pytest.mark.parametrize("block", range(8))
def test_oracle_matches_brute_force(oracle_mod, block):
    for seed in range(block * 60, (block + 1) * 60):
        pts, p, tau, mu = _case(seed)
        s = oracle_mod.scale_for_precision(p)
        rows, kept = brute_cluster(pts, s, tau, mu)
        r = oracle_mod.cluster(pts, tau=tau, mu=mu, scale=s)
        got = [(int(a), int(b), int(c), int(d), int(e)) for a, b, c, d, e in
               zip(r.kx, r.ky, r.count, r.label_x, r.label_y)]
        assert got == rows, (seed, p, tau, mu)
        assert r.stats["clusters"] == kept, seed


@pytest.mark.parametrize("seed", range(20))
def test_tile_counts_match_sort_and_run_length(oracle_mod, seed):
    pts, p, _, _ = _case(1000 + seed)
    s = oracle_mod.scale_for_precision(p)
    tiles, counts = brute_tile_counts(pts, s)
    st = oracle_mod.OracleStream(s, 1, 1)
    st.feed(pts)
    kx, ky, c = st.tile_counts()
    assert kx.tolist() == tiles[:, 0].tolist() if len(tiles) else kx.size == 0
    assert ky.tolist() == tiles[:, 1].tolist() if len(tiles) else ky.size == 0
    assert c.tolist() == counts.tolist()
    assert int(c.sum()) == pts.shape[0]


@pytest.mark.parametrize("metric,delta", [("chebyshev", 2), ("chebyshev", 3), ("manhattan", 1),
                                          ("manhattan", 2), ("manhattan", 4)])
def test_oracle_matches_brute_force_delta(oracle_mod, metric, delta):
    for seed in range(2000, 2080):
        pts, p, tau, mu = _case(seed)
        s = oracle_mod.scale_for_precision(p)
        rows, kept = brute_cluster(pts, s, tau, mu, metric, delta)
        r = oracle_mod.cluster(pts, tau=tau, mu=mu, scale=s, metric=metric, delta=delta)
        got = [(int(a), int(b), int(c), int(d), int(e)) for a, b, c, d, e in
               zip(r.kx, r.ky, r.count, r.label_x, r.label_y)]
        assert got == rows, (seed, metric, delta)
        assert r.stats["clusters"] == kept, seed


@pytest.mark.parametrize("metric,delta", [("chebyshev", 1), ("manhattan", 2)])
def test_oracle_matches_brute_force_2x2_step(oracle_mod, metric, delta):
    for seed in range(4000, 4100):
        pts, p, tau, mu = _case(seed)
        s = oracle_mod.scale_for_precision(p)
        rows, kept = brute_cluster(pts, s, tau, mu, metric, delta, window=True)
        r = oracle_mod.cluster(pts, tau=tau, mu=mu, scale=s, metric=metric, delta=delta, window=True)
        got = [(int(a), int(b), int(c), int(d), int(e)) for a, b, c, d, e in
               zip(r.kx, r.ky, r.count, r.label_x, r.label_y)]
        assert got == rows, (seed, metric, delta)
        assert r.stats["clusters"] == kept, seed


def _case3(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(0, 250))
    centre = rng.uniform(-1.0, 1.0, size=3)
    pts = centre + rng.normal(0.0, float(rng.choice([0.2, 0.4, 0.8])), size=(n, 3))
    if rng.random() < 0.3:
        pts = np.round(pts * 20) / 20
    dtype = np.float32 if rng.random() < 0.25 else np.float64
    return pts.astype(dtype), int(rng.integers(0, 2)), int(rng.integers(1, 4)), int(rng.integers(1, 5))


@pytest.mark.parametrize("metric,delta", [("chebyshev", 1), ("manhattan", 1), ("chebyshev", 2), ("manhattan", 3)])
def test_oracle_matches_brute_force_3d(oracle_mod, metric, delta):
    for seed in range(6000, 6080):
        pts, p, tau, mu = _case3(seed)
        s = oracle_mod.scale_for_precision(p)
        rows, kept = brute_cluster(pts, s, tau, mu, metric, delta)
        r = oracle_mod.cluster(pts, tau=tau, mu=mu, scale=s, metric=metric, delta=delta, dims=3)
        got = [tuple(int(v) for v in row) for row in
               zip(r.kx, r.ky, r.kz, r.count, r.label_x, r.label_y, r.label_z)]
        assert got == rows, (seed, metric, delta)
        assert r.stats["clusters"] == kept, seed

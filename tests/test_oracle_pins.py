"""Pins of the CPU oracle against facts fixed by the paper and by arithmetic.

Each test names what fixes its expected value: a worked example of the paper
(fixtures under tests/golden/), a closed form, or a special case.  Together
they are meant to fail on the plausible mistakes: a dropped neighbour
direction, floor instead of truncation, an FP32 product, x and y swapped, an
off-by-one in tau or mu, a wrong label.
"""
import json
import math
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def _rows(res):
    return [(int(a), int(b), int(c), int(d), int(e)) for a, b, c, d, e in
            zip(res.kx, res.ky, res.count, res.label_x, res.label_y)]


def test_scale_is_exact_power_of_ten(oracle_mod):
    for p in range(16):
        assert oracle_mod.scale_for_precision(p) == float(10 ** p)


def test_worked_example_section_3_2(oracle_mod):
    g = _golden("worked_example.json")
    s = oracle_mod.scale_for_precision(g["precision"])
    kx, ky = oracle_mod.project(np.array(g["points"]), s)
    assert set(zip(kx.tolist(), ky.tolist())) == {tuple(g["tile"])}
    st = oracle_mod.OracleStream(s, 1, 1)
    st.feed(np.array(g["points"]))
    kx, ky, c = st.tile_counts()
    assert (kx.tolist(), ky.tolist(), c.tolist()) == ([g["tile"][0]], [g["tile"][1]], [g["count"]])
    t_max = g["significant_for_tau_at_most"]
    for tau in range(1, t_max + 2):
        r = oracle_mod.cluster(np.array(g["points"]), tau=tau, mu=1, precision=g["precision"])
        assert r.stats["significant"] == (1 if tau <= t_max else 0)


def test_fig4_grid_corner(oracle_mod):
    g = _golden("fig4_grid_corner.json")
    pts = np.array(g["points"])
    r = oracle_mod.cluster(pts, tau=4, mu=1, precision=g["precision"])
    assert r.stats["significant"] == g["tau4_significant"] and r.num_tiles == 0
    r = oracle_mod.cluster(pts, tau=1, mu=4, precision=g["precision"])
    assert r.stats["clusters"] == g["tau1_mu4_clusters"]
    assert sorted(zip(r.kx.tolist(), r.ky.tolist())) == [tuple(t) for t in g["tiles"]]
    assert set(zip(r.label_x.tolist(), r.label_y.tolist())) == {tuple(g["tau1_mu4_label"])}
    r = oracle_mod.cluster(np.array(g["same_points_in_one_tile"]), tau=4, mu=1, precision=0)
    assert r.stats["significant"] == g["one_tile_tau4_significant"]


def test_projection_pins_f64(oracle_mod):
    g = _golden("projection_pins.json")
    for case in g["f64"]:
        s = oracle_mod.scale_for_precision(case["p"])
        pts = np.array([[case["x"], 0.0], [0.0, case["x"]]], np.float64)
        kx, ky = oracle_mod.project(pts, s)
        assert kx[0] == case["k"] and ky[1] == case["k"], case
        assert kx[1] == 0 and ky[0] == 0


def test_projection_pins_f32_widened(oracle_mod):
    g = _golden("projection_pins.json")
    for case in g["f32"]:
        s = oracle_mod.scale_for_precision(case["p"])
        pts = np.array([[case["x"], case["x"]]], np.float32)
        kx, ky = oracle_mod.project(pts, s)
        assert kx[0] == case["k"] and ky[0] == case["k"], case


def test_projection_range_errors(oracle_mod):
    g = _golden("projection_pins.json")
    for case in g["range_errors"]:
        x = float(case["x"])
        s = oracle_mod.scale_for_precision(case["p"])
        for pts in (np.array([[x, 0.0]]), np.array([[0.0, x]])):
            with pytest.raises(oracle_mod.OracleError) as e:
                oracle_mod.project(pts, s)
            assert e.value.code == oracle_mod.E_RANGE
            st = oracle_mod.OracleStream(s, 1, 1)
            st.feed(np.array([[0.0, 0.0]]))
            with pytest.raises(oracle_mod.OracleError):
                st.feed(np.concatenate([np.array([[-1.0, -1.0]]) / s, pts]))
            # the failing chunk left nothing behind and the stream is failed
            assert st.num_tiles() == 1 and st.stats()["n"] == 1 and st.stats()["failed"]
            with pytest.raises(oracle_mod.OracleError):
                st.finish()


def test_invalid_arguments(oracle_mod):
    for scale, tau, mu in [(100.0, 0, 1), (100.0, 1, 0), (0.0, 1, 1), (-1.0, 1, 1),
                           (math.inf, 1, 1), (math.nan, 1, 1)]:
        with pytest.raises(oracle_mod.OracleError):
            oracle_mod.OracleStream(scale, tau, mu)


def test_empty_input(oracle_mod):
    r = oracle_mod.cluster(np.zeros((0, 2)), tau=1, mu=1, precision=2)
    assert r.num_tiles == 0 and r.stats["distinct"] == 0 and r.stats["n"] == 0


def test_all_points_in_one_tile(oracle_mod):
    rng = np.random.default_rng(11)
    pts = 3.0 + rng.uniform(0.0, 0.0999, size=(1234, 2))  # tile (30, 30) at p=1
    r = oracle_mod.cluster(pts, tau=1234, mu=1, precision=1)
    assert _rows(r) == [(30, 30, 1234, 30, 30)]
    r = oracle_mod.cluster(pts, tau=1235, mu=1, precision=1)
    assert r.num_tiles == 0 and r.stats["significant"] == 0


def _tile_points(tiles, per_tile, scale=1.0):
    """per_tile points strictly inside each integer tile (positive quadrant)."""
    pts = []
    for (x, y) in tiles:
        for j in range(per_tile):
            f = (j + 1) / (per_tile + 1)
            pts.append(((x + 0.1 + 0.8 * f) / scale, (y + 0.1 + 0.8 * (1 - f)) / scale))
    return np.array(pts)


def test_block_is_one_cluster_labelled_by_min_tile(oracle_mod):
    tiles = [(x, y) for x in range(10, 15) for y in range(20, 24)]
    r = oracle_mod.cluster(_tile_points(tiles, 3), tau=3, mu=20, precision=0)
    assert r.stats["clusters"] == 1 and r.num_tiles == 20
    assert set(zip(r.label_x.tolist(), r.label_y.tolist())) == {(10, 20)}
    assert r.count.tolist() == [3] * 20


def test_exact_tau_boundary(oracle_mod):
    # tile (5,5) holds tau points, tile (5,6) tau-1: only the first is significant
    pts = np.concatenate([_tile_points([(5, 5)], 7), _tile_points([(5, 6)], 6)])
    r = oracle_mod.cluster(pts, tau=7, mu=1, precision=0)
    assert _rows(r) == [(5, 5, 7, 5, 5)]


def test_diagonal_chain_needs_eight_neighbours(oracle_mod):
    # tiles touch only at corners: one cluster under Chebyshev-1 adjacency,
    # and both diagonal directions are exercised
    up = [(i, i) for i in range(6)]
    down = [(10 + i, 20 - i) for i in range(6)]
    r = oracle_mod.cluster(_tile_points(up + down, 2), tau=2, mu=6, precision=0)
    assert r.stats["clusters"] == 2 and r.num_tiles == 12
    labels = dict(zip(zip(r.kx.tolist(), r.ky.tolist()), zip(r.label_x.tolist(), r.label_y.tolist())))
    assert all(labels[t] == (0, 0) for t in up)
    assert all(labels[t] == (10, 20) for t in down)


def test_gap_of_one_tile_separates(oracle_mod):
    left = [(0, y) for y in range(5)]
    right = [(2, y) for y in range(5)]  # column 1 empty: Chebyshev distance 2
    r = oracle_mod.cluster(_tile_points(left + right, 1), tau=1, mu=1, precision=0)
    assert r.stats["clusters"] == 2
    assert set(zip(r.label_x.tolist(), r.label_y.tolist())) == {(0, 0), (2, 0)}


def test_non_significant_tile_does_not_bridge(oracle_mod):
    a = [(0, 0), (0, 1)]
    bridge = [(1, 1)]
    b = [(2, 2), (2, 3)]
    pts = np.concatenate([_tile_points(a + b, 3), _tile_points(bridge, 2)])
    r = oracle_mod.cluster(pts, tau=3, mu=1, precision=0)
    assert r.stats["clusters"] == 2 and r.stats["significant"] == 4
    r = oracle_mod.cluster(pts, tau=2, mu=1, precision=0)
    assert r.stats["clusters"] == 1 and r.num_tiles == 5


@pytest.mark.parametrize("mu", [3, 4, 5])
def test_mu_boundary(oracle_mod, mu):
    # clusters of exactly 3, 4 and 5 tiles, far apart
    c3 = [(0, 0), (0, 1), (0, 2)]
    c4 = [(10, 0), (10, 1), (10, 2), (10, 3)]
    c5 = [(20, 0), (20, 1), (20, 2), (20, 3), (20, 4)]
    r = oracle_mod.cluster(_tile_points(c3 + c4 + c5, 1), tau=1, mu=mu, precision=0)
    sizes = {3: c3, 4: c4, 5: c5}
    expect = sorted(t for k, ts in sizes.items() if k >= mu for t in ts)
    assert sorted(zip(r.kx.tolist(), r.ky.tolist())) == expect
    assert r.stats["components"] == 3 and r.stats["clusters"] == sum(k >= mu for k in sizes)


def test_axes_are_not_swapped(oracle_mod):
    # an L-shape whose transpose is a different tile set
    tiles = [(3, 7), (4, 7), (5, 7), (5, 8)]
    r = oracle_mod.cluster(_tile_points(tiles, 1, scale=10.0), tau=1, mu=1, precision=1)
    assert sorted(zip(r.kx.tolist(), r.ky.tolist())) == tiles
    assert set(zip(r.label_x.tolist(), r.label_y.tolist())) == {(3, 7)}


def test_negative_coordinates_and_zero_tile(oracle_mod):
    # truncation toward zero makes tile 0 span (-1/s, 1/s) on each axis
    pts = np.array([[-0.05, -0.05], [0.05, 0.05], [-0.05, 0.05], [0.05, -0.05],
                    [-0.15, -0.15], [-0.15, -0.15]])
    r = oracle_mod.cluster(pts, tau=1, mu=1, precision=1)
    assert _rows(r) == [(-1, -1, 2, -1, -1), (0, 0, 4, -1, -1)]


def test_uniform_sparse_noise_gives_no_clusters(oracle_mod):
    # homogeneous data has no clusters at a suitable precision (Appendix A)
    rng = np.random.default_rng(5)
    pts = rng.uniform(0.0, 100.0, size=(20_000, 2))   # about 0.2 points per tile at p=1
    r = oracle_mod.cluster(pts, tau=5, mu=4, precision=1)
    assert r.stats["clusters"] == 0 and r.num_tiles == 0


def test_duplicate_points_each_count(oracle_mod):
    pts = np.array([[0.5, 0.5]] * 9)
    r = oracle_mod.cluster(pts, tau=9, mu=1, precision=0)
    assert _rows(r) == [(0, 0, 9, 0, 0)]


def test_non_integer_scale(oracle_mod):
    # Section 3.2 allows any non-zero real scale, e.g. precision 3.5
    s = 10.0 ** 3.5
    pts = np.array([[1.0, 2.0], [1.0001, 2.0001]])
    kx, ky = oracle_mod.project(pts, s)
    assert kx.tolist() == [int(math.trunc(1.0 * s)), int(math.trunc(1.0001 * s))]
    assert ky.tolist() == [int(math.trunc(2.0 * s)), int(math.trunc(2.0001 * s))]


def test_count_tiles_matches_accumulator(oracle_mod):
    # the single-tile query agrees with the full accumulator on every tile,
    # and reports zero for tiles no point falls on
    rng = np.random.default_rng(21)
    pts = rng.normal(0.0, 0.3, size=(5000, 2))
    s = oracle_mod.scale_for_precision(1)
    st = oracle_mod.OracleStream(s, 1, 1)
    st.feed(pts)
    kx, ky, c = st.tile_counts()
    qx = np.concatenate([kx, [999, -999]])
    qy = np.concatenate([ky, [0, 5]])
    got = oracle_mod.count_tiles(pts[:2500], s, qx, qy)
    got = oracle_mod.count_tiles(pts[2500:], s, qx, qy, out=got)
    assert got[:-2].tolist() == c.tolist() and got[-2:].tolist() == [0, 0]


# ---- neighbourhood: Chebyshev or Manhattan distance delta (Section 3.2) ----

def _sig_tiles(oracle_mod, tiles, metric, delta, mu=1):
    r = oracle_mod.cluster(_tile_points(tiles, 1, scale=10.0), tau=1, mu=mu, precision=1,
                           metric=metric, delta=delta)
    return r


def test_neighbour_counts_match_section_3_6(oracle_mod):
    # Section 3.6 (higher dimensions): at Manhattan distance 1 a tile has 2d
    # neighbours, and 3^d - 1 when all adjacent tiles count; for d = 2, 4 and 8.
    # Count the adjacent offsets whose tile joins (100, 100).
    units = [(dx, dy) for dx in (-1, 0, 1) for dy in (-1, 0, 1) if (dx, dy) != (0, 0)]
    for metric, want in (("chebyshev", 8), ("manhattan", 4)):
        joined = sum(_sig_tiles(oracle_mod, [(100, 100), (100 + dx, 100 + dy)], metric, 1).stats["clusters"] == 1
                     for dx, dy in units)
        assert joined == want, metric


def test_delta_two_joins_a_one_tile_gap(oracle_mod):
    # tiles two columns apart: separate at distance 1, one cluster at 2 in both
    # metrics; the joined cluster has tiles without direct neighbours, which
    # Section 3.2 notes for Manhattan distances above 1
    tiles = [(0, 0), (2, 0)]
    for metric in ("chebyshev", "manhattan"):
        assert _sig_tiles(oracle_mod, tiles, metric, 1).stats["clusters"] == 2
        r = _sig_tiles(oracle_mod, tiles, metric, 2)
        assert r.stats["clusters"] == 1
        assert set(zip(r.label_x.tolist(), r.label_y.tolist())) == {(0, 0)}


def test_diagonal_needs_chebyshev_or_manhattan_two(oracle_mod):
    tiles = [(5, 5), (6, 6)]
    assert _sig_tiles(oracle_mod, tiles, "chebyshev", 1).stats["clusters"] == 1
    assert _sig_tiles(oracle_mod, tiles, "manhattan", 1).stats["clusters"] == 2
    assert _sig_tiles(oracle_mod, tiles, "manhattan", 2).stats["clusters"] == 1


def test_knight_move_and_ring_radius(oracle_mod):
    # (0, 0)-(1, 2): Chebyshev 2 and Manhattan 3 apart
    tiles = [(0, 0), (1, 2)]
    assert _sig_tiles(oracle_mod, tiles, "chebyshev", 1).stats["clusters"] == 2
    assert _sig_tiles(oracle_mod, tiles, "chebyshev", 2).stats["clusters"] == 1
    assert _sig_tiles(oracle_mod, tiles, "manhattan", 2).stats["clusters"] == 2
    assert _sig_tiles(oracle_mod, tiles, "manhattan", 3).stats["clusters"] == 1
    # all tiles at Chebyshev distance exactly 3 from a centre: (2*3+1)^2 - (2*3-1)^2 = 24
    ring3 = [(dx, dy) for dx in range(-3, 4) for dy in range(-3, 4) if max(abs(dx), abs(dy)) == 3]
    assert len(ring3) == 24
    for metric, delta, want in (("chebyshev", 3, 24), ("chebyshev", 2, 0), ("manhattan", 3, 4),
                                ("manhattan", 6, 24), ("manhattan", 5, 20)):
        joined = sum(_sig_tiles(oracle_mod, [(50, 50), (50 + dx, 50 + dy)], metric, delta).stats["clusters"] == 1
                     for dx, dy in ring3)
        assert joined == want, (metric, delta)


def test_delta_chain_and_mu(oracle_mod):
    # a chain of tiles 3 apart: one cluster of 5 at delta 3, five singletons at 2
    tiles = [(3 * k, 0) for k in range(5)]
    assert _sig_tiles(oracle_mod, tiles, "chebyshev", 3, mu=5).stats["clusters"] == 1
    assert _sig_tiles(oracle_mod, tiles, "chebyshev", 3, mu=6).stats["clusters"] == 0
    assert _sig_tiles(oracle_mod, tiles, "manhattan", 2, mu=1).stats["clusters"] == 5


def test_invalid_neighbourhood(oracle_mod):
    pts = np.array([[0.5, 0.5]])
    for kw in (dict(delta=0), dict(delta=65), dict(metric="euclid")):
        with pytest.raises((oracle_mod.OracleError, KeyError)):
            oracle_mod.cluster(pts, tau=1, mu=1, precision=0, **kw)


# ---- the 2x2 post-step for disadvantageous grid layouts (Section 3.6) -------

def test_fig4_corner_with_2x2_step(oracle_mod):
    g = _golden("fig4_grid_corner.json")
    pts = np.array(g["points"])
    r = oracle_mod.cluster(pts, tau=4, mu=1, precision=g["precision"], window=True)
    assert r.stats["significant"] == g["tau4_with_2x2_step_significant"]
    assert r.stats["clusters"] == 1
    assert sorted(zip(r.kx.tolist(), r.ky.tolist())) == [tuple(t) for t in g["tiles"]]
    assert set(zip(r.label_x.tolist(), r.label_y.tolist())) == {tuple(g["tau1_mu4_label"])}
    assert r.count.tolist() == [1, 1, 1, 1]
    # without the step nothing is significant
    assert oracle_mod.cluster(pts, tau=4, mu=1, precision=g["precision"]).stats["significant"] == 0


def _square_case(oracle_mod, counts, tau):
    pts = _tile_points([t for t, c in counts.items() for _ in range(c)], 1, scale=10.0)
    r = oracle_mod.cluster(pts, tau=tau, mu=1, precision=1, window=True)
    return sorted(zip(r.kx.tolist(), r.ky.tolist()))


def test_2x2_step_closed_forms(oracle_mod):
    # three occupied tiles of one square: kept together at tau 3, not at 4;
    # the empty fourth tile is never output
    three = {(10, 10): 1, (11, 10): 1, (10, 11): 1}
    assert _square_case(oracle_mod, three, 3) == [(10, 10), (10, 11), (11, 10)]
    assert _square_case(oracle_mod, three, 4) == []
    # a diagonal pair is one square: both corners are found
    assert _square_case(oracle_mod, {(20, 20): 1, (21, 21): 2}, 3) == [(20, 20), (21, 21)]
    assert _square_case(oracle_mod, {(20, 21): 1, (21, 20): 2}, 3) == [(20, 21), (21, 20)]
    # two columns apart: no square holds both
    assert _square_case(oracle_mod, {(30, 30): 2, (32, 30): 2}, 4) == []
    # a significant tile does not make its light neighbours significant unless
    # a square reaches tau: (40, 40) has 5 of tau 5, its neighbour 1 point;
    # every square holding the neighbour also holds (40, 40), so it is kept
    assert _square_case(oracle_mod, {(40, 40): 5, (41, 40): 1, (43, 40): 1}, 5) == [(40, 40), (41, 40)]


def test_2x2_step_only_adds(oracle_mod):
    rng = np.random.default_rng(31)
    pts = rng.normal(0.0, 0.4, size=(3000, 2))
    a = oracle_mod.cluster(pts, tau=6, mu=1, precision=1)
    b = oracle_mod.cluster(pts, tau=6, mu=1, precision=1, window=True)
    sa = set(zip(a.kx.tolist(), a.ky.tolist()))
    sb = set(zip(b.kx.tolist(), b.ky.tolist()))
    assert sa < sb and b.stats["distinct"] == a.stats["distinct"]


# ---- three dimensions (Section 3.6: RASTER in d dimensions) ----------------

def _tiles3(tiles, per_tile=1, scale=10.0):
    """per_tile points at the centre of each (x, y, z) tile (non-negative tiles)."""
    return np.array([[(x + 0.5) / scale, (y + 0.5) / scale, (z + 0.5) / scale]
                     for x, y, z in tiles for _ in range(per_tile)])


def test_3d_neighbour_counts_match_section_3_6(oracle_mod):
    # in d = 3 a tile has 3^d - 1 = 26 neighbours when all adjacent tiles
    # count, and 2d = 6 at Manhattan distance 1
    units = [(dx, dy, dz) for dx in (-1, 0, 1) for dy in (-1, 0, 1) for dz in (-1, 0, 1) if (dx, dy, dz) != (0, 0, 0)]
    assert len(units) == 26
    for metric, want in (("chebyshev", 26), ("manhattan", 6)):
        joined = 0
        for dx, dy, dz in units:
            pts = _tiles3([(50, 50, 50), (50 + dx, 50 + dy, 50 + dz)])
            joined += oracle_mod.cluster(pts, tau=1, mu=1, precision=1, metric=metric).stats["clusters"] == 1
        assert joined == want, metric


def test_3d_projection_and_range(oracle_mod):
    # the same truncation per coordinate; |k| <= 2^20 - 2 in three dimensions
    r = oracle_mod.cluster(np.array([[0.29, -0.57, 104857.4]]), tau=1, mu=1, precision=1)
    assert (r.kx.tolist(), r.ky.tolist(), r.kz.tolist()) == ([2], [-5], [1048574])
    r = oracle_mod.cluster(np.array([[0.29, 2.675, -0.001]]), tau=1, mu=1, precision=2)
    assert (r.kx.tolist(), r.ky.tolist(), r.kz.tolist()) == ([28], [267], [0])
    for bad in ([[0.5, 0.5, 104857.5]], [[-104857.5, 0.5, 0.5]], [[0.5, np.nan, 0.5]], [[2e5, 0.5, 0.5]]):
        with pytest.raises(oracle_mod.OracleError) as e:
            oracle_mod.cluster(np.array(bad), tau=1, mu=1, precision=1)
        assert e.value.code == oracle_mod.E_RANGE
    # the 2x2 post-step is two-dimensional
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.cluster(np.array([[0.5, 0.5, 0.5]]), tau=1, mu=1, precision=1, window=True)


def test_3d_block_axes_and_z(oracle_mod):
    block = [(x, y, z) for x in (3, 4) for y in (7, 8) for z in (1, 2)]
    r = oracle_mod.cluster(_tiles3(block), tau=1, mu=8, precision=1)
    assert r.stats["clusters"] == 1 and r.num_tiles == 8
    assert set(zip(r.label_x.tolist(), r.label_y.tolist(), r.label_z.tolist())) == {(3, 7, 1)}
    # an L in the x-z plane whose transposes are other tile sets
    ell = [(3, 0, 7), (4, 0, 7), (5, 0, 7), (5, 0, 8)]
    r = oracle_mod.cluster(_tiles3(ell), tau=1, mu=1, precision=1)
    assert sorted(zip(r.kx.tolist(), r.ky.tolist(), r.kz.tolist())) == ell
    # tiles apart only in z: two clusters at distance 1, one at 2
    pair = [(9, 9, 0), (9, 9, 2)]
    assert oracle_mod.cluster(_tiles3(pair), tau=1, mu=1, precision=1).stats["clusters"] == 2
    assert oracle_mod.cluster(_tiles3(pair), tau=1, mu=1, precision=1, delta=2).stats["clusters"] == 1
    # counts and tau in 3-D
    r = oracle_mod.cluster(_tiles3([(1, 1, 1)], per_tile=4) , tau=4, mu=1, precision=1)
    assert r.count.tolist() == [4]
    assert oracle_mod.cluster(_tiles3([(1, 1, 1)], per_tile=3), tau=4, mu=1, precision=1).num_tiles == 0

"""The multi-core CPU P-RASTER baseline against the oracle (CPU only).

P-RASTER clusters vertical slices in parallel and joins clusters across slice
borders (Section 3.5, Algorithms 2 and 3); its result must equal plain
RASTER's (Appendix C shows the slicing is arbitrary).  The cases put clusters
across one, several and all borders, diagonally across a border, and split
clusters whose halves are each below mu.
"""
import numpy as np
import pytest

import cpu_baseline

GRID = 10.0   # precision 1


def _same(p, o, what=""):
    assert p.kx.tolist() == o.kx.tolist(), what
    assert p.ky.tolist() == o.ky.tolist(), what
    assert p.count.tolist() == o.count.tolist(), what
    assert p.label_x.tolist() == o.label_x.tolist(), what
    assert p.label_y.tolist() == o.label_y.tolist(), what
    assert p.stats["clusters"] == o.stats["clusters"], what
    assert p.stats["significant"] == o.stats["significant"], what
    assert p.stats["distinct"] == o.stats["distinct"], what


def _tiles(tiles, per_tile=1):
    """Points at the centres of the given tiles (precision 1)."""
    return np.array([[(x + 0.5) / GRID, (y + 0.5) / GRID] for x, y in tiles for _ in range(per_tile)])


def _case(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(0, 400))
    span = float(rng.choice([0.3, 0.6, 1.0, 2.0]))
    centre = rng.uniform(-1.0, 1.0, size=2)
    pts = centre + rng.normal(0.0, span / 3, size=(n, 2))
    if rng.random() < 0.3:
        pts = np.round(pts * 20) / 20
    dtype = np.float32 if rng.random() < 0.25 else np.float64
    return pts.astype(dtype), int(rng.integers(0, 3)), int(rng.integers(1, 5)), int(rng.integers(1, 6))


@pytest.mark.parametrize("threads", [1, 2, 3, 5, 8])
def test_random_small_inputs(oracle_mod, threads):
    for seed in range(120):
        pts, p, tau, mu = _case(7000 + seed)
        s = oracle_mod.scale_for_precision(p)
        _same(cpu_baseline.cluster(pts, tau=tau, mu=mu, scale=s, threads=threads),
              oracle_mod.cluster(pts, tau=tau, mu=mu, scale=s), (seed, threads))


@pytest.mark.parametrize("threads", [1, 4, 16])
def test_plain_small(oracle_mod, threads):
    import synth
    pts = synth.plain_small(1)
    r = cpu_baseline.cluster(pts, tau=5, mu=4, scale=10.0, threads=threads)
    _same(r, oracle_mod.cluster(pts, tau=5, mu=4, precision=1), threads)
    if threads > 1:
        assert r.stats["join_candidates"] > 0


@pytest.mark.parametrize("threads", [2, 3, 7, 16])
def test_row_across_every_slice(oracle_mod, threads):
    # one straight row of 40 tiles: every border cuts it
    pts = _tiles([(x, 3) for x in range(40)])
    r = cpu_baseline.cluster(pts, tau=1, mu=40, scale=GRID, threads=threads)
    assert r.stats["clusters"] == 1 and r.num_tiles == 40
    assert set(zip(r.label_x.tolist(), r.label_y.tolist())) == {(0, 3)}
    _same(r, oracle_mod.cluster(pts, tau=1, mu=40, scale=GRID))


def test_u_shape_joined_through_another_slice(oracle_mod):
    # two arms in the left slice meet only inside the right slice
    arms = [(x, 0) for x in range(0, 10)] + [(x, 6) for x in range(0, 10)]
    bridge = [(9, y) for y in range(1, 6)]
    pad = [(19, 20)]   # widens the kx range so that column 9 is the left slice's last
    pts = _tiles(arms + bridge + pad)
    r = cpu_baseline.cluster(pts, tau=1, mu=2, scale=GRID, threads=2)
    assert r.stats["clusters"] == 1
    _same(r, oracle_mod.cluster(pts, tau=1, mu=2, scale=GRID))
    # without the bridge column (in the right slice) the arms stay apart
    pts = _tiles([(x, 0) for x in range(0, 12)] + [(x, 6) for x in range(0, 12)] + [(23, 20)])
    r = cpu_baseline.cluster(pts, tau=1, mu=2, scale=GRID, threads=2)
    assert r.stats["clusters"] == 2
    _same(r, oracle_mod.cluster(pts, tau=1, mu=2, scale=GRID))


def test_diagonal_across_a_border(oracle_mod):
    # kx range [0, 20) in two slices [0, 10) and [10, 20): (9, 5) and (10, 6)
    # touch only diagonally
    pts = _tiles([(0, 50), (9, 5), (10, 6), (19, 50)])
    r = cpu_baseline.cluster(pts, tau=1, mu=2, scale=GRID, threads=2)
    assert r.stats["clusters"] == 1 and sorted(zip(r.kx.tolist(), r.ky.tolist())) == [(9, 5), (10, 6)]
    _same(r, oracle_mod.cluster(pts, tau=1, mu=2, scale=GRID))
    # two columns apart across the border: no join
    pts = _tiles([(0, 50), (9, 5), (10, 7), (19, 50)])
    assert cpu_baseline.cluster(pts, tau=1, mu=2, scale=GRID, threads=2).stats["clusters"] == 0


def test_halves_below_mu_are_kept_together(oracle_mod):
    # a 2x2 block split by the border: each half has 2 tiles, mu = 4
    pts = _tiles([(0, 50), (9, 5), (9, 6), (10, 5), (10, 6), (19, 50)], per_tile=3)
    r = cpu_baseline.cluster(pts, tau=3, mu=4, scale=GRID, threads=2)
    assert r.stats["clusters"] == 1 and r.num_tiles == 4
    _same(r, oracle_mod.cluster(pts, tau=3, mu=4, scale=GRID))


def test_non_significant_tile_does_not_join_across(oracle_mod):
    pts = np.concatenate([_tiles([(0, 50), (19, 50)]), _tiles([(8, 5), (9, 5), (11, 5), (12, 5)], 3),
                          _tiles([(10, 5)], 2)])
    r = cpu_baseline.cluster(pts, tau=3, mu=2, scale=GRID, threads=2)
    assert r.stats["clusters"] == 2
    _same(r, oracle_mod.cluster(pts, tau=3, mu=2, scale=GRID))


def test_chunks_and_f32(oracle_mod):
    import synth
    pts = synth.plain_small(1)
    parts = np.array_split(pts, 7)
    _same(cpu_baseline.cluster(parts, tau=5, mu=4, scale=10.0, threads=6),
          oracle_mod.cluster(pts, tau=5, mu=4, precision=1))
    f = pts.astype(np.float32)
    _same(cpu_baseline.cluster(f, tau=5, mu=4, scale=10.0, threads=6),
          oracle_mod.cluster(f, tau=5, mu=4, precision=1))


def test_empty_and_errors():
    r = cpu_baseline.cluster(np.zeros((0, 2)), tau=1, mu=1, scale=10.0, threads=4)
    assert r.num_tiles == 0 and r.stats["clusters"] == 0
    bad = np.array([[0.5, 0.5], [np.nan, 0.0]])
    with pytest.raises(cpu_baseline.PRasterError) as e:
        cpu_baseline.cluster(bad, tau=1, mu=1, scale=10.0, threads=2)
    assert e.value.code == -2
    with pytest.raises(cpu_baseline.PRasterError) as e:
        cpu_baseline.cluster(np.array([[3e8, 0.0]]), tau=1, mu=1, scale=10.0, threads=2)
    assert e.value.code == -2
    for kw in (dict(tau=0, mu=1, scale=10.0), dict(tau=1, mu=0, scale=10.0), dict(tau=1, mu=1, scale=0.0),
               dict(tau=1, mu=1, scale=10.0, threads=0)):
        with pytest.raises(cpu_baseline.PRasterError) as e:
            cpu_baseline.cluster(np.array([[0.5, 0.5]]), **{"threads": 2, **kw})
        assert e.value.code == -1

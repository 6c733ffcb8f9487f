"""Pins of the oracle's per-tile point lists (RASTER', Section 3.4).

RASTER' keeps the points of each tile; listing them after clustering must give
every point of every kept tile exactly once, under its tile's row.  Expected
values come from the paper's worked examples (tests/golden/), from the counts
of the clustering itself, from the per-point labels (pinned separately) and
from a brute force; the last test plants mistakes in a copy of the function.
"""
import json
import os
import sys
import types

import numpy as np
import pytest

from brute import brute_cluster

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def _lists(mod, pts, tau, mu, precision=None, scale=None):
    r = mod.cluster(pts, tau=tau, mu=mu, precision=precision, scale=scale)
    start, index = mod.tile_points(pts, r, precision=precision, scale=scale)
    rows = list(zip(r.kx.tolist(), r.ky.tolist()))
    return r, {rows[j]: index[start[j]:start[j + 1]].tolist() for j in range(len(rows))}, start


def pin_worked_example(mod):
    g = _golden("worked_example.json")
    pts = np.array(g["points"])
    _, lists, start = _lists(mod, pts, 3, 1, precision=g["precision"])
    assert lists == {tuple(g["tile"]): [0, 1, 2]} and start.tolist() == [0, 3]
    _, lists, start = _lists(mod, pts, 4, 1, precision=g["precision"])
    assert lists == {} and start.tolist() == [0]


def pin_fig4_corner(mod):
    g = _golden("fig4_grid_corner.json")
    pts = np.array(g["points"])
    _, lists, _ = _lists(mod, pts, 1, 4, precision=g["precision"])
    # point i sits alone on its own tile of the corner
    assert lists == {(0, 0): [0], (1, 0): [1], (0, 1): [2], (1, 1): [3]}


def pin_row_sizes_are_counts(mod):
    rng = np.random.default_rng(8)
    pts = np.concatenate([rng.normal(c, 0.2, size=(300, 2)) for c in ((0, 0), (2, 2), (-3, 1))]
                         + [rng.uniform(-4, 4, size=(200, 2))])
    rng.shuffle(pts)
    r = mod.cluster(pts, tau=3, mu=3, precision=1)
    start, index = mod.tile_points(pts, r, precision=1)
    assert np.diff(start).tolist() == r.count.astype(np.int64).tolist()
    # exactly the points that carry a label, each once
    labelled = np.nonzero(mod.point_labels(pts, r, precision=1) != -1)[0]
    assert sorted(index.tolist()) == labelled.tolist()
    for j in range(r.num_tiles):
        seg = index[start[j]:start[j + 1]]
        assert np.all(np.diff(seg) > 0)


def pin_brute_force(mod):
    for seed in range(80):
        rng = np.random.default_rng(900 + seed)
        n = int(rng.integers(0, 200))
        pts = rng.uniform(-1.0, 1.0, size=2) + rng.normal(0.0, 0.4, size=(n, 2))
        p, tau, mu = int(rng.integers(0, 3)), int(rng.integers(1, 5)), int(rng.integers(1, 5))
        s = mod.scale_for_precision(p)
        rows, _ = brute_cluster(pts, s, tau, mu)
        k = np.trunc(np.asarray(pts, dtype=np.float64) * s).astype(np.int64)
        want = {(x, y): [i for i in range(n) if (k[i, 0], k[i, 1]) == (x, y)] for x, y, _, _, _ in rows}
        _, lists, _ = _lists(mod, pts, tau, mu, scale=s)
        assert lists == want, seed


def pin_rows_in_result_order(mod):
    # the lists follow the result's rows, whatever their order (the GPU's rows
    # come in compaction order): permuting the rows permutes the lists
    rng = np.random.default_rng(12)
    pts = rng.normal(0.0, 0.3, size=(2000, 2))
    r = mod.cluster(pts, tau=2, mu=1, precision=1)
    start, index = mod.tile_points(pts, r, precision=1)
    perm = rng.permutation(r.num_tiles)
    rp = mod.OracleResult(r.kx[perm], r.ky[perm], r.count[perm], r.label_x[perm], r.label_y[perm], r.stats)
    ps, pi = mod.tile_points(pts, rp, precision=1)
    for j, q in enumerate(perm.tolist()):
        assert pi[ps[j]:ps[j + 1]].tolist() == index[start[q]:start[q + 1]].tolist()


def pin_brute_force_3d(mod):
    # Section 3.6's three dimensions: the rows' lists from the brute force
    for seed in range(50):
        rng = np.random.default_rng(1900 + seed)
        n = int(rng.integers(0, 250))
        pts = rng.uniform(-1.0, 1.0, size=3) + rng.normal(0.0, 0.3, size=(n, 3))
        p, tau, mu = int(rng.integers(0, 3)), int(rng.integers(1, 4)), int(rng.integers(1, 4))
        s = mod.scale_for_precision(p)
        rows, _ = brute_cluster(pts, s, tau, mu)
        k = np.trunc(np.asarray(pts, dtype=np.float64) * s).astype(np.int64)
        want = {row[:3]: [i for i in range(n) if tuple(int(v) for v in k[i]) == row[:3]] for row in rows}
        r = mod.cluster(pts, tau=tau, mu=mu, scale=s)
        start, index = mod.tile_points(pts, r, scale=s)
        got = {(int(r.kx[j]), int(r.ky[j]), int(r.kz[j])): index[start[j]:start[j + 1]].tolist()
               for j in range(r.num_tiles)}
        assert got == want, seed
        assert start.tolist() == [0] + np.cumsum(r.count.astype(np.int64)).tolist(), seed


PINS = [pin_worked_example, pin_fig4_corner, pin_row_sizes_are_counts, pin_brute_force, pin_rows_in_result_order,
        pin_brute_force_3d]


@pytest.mark.parametrize("pin", PINS, ids=[f.__name__ for f in PINS])
def test_tile_points_pin(oracle_mod, pin):
    pin(oracle_mod)


def test_empty(oracle_mod):
    r = oracle_mod.cluster(np.array([[0.5, 0.5]]), tau=1, mu=1, precision=0)
    start, index = oracle_mod.tile_points(np.zeros((0, 2)), r, precision=0)
    assert start.tolist() == [0, 0] and index.shape == (0,)


MUTANTS = {
    "rows_in_sorted_order_not_result_order": ("row = order[pos[hit]]", "row = pos[hit]"),
    "nearest_not_equal": ("hit[hit] = tiles[order][pos[hit]] == q[hit]", "pass"),
    "axes_swapped": ("q = kx * (1 << 32) + ky\n    pos = np.searchsorted(tiles[order], q)",
                     "q = ky * (1 << 32) + kx\n    pos = np.searchsorted(tiles[order], q)"),
    "offsets_shifted": ("row_start[1:] = np.cumsum(np.bincount(row, minlength=t))",
                        "row_start[:-1] = np.cumsum(np.bincount(row, minlength=t))"),
    "point_order_lost": ('by_row = np.argsort(row, kind="stable")', 'by_row = np.argsort(-row, kind="stable")[::-1]'),
    "3d_points_before_rows": ("np.lexsort((point, row[point]))", "np.lexsort((row[point], point))"),
    "3d_offsets_shifted": ("starts[1:] = np.add.accumulate(", "starts[:-1] = np.add.accumulate("),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(oracle_mod, name):
    old, new = MUTANTS[name]
    src = open(os.path.join(ROOT, "oracle", "__init__.py")).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not found"
    mod = types.ModuleType("oracle_tp_mutant")
    mod.__file__ = os.path.join(ROOT, "oracle", "__init__.py")
    sys.modules[mod.__name__] = mod     # dataclasses look their module up there
    try:
        exec(compile(src.replace(old, new), mod.__file__, "exec"), mod.__dict__)
    finally:
        sys.modules.pop(mod.__name__, None)
    caught = []
    for pin in PINS:
        try:
            pin(mod)
        except AssertionError:
            caught.append(pin.__name__)
    assert caught, f"mutant {name} passed every tile-point pin"

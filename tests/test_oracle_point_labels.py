"""Pins of the oracle's per-point labels (Section 4.1's RASTER-star).

A point on a tile of a kept cluster carries the cluster's label, packed as
((label_x + 2^31) << 32) | (label_y + 2^31) and read as int64; every other
point carries -1.  The expected values come from the paper's worked examples
(tests/golden/), from packing written out with Python integers, and from the
brute force of tests/brute.py; the last test plants mistakes in a copy of the
oracle's function and checks that these pins catch each one.
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


def _pack(lx, ly):
    """The label word of tile (lx, ly) as a signed 64-bit Python integer."""
    v = ((lx + (1 << 31)) << 32) | (ly + (1 << 31))
    return v - (1 << 64) if v >= (1 << 63) else v


def _labels(oracle_mod, pts, tau, mu, precision=None, scale=None):
    r = oracle_mod.cluster(pts, tau=tau, mu=mu, precision=precision, scale=scale)
    return oracle_mod.point_labels(pts, r, precision=precision, scale=scale).tolist()


def pin_worked_example(oracle_mod):
    g = _golden("worked_example.json")
    pts = np.array(g["points"])
    lab = _pack(*g["tile"])
    assert lab == 0x8000006480000064 - (1 << 64)
    for tau in range(1, g["significant_for_tau_at_most"] + 2):
        want = [lab] * len(pts) if tau <= g["significant_for_tau_at_most"] else [-1] * len(pts)
        assert _labels(oracle_mod, pts, tau, 1, precision=g["precision"]) == want


def pin_fig4_corner(oracle_mod):
    g = _golden("fig4_grid_corner.json")
    pts = np.array(g["points"])
    assert _labels(oracle_mod, pts, 1, 4, precision=g["precision"]) == [_pack(*g["tau1_mu4_label"])] * 4
    assert _labels(oracle_mod, pts, 1, 5, precision=g["precision"]) == [-1] * 4
    assert _labels(oracle_mod, pts, 4, 1, precision=g["precision"]) == [-1] * 4


def pin_negative_tiles_and_order(oracle_mod):
    # two clusters on the negative side; points given in an order unlike the tiles'
    pts = np.array([[-0.15, -0.15], [0.55, 0.05], [-0.15, -0.05], [0.55, 0.15], [3.0, 3.0], [-0.15, -0.15]])
    got = _labels(oracle_mod, pts, 1, 2, precision=1)
    a, b = _pack(-1, -1), _pack(5, 0)
    assert a == 0x7FFFFFFF7FFFFFFF
    assert got == [a, b, a, b, -1, a]


def pin_lookup_needs_both_axes(oracle_mod):
    # tiles (1, 2) and (2, 1) are far apart; a query on (2, 1) must not find (1, 2)
    pts = np.array([[1.5, 2.5]] * 3 + [[2.5, 1.5]])
    assert _labels(oracle_mod, pts, 3, 1, precision=0) == [_pack(1, 2)] * 3 + [-1]


def pin_counts_per_label(oracle_mod):
    rng = np.random.default_rng(3)
    pts = np.concatenate([rng.normal(c, 0.25, size=(400, 2)) for c in ((0, 0), (3, 1), (-2, 4))]
                         + [rng.uniform(-5, 5, size=(300, 2))])
    r = oracle_mod.cluster(pts, tau=3, mu=3, precision=1)
    got = oracle_mod.point_labels(pts, r, precision=1)
    packed = [_pack(int(x), int(y)) for x, y in zip(r.label_x, r.label_y)]
    want = {}
    for lab, c in zip(packed, r.count):
        want[lab] = want.get(lab, 0) + int(c)
    labs, cnt = np.unique(got[got != -1], return_counts=True)
    assert dict(zip(labs.tolist(), cnt.tolist())) == want
    assert int((got == -1).sum()) == pts.shape[0] - sum(want.values())


def pin_brute_force(oracle_mod):
    for seed in range(120):
        rng = np.random.default_rng(500 + seed)
        n = int(rng.integers(0, 200))
        pts = rng.uniform(-1.0, 1.0, size=2) + rng.normal(0.0, 0.4, size=(n, 2))
        if seed % 4 == 0:
            pts = pts.astype(np.float32)
        p, tau, mu = int(rng.integers(0, 3)), int(rng.integers(1, 5)), int(rng.integers(1, 5))
        s = oracle_mod.scale_for_precision(p)
        rows, _ = brute_cluster(pts, s, tau, mu)
        tile_label = {(kx, ky): _pack(lx, ly) for kx, ky, _, lx, ly in rows}
        a = np.asarray(pts).astype(np.float64)
        k = np.trunc(a * s).astype(np.int64)
        want = [tile_label.get((int(x), int(y)), -1) for x, y in k]
        assert _labels(oracle_mod, pts, tau, mu, scale=s) == want, seed


def _pack3(lx, ly, lz):
    """The label word of a 3-D tile: three biased 21-bit fields, x highest."""
    return ((lx + (1 << 20)) << 42) | ((ly + (1 << 20)) << 21) | (lz + (1 << 20))


def pin_brute_force_3d(oracle_mod):
    # Section 3.6's three dimensions: every point carries the label of its
    # tile's kept cluster, from the brute force's rows
    for seed in range(60):
        rng = np.random.default_rng(1500 + seed)
        n = int(rng.integers(0, 250))
        pts = rng.uniform(-1.0, 1.0, size=3) + rng.normal(0.0, 0.3, size=(n, 3))
        if seed % 4 == 0:
            pts = pts.astype(np.float32)
        p, tau, mu = int(rng.integers(0, 3)), int(rng.integers(1, 4)), int(rng.integers(1, 4))
        s = oracle_mod.scale_for_precision(p)
        rows, _ = brute_cluster(pts, s, tau, mu)
        tile_label = {(kx, ky, kz): _pack3(lx, ly, lz) for kx, ky, kz, _, lx, ly, lz in rows}
        k = np.trunc(np.asarray(pts).astype(np.float64) * s).astype(np.int64)
        want = [tile_label.get(tuple(int(v) for v in t), -1) for t in k]
        assert _labels(oracle_mod, pts, tau, mu, scale=s) == want, seed


def pin_3d_lookup_needs_every_axis(oracle_mod):
    # tiles that are permutations of one another's coordinates: only the point
    # on the kept tile (1, 2, 3) gets a label
    pts = np.array([[1.5, 2.5, 3.5]] * 3 + [[3.5, 2.5, 1.5], [2.5, 1.5, 3.5], [1.5, 3.5, 2.5], [-1.5, -2.5, -3.5]])
    assert _labels(oracle_mod, pts, 3, 1, precision=0) == [_pack3(1, 2, 3)] * 3 + [-1] * 4
    pts = np.array([[-1.5, -2.5, -3.5]] * 2 + [[-1.5, -2.5, -2.5]])
    assert _labels(oracle_mod, pts, 1, 2, precision=0) == [_pack3(-1, -2, -3)] * 3


def pin_3d_rows_in_any_order(oracle_mod):
    # a result's rows may come in any order (the GPU's come in compaction
    # order): permuting them changes no label
    rng = np.random.default_rng(21)
    pts = rng.normal(0.0, 0.3, size=(3000, 3))
    r = oracle_mod.cluster(pts, tau=2, mu=2, precision=1)
    want = oracle_mod.point_labels(pts, r, precision=1).tolist()
    assert r.num_tiles > 10 and sum(v != -1 for v in want) > 100
    perm = rng.permutation(r.num_tiles)
    rp = oracle_mod.OracleResult(r.kx[perm], r.ky[perm], r.count[perm], r.label_x[perm], r.label_y[perm], r.stats,
                                 r.kz[perm], r.label_z[perm])
    assert oracle_mod.point_labels(pts, rp, precision=1).tolist() == want


PINS = [pin_worked_example, pin_fig4_corner, pin_negative_tiles_and_order, pin_lookup_needs_both_axes,
        pin_counts_per_label, pin_brute_force, pin_brute_force_3d, pin_3d_lookup_needs_every_axis,
        pin_3d_rows_in_any_order]


@pytest.mark.parametrize("pin", PINS, ids=[f.__name__ for f in PINS])
def test_point_label_pin(oracle_mod, pin):
    pin(oracle_mod)


def test_point_labels_of_empty_input(oracle_mod):
    r = oracle_mod.cluster(np.zeros((0, 2)), tau=1, mu=1, precision=0)
    assert oracle_mod.point_labels(np.zeros((0, 2)), r, precision=0).shape == (0,)
    r = oracle_mod.cluster(np.array([[0.5, 0.5]]), tau=1, mu=1, precision=0)
    assert oracle_mod.point_labels(np.zeros((0, 2)), r, precision=0).shape == (0,)


MUTANTS = {
    "halves_swapped": ("(((result.label_x[order]", "(((result.label_y[order]"),
    "no_bias_on_y": ("| (result.label_y[order].astype(np.int64) + (1 << 31))",
                     "| (result.label_y[order].astype(np.int64))"),
    "query_axes_swapped": ("q = kx * (1 << 32) + ky\n    pos = np.searchsorted(tiles, q)",
                           "q = ky * (1 << 32) + kx\n    pos = np.searchsorted(tiles, q)"),
    "noise_is_zero": ("out = np.full(kx.shape[0], -1, dtype=np.int64)",
                      "out = np.full(kx.shape[0], 0, dtype=np.int64)"),
    "nearest_not_equal": ("hit[hit] = tiles[pos[hit]] == q[hit]", "pass"),
    "3d_x_y_swapped": ("return (x * base + y) * base + z", "return (y * base + x) * base + z"),
    "3d_no_bias": ("bias = 1 << 20", "bias = 0"),
    "3d_nearest_not_equal": ("found = ids[by_id][at] == want", "found = at >= 0"),
    "3d_sorted_row_not_result_row": ("row[found] = by_id[at[found]]", "row[found] = at[found]"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_label_mistake(oracle_mod, name):
    old, new = MUTANTS[name]
    src = open(os.path.join(ROOT, "oracle", "__init__.py")).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not found"
    mod = types.ModuleType("oracle_mutant")
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
    assert caught, f"mutant {name} passed every point-label pin"

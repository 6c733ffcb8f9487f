"""Invariants of the oracle that hold at any size.

* the tile counts sum to n (every point lands in exactly one tile);
* permuting the input, or cutting it into chunks fed in any order, does not
  change the result (Section 3.6: the input may be partitioned arbitrarily and
  processed in any order);
* every output tile meets tau, every cluster is connected, maximal among the
  significant tiles, holds at least mu tiles and is labelled by its smallest
  tile; every dropped component has fewer than mu tiles.
"""
import numpy as np
import pytest

import synth


def _rows(r):
    return list(zip(r.kx.tolist(), r.ky.tolist(), r.count.tolist(),
                    r.label_x.tolist(), r.label_y.tolist()))


@pytest.fixture(scope="module")
def small_pts():
    return synth.plain_small(1)


def test_counts_sum_to_n(oracle_mod, small_pts):
    st = oracle_mod.OracleStream(oracle_mod.scale_for_precision(1), 5, 4)
    st.feed(small_pts)
    _, _, c = st.tile_counts()
    assert int(c.sum()) == small_pts.shape[0]
    assert st.num_tiles() <= small_pts.shape[0]


def test_permutation_invariance(oracle_mod, small_pts):
    a = oracle_mod.cluster(small_pts, tau=5, mu=4, precision=1)
    perm = np.random.default_rng(3).permutation(small_pts.shape[0])
    b = oracle_mod.cluster(small_pts[perm], tau=5, mu=4, precision=1)
    assert _rows(a) == _rows(b) and a.stats == b.stats


@pytest.mark.parametrize("k", [1, 2, 7, 10])
def test_chunk_invariance(oracle_mod, small_pts, k):
    whole = oracle_mod.cluster(small_pts, tau=5, mu=4, precision=1)
    rng = np.random.default_rng(k)
    cuts = np.sort(rng.choice(np.arange(1, small_pts.shape[0]), size=k - 1, replace=False))
    chunks = np.split(small_pts, cuts)
    order = rng.permutation(len(chunks))
    got = oracle_mod.cluster_chunks([chunks[i] for i in order], tau=5, mu=4, precision=1)
    assert _rows(got) == _rows(whole)


def test_structure_of_result(oracle_mod, small_pts):
    tau, mu = 5, 4
    st = oracle_mod.OracleStream(oracle_mod.scale_for_precision(1), tau, mu)
    st.feed(small_pts)
    kx, ky, c = st.tile_counts()
    sig = {(x, y) for x, y, n in zip(kx.tolist(), ky.tolist(), c.tolist()) if n >= tau}
    r = st.finish()
    out = {(x, y): (n, (lx, ly)) for x, y, n, lx, ly in _rows(r)}
    assert all(n >= tau for n, _ in out.values())
    assert set(out) <= sig
    # components of the significant tiles, by a flood fill over a set
    seen, comps = set(), []
    for t in sorted(sig):
        if t in seen:
            continue
        comp, stack = [], [t]
        seen.add(t)
        while stack:
            u = stack.pop()
            comp.append(u)
            for dx in (-1, 0, 1):
                for dy in (-1, 0, 1):
                    v = (u[0] + dx, u[1] + dy)
                    if v in sig and v not in seen:
                        seen.add(v)
                        stack.append(v)
        comps.append(comp)
    kept = 0
    for comp in comps:
        if len(comp) >= mu:
            kept += 1
            lab = min(comp)
            assert all(t in out and out[t][1] == lab for t in comp)
        else:
            assert all(t not in out for t in comp)
    assert kept == r.stats["clusters"] and len(comps) == r.stats["components"]
    # the plain-small workload has 100 dense centres; nearly all are found
    assert 90 <= r.stats["clusters"] <= 110

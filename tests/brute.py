"""Brute-force RASTER for tiny inputs, used to pin the oracle.

Structurally unlike the oracle on purpose: tiles are counted by sorting and
run-length encoding (numpy ``unique``) instead of a hash map, and clusters are
found from an explicit O(T^2) adjacency matrix with breadth-first search
instead of a depth-first walk over hash lookups.  Each step is a direct
reading of the paper: projection by scaling and truncation (Section 3.2),
significance as count >= tau, adjacency as a Chebyshev or Manhattan
distance between 1 and delta (Section 3.2; by default Chebyshev 1, all eight
neighbours), clusters kept when they hold at least mu tiles (Algorithm 1).
"""
from __future__ import annotations

from collections import deque

import numpy as np


def brute_tile_counts(points, scale: float):
    """Sorted unique tiles and their counts via sort + run length."""
    a = np.asarray(points)
    a = a.astype(np.float64) if a.dtype == np.float32 else a.astype(np.float64, copy=False)
    a = a.reshape(-1, 2)
    prod = a * scale
    if not np.all(np.abs(prod) < 2147483647.0):
        raise ValueError("coordinate out of range")
    k = np.trunc(prod).astype(np.int64)
    if k.shape[0] == 0:
        return np.zeros((0, 2), np.int64), np.zeros(0, np.int64)
    tiles, counts = np.unique(k, axis=0, return_counts=True)
    return tiles, counts


def brute_cluster(points, scale: float, tau: int, mu: int, metric: str = "chebyshev", delta: int = 1,
                  window: bool = False):
    """Returns rows (kx, ky, count, label_x, label_y) sorted by tile, plus the
    number of kept clusters.  Two significant tiles are adjacent when their
    distance in ``metric`` is between 1 and ``delta`` (Section 3.2).  With
    ``window`` (Section 3.6's 2x2 post-step) a tile is also significant when
    some 2x2 square of tiles containing it holds at least tau points."""
    tiles, counts = brute_tile_counts(points, scale)
    sig = counts >= tau
    if window and tiles.shape[0]:
        # every 2x2 square with at least one occupied tile, by its lower-left corner
        total = {}
        for (x, y), c in zip(tiles.tolist(), counts.tolist()):
            for cx in (x - 1, x):
                for cy in (y - 1, y):
                    total[(cx, cy)] = total.get((cx, cy), 0) + c
        heavy = {corner for corner, c in total.items() if c >= tau}
        for i, (x, y) in enumerate(tiles.tolist()):
            if any((cx, cy) in heavy for cx in (x - 1, x) for cy in (y - 1, y)):
                sig[i] = True
    st, sc = tiles[sig], counts[sig]
    t = st.shape[0]
    if t == 0:
        return [], 0
    ax = np.abs(st[:, None, 0] - st[None, :, 0])
    ay = np.abs(st[:, None, 1] - st[None, :, 1])
    d = np.maximum(ax, ay) if metric == "chebyshev" else ax + ay
    adj = (d >= 1) & (d <= delta)
    comp = -np.ones(t, np.int64)
    ncomp = 0
    for s in range(t):
        if comp[s] >= 0:
            continue
        comp[s] = ncomp
        q = deque([s])
        while q:
            u = q.popleft()
            for v in np.nonzero(adj[u])[0]:
                if comp[v] < 0:
                    comp[v] = ncomp
                    q.append(v)
        ncomp += 1
    rows, kept = [], 0
    for c in range(ncomp):
        members = np.nonzero(comp == c)[0]
        if members.shape[0] < mu:
            continue
        kept += 1
        lab = min((int(st[i, 0]), int(st[i, 1])) for i in members)
        for i in members:
            rows.append((int(st[i, 0]), int(st[i, 1]), int(sc[i]), lab[0], lab[1]))
    rows.sort()
    return rows, kept

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
    """Sorted unique tiles and their counts via sort + run length.  Points are
    (n, 2), or (n, 3) in three dimensions (tiles then need |k| <= 2^20 - 2)."""
    a = np.asarray(points)
    dims = 3 if a.ndim == 2 and a.shape[1] == 3 else 2
    a = a.astype(np.float64) if a.dtype == np.float32 else a.astype(np.float64, copy=False)
    a = a.reshape(-1, dims)
    prod = a * scale
    if not np.all(np.abs(prod) < (2147483647.0 if dims == 2 else 1048575.0)):
        raise ValueError("coordinate out of range")
    k = np.trunc(prod).astype(np.int64)
    if k.shape[0] == 0:
        return np.zeros((0, dims), np.int64), np.zeros(0, np.int64)
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
    diff = np.abs(st[:, None, :] - st[None, :, :])          # per coordinate
    d = diff.max(axis=2) if metric == "chebyshev" else diff.sum(axis=2)
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
        lab = min(tuple(int(v) for v in st[i]) for i in members)
        for i in members:
            tile = tuple(int(v) for v in st[i])
            # 2-D rows: (kx, ky, count, lx, ly); 3-D rows: (kx, ky, kz, count, lx, ly, lz)
            rows.append(tile + (int(sc[i]),) + lab)
    rows.sort()
    return rows, kept

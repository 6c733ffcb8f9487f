"""Canonical digests of clustering results, for comparing full-size GPU runs
with oracle results computed once and stored (tests/golden/full_size_digests.json).

A result is the set of rows (kx, ky, count, label_x, label_y), the label being
the cluster's smallest tile.  Rows are put in (kx, ky) order and each column is
hashed as little-endian 64-bit integers, column after column, with SHA-256.
Input point sets are hashed as their raw bytes.  Nothing here computes any
part of the clustering."""
from __future__ import annotations

import hashlib

import numpy as np


def rows_digest(kx, ky, count, label_x, label_y) -> str:
    kx, ky = np.asarray(kx, np.int64), np.asarray(ky, np.int64)
    order = np.lexsort((ky, kx))
    h = hashlib.sha256()
    for col, dt in ((kx, "<i8"), (ky, "<i8"), (count, "<u8"), (label_x, "<i8"), (label_y, "<i8")):
        h.update(np.ascontiguousarray(np.asarray(col)[order].astype(dt)).tobytes())
    return h.hexdigest()


def points_digest(points) -> str:
    return hashlib.sha256(np.ascontiguousarray(points).tobytes()).hexdigest()


def unbias_label(label):
    """(label_x, label_y) of a label written as the biased tile key
    ((label_x + 2^31) << 32) | (label_y + 2^31)."""
    lab = np.asarray(label).astype(np.uint64)
    lx = (lab >> np.uint64(32)).astype(np.int64) - (1 << 31)
    ly = (lab & np.uint64(0xFFFFFFFF)).astype(np.int64) - (1 << 31)
    return lx, ly


def biased(kx, ky):
    """The biased tile key ((kx + 2^31) << 32) | (ky + 2^31) that the
    library's labels use, packed here by the tests."""
    kx = np.asarray(kx, dtype=np.int64)
    ky = np.asarray(ky, dtype=np.int64)
    return ((kx + (1 << 31)).astype(np.uint64) << np.uint64(32)) | (ky + (1 << 31)).astype(np.uint64)


STAT_KEYS = ("n", "distinct", "significant", "components", "clusters", "tiles")

"""RASTER CPU oracle -- TEST INFRASTRUCTURE ONLY.

ctypes wrapper around ``raster_oracle.cpp``, a plain single-threaded
implementation of Algorithm 1 of the RASTER paper (contraction, then
agglomeration) with the chunked input of Section 3.6.  Only the tests, the
package smoke check and the benchmark's CPU-baseline leg may import this
module; the product library neither imports nor links it, and they share no
code.

Results come back as numpy arrays sorted by tile: ``kx``, ``ky`` (int64),
``count`` (uint64) and the label tile ``label_x``, ``label_y`` (the
lexicographically smallest tile of the cluster).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "raster_oracle.cpp")
_DEFAULT_LIB = os.path.join(_HERE, "liboracle.so")
# A test may point the wrapper at a deliberately broken build of the oracle
# (see tests/test_oracle_mutants.py) to show that the pins catch the mistake.
_LIB = os.environ.get("RASTER_ORACLE_LIB") or _DEFAULT_LIB

OK, E_INVAL, E_RANGE, E_STATE = 0, -1, -2, -5
F32, F64 = 1, 2

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (-O2, no FMA contraction, no fast-math)."""
    if force or not os.path.exists(_DEFAULT_LIB):
        compile_oracle(_SRC, _DEFAULT_LIB)
    return _DEFAULT_LIB


def compile_oracle(src: str, out: str) -> str:
    tmp = out + ".tmp%d" % os.getpid()
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-ffp-contract=off",
                           "-fno-fast-math", "-fPIC", "-shared", "-o", tmp, src])
    os.replace(tmp, out)
    return out


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    vp, i64, i32, u64, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, ctypes.c_double
    lib.oracle_scale_for_precision.argtypes = [i32]
    lib.oracle_scale_for_precision.restype = dbl
    lib.oracle_project.argtypes = [vp, i64, i32, dbl, vp, vp]
    lib.oracle_project.restype = ctypes.c_int
    lib.oracle_project3.argtypes = [vp, i64, i32, dbl, vp, vp, vp]
    lib.oracle_project3.restype = ctypes.c_int
    lib.oracle_begin.argtypes = [dbl, u64, u64]
    lib.oracle_begin.restype = vp
    lib.oracle_begin_ex.argtypes = [dbl, u64, u64, i32, i64, i32, i32]
    lib.oracle_begin_ex.restype = vp
    lib.oracle_feed.argtypes = [vp, vp, i64, i32]
    lib.oracle_feed.restype = ctypes.c_int
    lib.oracle_num_tiles.argtypes = [vp]
    lib.oracle_num_tiles.restype = i64
    lib.oracle_tile_counts.argtypes = [vp, vp, vp, vp, vp]
    lib.oracle_tile_counts.restype = ctypes.c_int
    lib.oracle_finish.argtypes = [vp]
    lib.oracle_finish.restype = ctypes.c_int
    lib.oracle_stats.argtypes = [vp, vp]
    lib.oracle_stats.restype = ctypes.c_int
    lib.oracle_result.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    lib.oracle_result.restype = ctypes.c_int
    lib.oracle_count_tiles.argtypes = [vp, i64, i32, dbl, vp, vp, i64, vp]
    lib.oracle_count_tiles.restype = ctypes.c_int
    lib.oracle_free.argtypes = [vp]
    lib.oracle_free.restype = None
    _lib = lib
    return lib


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: oracle status {code}")
        self.code = code


def scale_for_precision(p: int) -> float:
    return float(_load().oracle_scale_for_precision(int(p)))


def _as_points(points, dims: int = 2):
    a = np.asarray(points)
    if a.dtype == np.float32:
        dt = F32
    else:
        a = a.astype(np.float64, copy=False)
        dt = F64
    a = np.ascontiguousarray(a.reshape(-1, dims))
    return a, dt


def _dims_of(points) -> int:
    """3 for an (n, 3) array, else 2."""
    a = np.asarray(points)
    return 3 if a.ndim == 2 and a.shape[1] == 3 else 2


def project(points, scale: float):
    """Tile coordinates (kx, ky) of every point (Section 3.2)."""
    a, dt = _as_points(points)
    n = a.shape[0]
    kx = np.empty(n, np.int64)
    ky = np.empty(n, np.int64)
    rc = _load().oracle_project(a.ctypes.data, n, dt, float(scale), kx.ctypes.data, ky.ctypes.data)
    if rc != OK:
        raise OracleError(rc, "project")
    return kx, ky


def project3(points, scale: float):
    """Tile coordinates (kx, ky, kz) of every three-dimensional point
    (Section 3.2's projection per coordinate, Section 3.6's d dimensions)."""
    a, dt = _as_points(points, 3)
    n = a.shape[0]
    k = [np.empty(n, np.int64) for _ in range(3)]
    rc = _load().oracle_project3(a.ctypes.data, n, dt, float(scale), *(c.ctypes.data for c in k))
    if rc != OK:
        raise OracleError(rc, "project3")
    return tuple(k)


def count_tiles(points, scale: float, qx, qy, out=None):
    """Adds to ``out`` (uint64, one per query tile) the number of points of
    ``points`` on each query tile (qx[i], qy[i]); returns ``out``."""
    a, dt = _as_points(points)
    qx = np.ascontiguousarray(qx, dtype=np.int64)
    qy = np.ascontiguousarray(qy, dtype=np.int64)
    if out is None:
        out = np.zeros(qx.shape[0], np.uint64)
    rc = _load().oracle_count_tiles(a.ctypes.data, a.shape[0], dt, float(scale), qx.ctypes.data,
                                    qy.ctypes.data, qx.shape[0], out.ctypes.data)
    if rc != OK:
        raise OracleError(rc, "count_tiles")
    return out


@dataclass
class OracleResult:
    kx: np.ndarray
    ky: np.ndarray
    count: np.ndarray
    label_x: np.ndarray
    label_y: np.ndarray
    stats: dict = field(default_factory=dict)
    kz: np.ndarray | None = None       # 3-D only
    label_z: np.ndarray | None = None  # 3-D only

    @property
    def num_tiles(self) -> int:
        return int(self.kx.shape[0])

    @property
    def num_clusters(self) -> int:
        return int(self.stats.get("clusters", 0))


METRICS = {"chebyshev": 0, "manhattan": 1}


class OracleStream:
    """Chunked contraction (Section 3.6) followed by one agglomeration.
    Clusters join significant tiles within ``delta`` steps of each other in
    the given metric (Section 3.2); the default is the eight adjacent tiles.
    ``window`` adds the 2x2 post-step of Section 3.6; ``dims`` = 3 takes
    three-dimensional points (Section 3.6's generalisation)."""

    def __init__(self, scale: float, tau: int, mu: int, metric: str = "chebyshev", delta: int = 1,
                 window: bool = False, dims: int = 2):
        self._lib = _load()
        self._dims = int(dims)
        self._h = self._lib.oracle_begin_ex(float(scale), int(tau), int(mu), METRICS[metric], int(delta),
                                            int(bool(window)), self._dims)
        if not self._h:
            raise OracleError(E_INVAL, "begin")

    def feed(self, points) -> None:
        a, dt = _as_points(points, self._dims)
        rc = self._lib.oracle_feed(self._h, a.ctypes.data, a.shape[0], dt)
        if rc != OK:
            raise OracleError(rc, "feed")

    def num_tiles(self) -> int:
        return int(self._lib.oracle_num_tiles(self._h))

    def tile_counts(self):
        """All (kx, ky, count) of the accumulator, sorted by tile."""
        m = self.num_tiles()
        kx = np.empty(m, np.int64)
        ky = np.empty(m, np.int64)
        kz = np.empty(m, np.int64) if self._dims == 3 else None
        c = np.empty(m, np.uint64)
        rc = self._lib.oracle_tile_counts(self._h, kx.ctypes.data, ky.ctypes.data,
                                          kz.ctypes.data if kz is not None else None, c.ctypes.data)
        if rc != OK:
            raise OracleError(rc, "tile_counts")
        return (kx, ky, c) if kz is None else (kx, ky, kz, c)

    def stats(self) -> dict:
        st = np.zeros(7, np.int64)
        self._lib.oracle_stats(self._h, st.ctypes.data)
        return dict(n=int(st[0]), distinct=int(st[1]), significant=int(st[2]),
                    components=int(st[3]), clusters=int(st[4]), tiles=int(st[5]),
                    failed=bool(st[6]))

    def finish(self) -> OracleResult:
        rc = self._lib.oracle_finish(self._h)
        if rc != OK:
            raise OracleError(rc, "finish")
        st = self.stats()
        t = st["tiles"]
        kx = np.empty(t, np.int64)
        ky = np.empty(t, np.int64)
        c = np.empty(t, np.uint64)
        lx = np.empty(t, np.int64)
        ly = np.empty(t, np.int64)
        kz = np.empty(t, np.int64) if self._dims == 3 else None
        lz = np.empty(t, np.int64) if self._dims == 3 else None
        rc = self._lib.oracle_result(self._h, kx.ctypes.data, ky.ctypes.data,
                                     kz.ctypes.data if kz is not None else None, c.ctypes.data,
                                     lx.ctypes.data, ly.ctypes.data, lz.ctypes.data if lz is not None else None)
        if rc != OK:
            raise OracleError(rc, "result")
        return OracleResult(kx, ky, c, lx, ly, st, kz, lz)

    def close(self) -> None:
        if self._h:
            self._lib.oracle_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _scale(precision, scale):
    if scale is None:
        if precision is None:
            raise ValueError("give precision or scale")
        return scale_for_precision(precision)
    return float(scale)


def cluster(points, tau: int, mu: int, precision: int | None = None,
            scale: float | None = None, metric: str = "chebyshev", delta: int = 1,
            window: bool = False, dims: int | None = None) -> OracleResult:
    """RASTER on one in-memory point set ((n, 2), or (n, 3) for 3-D)."""
    st = OracleStream(_scale(precision, scale), tau, mu, metric, delta, window,
                      dims if dims is not None else _dims_of(points))
    try:
        st.feed(points)
        return st.finish()
    finally:
        st.close()


def _id_3d(kx, ky, kz):
    """Three-dimensional tiles with |k| <= 2^20 - 2 as int64: the biased
    coordinates k + 2^20 lie in [2, 2^21 - 2] and are written as the digits of
    a number in base 2^21, most significant first, so the numbers order the
    tiles lexicographically.  For a cluster's smallest tile this is its
    label."""
    base = 1 << 21
    bias = 1 << 20
    x, y, z = (np.asarray(c, dtype=np.int64) + bias for c in (kx, ky, kz))
    return (x * base + y) * base + z


def _rows_3d(points, result: OracleResult, s: float):
    """Row of ``result`` holding each three-dimensional point's tile, or -1."""
    kx, ky, kz = project3(points, s)
    row = np.full(kx.shape[0], -1, dtype=np.int64)
    if result.num_tiles == 0 or kx.shape[0] == 0:
        return row
    ids = _id_3d(result.kx, result.ky, result.kz)
    by_id = np.argsort(ids)
    want = _id_3d(kx, ky, kz)
    at = np.minimum(np.searchsorted(ids[by_id], want), ids.shape[0] - 1)
    found = ids[by_id][at] == want
    row[found] = by_id[at[found]]
    return row


def point_labels(points, result: OracleResult, precision: int | None = None,
                 scale: float | None = None):
    """Per-point labels as in the paper's comparison experiment (Section 4.1, RASTER-star):
    the points are projected a second time (Section 3.2), and a point on a
    tile of a kept cluster gets that cluster's label; the others get -1.  A
    label is the cluster's smallest tile (label_x, label_y) written as
    ((label_x + 2^31) << 32) | (label_y + 2^31), returned as int64 (two's
    complement), so that -1 is never a label.  A tile (kx, ky) is looked up
    among the result's tiles through the bijection kx * 2^32 + ky, which keeps
    the lexicographic order for |k| <= 2^31 - 2.  For a three-dimensional
    result (Section 3.6) the points are (n, 3) and the label is _id_3d of the
    cluster's smallest tile."""
    if result.kz is not None:
        row = _rows_3d(points, result, _scale(precision, scale))
        out = np.full(row.shape[0], -1, dtype=np.int64)
        on = row >= 0
        out[on] = _id_3d(result.label_x, result.label_y, result.label_z)[row[on]]
        return out
    kx, ky = project(points, _scale(precision, scale))
    out = np.full(kx.shape[0], -1, dtype=np.int64)
    if result.num_tiles == 0 or kx.shape[0] == 0:
        return out
    tiles = result.kx.astype(np.int64) * (1 << 32) + result.ky.astype(np.int64)
    order = np.argsort(tiles, kind="stable")
    tiles = tiles[order]
    lab = (((result.label_x[order].astype(np.int64) + (1 << 31)).astype(np.uint64) << np.uint64(32))
           | (result.label_y[order].astype(np.int64) + (1 << 31)).astype(np.uint64)).view(np.int64)
    q = kx * (1 << 32) + ky
    pos = np.searchsorted(tiles, q)
    hit = pos < tiles.shape[0]
    hit[hit] = tiles[pos[hit]] == q[hit]
    out[hit] = lab[pos[hit]]
    return out


def tile_points(points, result: OracleResult, precision: int | None = None,
                scale: float | None = None):
    """Points of every kept tile (RASTER', Section 3.4): the points are
    projected a second time (Section 3.2) and each point on a row's tile is
    listed under that row.  Returns (row_start, index) for the rows of
    ``result`` in its order: the points on row j are
    index[row_start[j]:row_start[j + 1]], ascending.  Points are (n, 3) for a
    three-dimensional result."""
    t = result.num_tiles
    if result.kz is not None:
        row = _rows_3d(points, result, _scale(precision, scale))
        point = np.flatnonzero(row >= 0)
        listed = point[np.lexsort((point, row[point]))]     # by row, then ascending point
        starts = np.zeros(t + 1, dtype=np.int64)
        starts[1:] = np.add.accumulate(np.bincount(row[point], minlength=t))
        return starts, listed.astype(np.int64)
    kx, ky = project(points, _scale(precision, scale))
    row_start = np.zeros(t + 1, dtype=np.int64)
    if t == 0 or kx.shape[0] == 0:
        return row_start, np.zeros(0, dtype=np.int64)
    tiles = result.kx.astype(np.int64) * (1 << 32) + result.ky.astype(np.int64)
    order = np.argsort(tiles, kind="stable")
    q = kx * (1 << 32) + ky
    pos = np.searchsorted(tiles[order], q)
    hit = pos < t
    hit[hit] = tiles[order][pos[hit]] == q[hit]
    point = np.nonzero(hit)[0]
    row = order[pos[hit]]
    by_row = np.argsort(row, kind="stable")          # rows in order, points ascending within a row
    row_start[1:] = np.cumsum(np.bincount(row, minlength=t))
    return row_start, point[by_row].astype(np.int64)


def cluster_chunks(chunks, tau: int, mu: int, precision: int | None = None,
                   scale: float | None = None, metric: str = "chebyshev", delta: int = 1,
                   window: bool = False, dims: int = 2) -> OracleResult:
    """RASTER over an iterable of point chunks (Section 3.6)."""
    st = OracleStream(_scale(precision, scale), tau, mu, metric, delta, window, dims)
    try:
        for c in chunks:
            st.feed(c)
        return st.finish()
    finally:
        st.close()

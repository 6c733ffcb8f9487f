"""Multi-core CPU P-RASTER (Section 3.5, Algorithms 2 and 3): a host baseline
beside the GPU library.

A ctypes wrapper around ``p_raster.cpp``, built with g++.  It is neither the
product path nor the oracle: the GPU library never calls it, and it shares no
code with either.  ``bench.py`` times it on the host cores and the CPU tests
check it against the oracle.  Results have the oracle's layout: ``kx``,
``ky``, ``count``, ``label_x``, ``label_y`` as numpy arrays sorted by tile.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "p_raster.cpp")
_LIB = os.path.join(_HERE, "libpraster.so")
_lib = None


class PRasterError(RuntimeError):
    def __init__(self, code: int):
        super().__init__(f"praster_cluster failed with status {code}")
        self.code = code


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O3", "-std=c++17", "-pthread", "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        vp, i64 = ctypes.c_void_p, ctypes.c_int64
        lib.praster_cluster.argtypes = [vp, vp, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_uint64,
                                        ctypes.c_uint64, ctypes.c_int, ctypes.POINTER(vp)]
        lib.praster_cluster.restype = ctypes.c_int
        lib.praster_num_tiles.argtypes = [vp]
        lib.praster_num_tiles.restype = i64
        lib.praster_stats.argtypes = [vp, vp, vp]
        lib.praster_stats.restype = None
        lib.praster_rows.argtypes = [vp, vp, vp, vp, vp, vp]
        lib.praster_rows.restype = None
        lib.praster_free.argtypes = [vp]
        lib.praster_free.restype = None
        _lib = lib
    return _lib


@dataclass
class PRasterResult:
    kx: np.ndarray
    ky: np.ndarray
    count: np.ndarray
    label_x: np.ndarray
    label_y: np.ndarray
    stats: dict = field(default_factory=dict)

    @property
    def num_tiles(self) -> int:
        return int(self.kx.shape[0])


def default_threads() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cluster(chunks, tau: int, mu: int, scale: float, threads: int | None = None) -> PRasterResult:
    """P-RASTER over one point array or a list of chunks ((n, 2) float32 or
    float64 arrays; all chunks of one call share a dtype)."""
    if isinstance(chunks, np.ndarray):
        chunks = [chunks]
    arrs = [np.ascontiguousarray(np.asarray(c).reshape(-1, 2)) for c in chunks]
    dtypes = {a.dtype for a in arrs if a.shape[0]}
    if len(dtypes) > 1:
        raise ValueError("chunks of one call must share a dtype")
    dt = dtypes.pop() if dtypes else np.dtype(np.float64)
    if dt not in (np.float32, np.float64):
        arrs = [a.astype(np.float64) for a in arrs]
        dt = np.dtype(np.float64)
    arrs = [a if a.dtype == dt else a.astype(dt) for a in arrs]
    lib = _load()
    ptrs = (ctypes.c_void_p * max(1, len(arrs)))(*[a.ctypes.data for a in arrs])
    cnts = (ctypes.c_int64 * max(1, len(arrs)))(*[a.shape[0] for a in arrs])
    out = ctypes.c_void_p()
    rc = lib.praster_cluster(ptrs, cnts, len(arrs), 1 if dt == np.float32 else 2, float(scale), int(tau), int(mu),
                             int(default_threads() if threads is None else threads), ctypes.byref(out))
    if rc != 0:
        raise PRasterError(rc)
    try:
        t = lib.praster_num_tiles(out)
        kx, ky, lx, ly = (np.empty(t, np.int64) for _ in range(4))
        c = np.empty(t, np.uint64)
        lib.praster_rows(out, kx.ctypes.data, ky.ctypes.data, c.ctypes.data, lx.ctypes.data, ly.ctypes.data)
        st = np.zeros(4, np.int64)
        sec = np.zeros(5, np.float64)
        lib.praster_stats(out, st.ctypes.data, sec.ctypes.data)
    finally:
        lib.praster_free(out)
    stats = dict(distinct=int(st[0]), significant=int(st[1]), clusters=int(st[2]), join_candidates=int(st[3]),
                 tiles=int(t), seconds=dict(zip(("project", "join_threshold", "slices", "border_join", "output"),
                                                sec.tolist())))
    return PRasterResult(kx, ky, c, lx, ly, stats)

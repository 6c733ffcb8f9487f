"""Python binding of the MI355X RASTER library (``libraster.so``).

Argument marshalling only: every step of the clustering runs in the library's
HIP kernels.  PyTorch supplies device memory (point tensors, output tensors)
and the HIP stream; nothing here computes tiles, counts or clusters.

    import paper_1907_03620_amd as raster
    res = raster.cluster(points_cuda_f64, precision=2, tau=5, mu=4)
    kx, ky, count, label = res.tensors()       # device tensors, one row per tile

If the library is not built, every call raises ``RasterNotBuilt``: there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

__all__ = [
    "cluster", "Stream", "cluster_batch", "Server", "Result", "RasterError", "RasterNotBuilt",
    "set_tuning", "get_tuning", "library_path", "load", "memory_stats", "F32", "F64", "cluster_noalloc",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libraster.so")

F32, F64 = 1, 2
STATUS = {0: "RASTER_OK", -1: "RASTER_E_INVAL", -2: "RASTER_E_RANGE", -3: "RASTER_E_NOMEM",
          -4: "RASTER_E_DEVICE", -5: "RASTER_E_STATE", -6: "RASTER_E_BUDGET"}
E_INVAL, E_RANGE, E_NOMEM, E_DEVICE, E_STATE, E_BUDGET = -1, -2, -3, -4, -5, -6


class RasterNotBuilt(RuntimeError):
    pass


class RasterError(RuntimeError):
    def __init__(self, code: int, what: str, detail: str = ""):
        super().__init__(f"{what}: {STATUS.get(code, code)}" + (f" ({detail})" if detail else ""))
        self.code = code


class _Options(ctypes.Structure):
    _fields_ = [("metric", ctypes.c_int), ("delta", ctypes.c_uint32), ("square_step", ctypes.c_uint32),
                ("dims", ctypes.c_uint32)]


class _Stats(ctypes.Structure):
    _fields_ = [("n_points", ctypes.c_int64), ("distinct_tiles", ctypes.c_int64),
                ("significant_tiles", ctypes.c_int64), ("components", ctypes.c_int64),
                ("clusters", ctypes.c_int64), ("tiles", ctypes.c_int64),
                ("table_capacity", ctypes.c_int64), ("grow_events", ctypes.c_int64),
                ("us_contract", ctypes.c_float), ("us_threshold", ctypes.c_float),
                ("us_agglomerate", ctypes.c_float), ("us_filter", ctypes.c_float),
                ("count_launches", ctypes.c_int64), ("us_count_kernel", ctypes.c_float),
                ("us_bin_keys", ctypes.c_float), ("us_aggregate", ctypes.c_float),
                ("flushes", ctypes.c_int32), ("redone", ctypes.c_int32),
                ("key_frame", ctypes.c_int32), ("reserved_", ctypes.c_int32)]


class _Tuning(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("items", ctypes.c_int32),
                ("preagg_slots", ctypes.c_int32), ("load_factor", ctypes.c_float),
                ("mode", ctypes.c_int32), ("group_mpoints", ctypes.c_int32)]


class _Job(ctypes.Structure):
    _fields_ = [("d_points", ctypes.c_void_p), ("n", ctypes.c_int64), ("dt", ctypes.c_int),
                ("precision", ctypes.c_int32), ("scale", ctypes.c_double),
                ("tau", ctypes.c_uint32), ("mu", ctypes.c_uint32)]


_lib = None


def library_path() -> str:
    return _LIB_PATH


def load():
    """Load libraster.so (raises RasterNotBuilt if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RasterNotBuilt(f"{_LIB_PATH} is missing; build it with paper_1907_03620_amd.build.build()")
    lib = ctypes.CDLL(_LIB_PATH)
    vp, i64, i32, u32, dbl, st = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32,
                                  ctypes.c_double, ctypes.c_int)
    pp = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "raster_cluster": (st, [vp, i64, ctypes.c_int, i32, u32, u32, vp, pp]),
        "raster_cluster_scaled": (st, [vp, i64, ctypes.c_int, dbl, u32, u32, vp, pp]),
        "raster_cluster_noalloc": (st, [vp, i64, ctypes.c_int, i32, u32, u32, vp, vp, vp, vp, vp, i64,
                                        ctypes.POINTER(i64), ctypes.POINTER(_Stats)]),
        "raster_result_num_tiles": (i64, [vp]),
        "raster_result_num_clusters": (i64, [vp]),
        "raster_result_arrays": (st, [vp, pp, pp, pp, pp]),
        "raster_result_copy": (st, [vp, vp, vp, vp, vp, vp]),
        "raster_result_stats": (st, [vp, ctypes.POINTER(_Stats)]),
        "raster_result_free": (None, [vp]),
        "raster_result_point_labels": (st, [vp, vp, i64, ctypes.c_int, vp, vp]),
        "raster_result_tile_points": (st, [vp, vp, i64, ctypes.c_int, vp, vp, i64, ctypes.POINTER(i64), vp]),
        "raster_begin": (st, [i32, u32, u32, i64, vp, pp]),
        "raster_begin_scaled": (st, [dbl, u32, u32, i64, vp, pp]),
        "raster_begin_delta": (st, [dbl, u32, u32, ctypes.c_int, u32, i64, vp, pp]),
        "raster_cluster_delta": (st, [vp, i64, ctypes.c_int, dbl, u32, u32, ctypes.c_int, u32, vp, pp]),
        "raster_cluster_opts": (st, [vp, i64, ctypes.c_int, dbl, u32, u32, ctypes.POINTER(_Options), vp, pp]),
        "raster_cluster_p_opts": (st, [vp, i64, ctypes.c_int, i32, u32, u32, ctypes.POINTER(_Options), vp, pp]),
        "raster_begin_p_opts": (st, [i32, u32, u32, ctypes.POINTER(_Options), i64, vp, pp]),
        "raster_result_kz": (st, [vp, ctypes.POINTER(vp)]),
        "raster_result_copy_kz": (st, [vp, vp, vp]),
        "raster_begin_opts": (st, [dbl, u32, u32, ctypes.POINTER(_Options), i64, vp, pp]),
        "raster_feed_chunk": (st, [vp, vp, i64, ctypes.c_int]),
        "raster_finish": (st, [vp, pp]),
        "raster_stream_tiles": (st, [vp, vp, vp, i64, ctypes.POINTER(i64)]),
        "raster_stream_destroy": (None, [vp]),
        "raster_cluster_batch": (st, [ctypes.POINTER(_Job), i32, vp, pp]),
        "raster_cluster_batch_opts": (st, [ctypes.POINTER(_Job), ctypes.POINTER(_Options), i32, vp, pp]),
        "raster_server_create": (st, [ctypes.c_size_t, i32, pp]),
        "raster_server_submit": (st, [vp, ctypes.POINTER(_Job), ctypes.POINTER(ctypes.c_uint64)]),
        "raster_server_submit_opts": (st, [vp, ctypes.POINTER(_Job), ctypes.POINTER(_Options),
                                           ctypes.POINTER(ctypes.c_uint64)]),
        "raster_server_submit_stream": (st, [vp, ctypes.POINTER(_Job), ctypes.POINTER(_Options), vp,
                                             ctypes.POINTER(ctypes.c_uint64)]),
        "raster_server_wait": (st, [vp, ctypes.c_uint64, pp, ctypes.POINTER(dbl)]),
        "raster_server_memory": (st, [vp, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]),
        "raster_memory_stats": (st, [ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t),
                                     ctypes.POINTER(ctypes.c_size_t), i32]),
        "raster_server_destroy": (None, [vp]),
        "raster_set_tuning": (st, [ctypes.POINTER(_Tuning)]),
        "raster_get_tuning": (st, [ctypes.POINTER(_Tuning)]),
        "raster_status_string": (ctypes.c_char_p, [st]),
        "raster_last_error": (ctypes.c_char_p, []),
        "raster_version": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(rc: int, what: str):
    if rc != 0:
        detail = load().raster_last_error()
        raise RasterError(rc, what, detail.decode() if detail else "")


def _torch():
    import torch
    return torch


def _stream_handle(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _points(points, dims: int = 2):
    """(pointer, n, dtype) of a CUDA tensor of shape (n, dims)."""
    torch = _torch()
    if not isinstance(points, torch.Tensor):
        raise TypeError("points must be a torch tensor on the GPU")
    if points.device.type != "cuda":
        raise ValueError("points must be on the GPU (device memory)")
    if points.dim() != 2 or points.shape[1] != dims:
        raise ValueError(f"points must have shape (n, {dims})")
    if not points.is_contiguous():
        raise ValueError(f"points must be contiguous (row-major (n, {dims}))")
    if points.dtype == torch.float64:
        dt = F64
    elif points.dtype == torch.float32:
        dt = F32
    else:
        raise ValueError("points must be float32 or float64")
    return ctypes.c_void_p(points.data_ptr()), int(points.shape[0]), dt


class Result:
    """One clustering result; the rows live in library-owned device memory."""

    def __init__(self, handle: ctypes.c_void_p, stream=None):
        self._h = handle
        self._stream = stream
        s = _Stats()
        _check(load().raster_result_stats(self._h, ctypes.byref(s)), "raster_result_stats")
        self.stats = {name: getattr(s, name) for name, _ in _Stats._fields_}

    @property
    def num_tiles(self) -> int:
        return int(self.stats["tiles"])

    @property
    def num_clusters(self) -> int:
        return int(self.stats["clusters"])

    def tensors(self, device=None):
        """(kx int32, ky int32, count uint32, label uint64) device tensors."""
        torch = _torch()
        t = self.num_tiles
        device = device or torch.device("cuda", torch.cuda.current_device())
        kx = torch.empty(t, dtype=torch.int32, device=device)
        ky = torch.empty(t, dtype=torch.int32, device=device)
        cnt = torch.empty(t, dtype=torch.uint32, device=device)
        lab = torch.empty(t, dtype=torch.uint64, device=device)
        if t:
            st = _stream_handle(self._stream)
            _check(load().raster_result_copy(self._h, ctypes.c_void_p(kx.data_ptr()), ctypes.c_void_p(ky.data_ptr()),
                                             ctypes.c_void_p(cnt.data_ptr()), ctypes.c_void_p(lab.data_ptr()), st),
                   "raster_result_copy")
        return kx, ky, cnt, lab

    def numpy(self, sort: bool = True):
        """Host copies (kx, ky, count, label) as numpy arrays, sorted by tile if ``sort``
        (three-dimensional results: (kx, ky, kz, count, label))."""
        import numpy as np
        kx, ky, cnt, lab = (a.cpu().numpy() for a in self.tensors())
        kz = self.kz().cpu().numpy() if self.dims == 3 else None
        if sort and kx.shape[0]:
            order = np.lexsort((ky, kx)) if kz is None else np.lexsort((kz, ky, kx))
            kx, ky, cnt, lab = kx[order], ky[order], cnt[order], lab[order]
            kz = kz[order] if kz is not None else None
        return (kx, ky, cnt, lab) if kz is None else (kx, ky, kz, cnt, lab)

    @property
    def dims(self) -> int:
        p = ctypes.c_void_p()
        _check(load().raster_result_kz(self._h, ctypes.byref(p)), "raster_result_kz")
        return 3 if p.value else 2

    def kz(self, device=None):
        """The third tile coordinate of every row (three-dimensional results), int32."""
        torch = _torch()
        device = device or torch.device("cuda", torch.cuda.current_device())
        kz = torch.empty(self.num_tiles, dtype=torch.int32, device=device)
        _check(load().raster_result_copy_kz(self._h, ctypes.c_void_p(kz.data_ptr()), _stream_handle(self._stream)),
               "raster_result_copy_kz")
        return kz

    def point_labels(self, points, stream=None):
        """Label of every point (Section 4.1, RASTER-star): the cluster label of its tile as
        int64 (the biased key of the cluster's smallest tile, read as
        two's complement), or -1 for a point on no kept tile.  Points are (n, 3)
        for a three-dimensional result."""
        torch = _torch()
        p, n, dt = _points(points, self.dims)
        out = torch.empty(n, dtype=torch.int64, device=points.device)
        st = _stream_handle(stream if stream is not None else self._stream)
        _check(load().raster_result_point_labels(self._h, p, n, dt, ctypes.c_void_p(out.data_ptr()), st),
               "raster_result_point_labels")
        return out

    def tile_points(self, points, stream=None):
        """Points of every kept tile (RASTER', Section 3.4): ``(row_start,
        index)`` as int64 tensors, where the points on row j of
        :meth:`tensors` are ``index[row_start[j]:row_start[j + 1]]`` (indices
        into ``points``, unordered within a row).  Points are (n, 3) for a
        three-dimensional result."""
        torch = _torch()
        p, n, dt = _points(points, self.dims)
        start = torch.empty(self.num_tiles + 1, dtype=torch.int64, device=points.device)
        index = torch.empty(max(n, 1), dtype=torch.int64, device=points.device)
        kept = ctypes.c_int64()
        st = _stream_handle(stream if stream is not None else self._stream)
        _check(load().raster_result_tile_points(self._h, p, n, dt, ctypes.c_void_p(start.data_ptr()),
                                                ctypes.c_void_p(index.data_ptr()), n, ctypes.byref(kept), st),
               "raster_result_tile_points")
        return start, index[: kept.value]

    def free(self):
        if self._h:
            load().raster_result_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


METRICS = {"chebyshev": 0, "manhattan": 1}


def _options(metric: str, delta: int, square: bool, dims: int = 2):
    """The options struct, or None for the defaults."""
    if metric == "chebyshev" and delta == 1 and not square and dims == 2:
        return None
    if metric not in METRICS:
        raise RasterError(E_INVAL, "options", f"unknown metric {metric!r}")
    return _Options(METRICS[metric], int(delta), int(bool(square)), int(dims))


def _dims_of(points) -> int:
    return 3 if points.dim() == 2 and points.shape[1] == 3 else 2


def _need_precision(precision, scale, what):
    if scale is None and precision is None:
        raise RasterError(E_INVAL, what, "give precision or scale")


def cluster(points, tau: int, mu: int, precision: int | None = None, scale: float | None = None,
            stream=None, metric: str = "chebyshev", delta: int = 1, square: bool = False) -> Result:
    """RASTER on one resident point tensor (Algorithm 1).  ``metric`` and
    ``delta`` choose the neighbourhood of the agglomeration (Section 3.2); the
    default is the eight adjacent tiles.  ``square`` adds the 2x2 post-step
    of Section 3.6.  Points of shape (n, 3) are clustered in three dimensions
    (Section 3.6's generalisation)."""
    lib = load()
    dims = _dims_of(points)
    p, n, dt = _points(points, dims)
    out = ctypes.c_void_p()
    st = _stream_handle(stream)
    opts = _options(metric, delta, square, dims)
    _need_precision(precision, scale, "raster_cluster")
    if opts is not None and scale is not None:
        rc = lib.raster_cluster_opts(p, n, dt, float(scale), int(tau), int(mu), ctypes.byref(opts), st,
                                     ctypes.byref(out))
    elif opts is not None:
        rc = lib.raster_cluster_p_opts(p, n, dt, int(precision), int(tau), int(mu), ctypes.byref(opts), st,
                                       ctypes.byref(out))
    elif scale is not None:
        rc = lib.raster_cluster_scaled(p, n, dt, float(scale), int(tau), int(mu), st, ctypes.byref(out))
    else:
        rc = lib.raster_cluster(p, n, dt, int(precision), int(tau), int(mu), st, ctypes.byref(out))
    _check(rc, "raster_cluster")
    return Result(out, stream)


NOALLOC_MAX_POINTS = 1 << 19


def cluster_noalloc(points, tau: int, mu: int, precision: int, max_rows: int | None = None, stream=None):
    """raster_cluster_noalloc: Algorithm 1 (eight neighbours) on at most
    NOALLOC_MAX_POINTS points with the library's fixed scratch, so that the
    library allocates no device memory.  The output rows go to device tensors
    allocated here, on the caller's side of the boundary, with room for
    ``max_rows`` rows (default: one per point).  Returns ``(kx, ky, count,
    label, stats)``: int32, int32, uint32 and uint64 tensors of the t rows (in
    no particular order) and the counters as a dict."""
    torch = _torch()
    lib = load()
    p, n, dt = _points(points, 2)
    cap = n if max_rows is None else int(max_rows)
    dev = points.device
    kx = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
    ky = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
    cnt = torch.empty(max(cap, 1), dtype=torch.uint32, device=dev)
    lab = torch.empty(max(cap, 1), dtype=torch.uint64, device=dev)
    rows = ctypes.c_int64()
    s = _Stats()
    rc = lib.raster_cluster_noalloc(p, n, dt, int(precision), int(tau), int(mu), _stream_handle(stream),
                                    ctypes.c_void_p(kx.data_ptr()), ctypes.c_void_p(ky.data_ptr()),
                                    ctypes.c_void_p(cnt.data_ptr()), ctypes.c_void_p(lab.data_ptr()), cap,
                                    ctypes.byref(rows), ctypes.byref(s))
    if rc != 0:
        err = RasterError(rc, "raster_cluster_noalloc", (lib.raster_last_error() or b"").decode())
        err.rows = int(rows.value)
        raise err
    t = int(rows.value)
    stats = {name: getattr(s, name) for name, _ in _Stats._fields_}
    return kx[:t], ky[:t], cnt[:t], lab[:t], stats


class Stream:
    """Chunked contraction with a device-resident table (Section 3.6)."""

    def __init__(self, tau: int, mu: int, precision: int | None = None, scale: float | None = None,
                 tile_hint: int = 0, stream=None, metric: str = "chebyshev", delta: int = 1, square: bool = False,
                 dims: int = 2):
        self._lib = load()
        self._stream = stream
        self._dims = int(dims)
        self._h = ctypes.c_void_p()
        self._keep = []  # chunks stay referenced until the stream has consumed them
        st = _stream_handle(stream)
        opts = _options(metric, delta, square, self._dims)
        _need_precision(precision, scale, "raster_begin")
        if opts is not None and scale is not None:
            rc = self._lib.raster_begin_opts(float(scale), int(tau), int(mu), ctypes.byref(opts), int(tile_hint), st,
                                             ctypes.byref(self._h))
        elif opts is not None:
            rc = self._lib.raster_begin_p_opts(int(precision), int(tau), int(mu), ctypes.byref(opts),
                                               int(tile_hint), st, ctypes.byref(self._h))
        elif scale is not None:
            rc = self._lib.raster_begin_scaled(float(scale), int(tau), int(mu), int(tile_hint), st,
                                               ctypes.byref(self._h))
        else:
            rc = self._lib.raster_begin(int(precision), int(tau), int(mu), int(tile_hint), st, ctypes.byref(self._h))
        _check(rc, "raster_begin")

    def feed(self, points) -> None:
        p, n, dt = _points(points, self._dims)
        self._keep.append(points)
        _check(self._lib.raster_feed_chunk(self._h, p, n, dt), "raster_feed_chunk")

    def tiles(self):
        """All (key uint64, count uint32) pairs counted so far, as device tensors."""
        torch = _torch()
        m = ctypes.c_int64()
        _check(self._lib.raster_stream_tiles(self._h, None, None, 0, ctypes.byref(m)), "raster_stream_tiles")
        dev = torch.device("cuda", torch.cuda.current_device())
        keys = torch.empty(m.value, dtype=torch.uint64, device=dev)
        cnts = torch.empty(m.value, dtype=torch.uint32, device=dev)
        _check(self._lib.raster_stream_tiles(self._h, ctypes.c_void_p(keys.data_ptr()),
                                             ctypes.c_void_p(cnts.data_ptr()), m.value, ctypes.byref(m)),
               "raster_stream_tiles")
        return keys, cnts

    def finish(self) -> Result:
        out = ctypes.c_void_p()
        _check(self._lib.raster_finish(self._h, ctypes.byref(out)), "raster_finish")
        self._keep.clear()
        return Result(out, self._stream)

    def close(self) -> None:
        if self._h:
            self._lib.raster_stream_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _job(points, precision=None, tau=5, mu=4, scale=None) -> _Job:
    p, n, dt = _points(points)
    return _Job(p, n, dt, int(precision if precision is not None else 0),
                float(scale) if scale is not None else 0.0, int(tau), int(mu))


def cluster_batch(jobs, stream=None) -> list:
    """jobs: iterable of dicts with keys points, tau, mu and precision or
    scale, and optionally metric, delta (the job's neighbourhood, Section 3.2)
    and square (the 2x2 post-step of Section 3.6); jobs with other options
    than the defaults go through raster_cluster_batch_opts."""
    lib = load()
    jobs = [dict(j) for j in jobs]
    var = [(j.pop("metric", "chebyshev"), int(j.pop("delta", 1)), bool(j.pop("square", False))) for j in jobs]
    arr = (_Job * max(1, len(jobs)))(*[_job(**j) for j in jobs])
    outs = (ctypes.c_void_p * max(1, len(jobs)))()
    if all(m == "chebyshev" and d == 1 and not q for m, d, q in var):
        _check(lib.raster_cluster_batch(arr, len(jobs), _stream_handle(stream), outs), "raster_cluster_batch")
    else:
        for m, _, _ in var:
            if m not in METRICS:
                raise RasterError(E_INVAL, "cluster_batch", f"unknown metric {m!r}")
        opts = (_Options * len(jobs))(*[_Options(METRICS[m], d, int(q), 2) for m, d, q in var])
        _check(lib.raster_cluster_batch_opts(arr, opts, len(jobs), _stream_handle(stream), outs),
               "raster_cluster_batch_opts")
    return [Result(ctypes.c_void_p(outs[i]), stream) for i in range(len(jobs))]


class Server:
    """Serving loop with memory-budget admission and continuous batching."""

    def __init__(self, budget_bytes: int, max_slots: int = 4):
        self._lib = load()
        self._h = ctypes.c_void_p()
        self._keep = {}
        _check(self._lib.raster_server_create(int(budget_bytes), int(max_slots), ctypes.byref(self._h)),
               "raster_server_create")

    def submit(self, points, tau: int, mu: int, precision: int | None = None, scale: float | None = None,
               metric: str = "chebyshev", delta: int = 1, square: bool = False, stream=None) -> int:
        """Queue a job; its device work is ordered after the work already
        enqueued on ``stream`` (default: the current torch stream), which may
        still be producing the points."""
        job = _job(points, precision, tau, mu, scale)
        t = ctypes.c_uint64()
        opts = _options(metric, delta, square)
        _check(self._lib.raster_server_submit_stream(self._h, ctypes.byref(job),
                                                     ctypes.byref(opts) if opts is not None else None,
                                                     _stream_handle(stream), ctypes.byref(t)),
               "raster_server_submit_stream")
        self._keep[t.value] = points
        return t.value

    def memory(self):
        """(budget, largest footprint charged at once) in bytes."""
        b, p = ctypes.c_size_t(), ctypes.c_size_t()
        _check(self._lib.raster_server_memory(self._h, ctypes.byref(b), ctypes.byref(p)), "raster_server_memory")
        return b.value, p.value

    def wait(self, ticket: int):
        out = ctypes.c_void_p()
        lat = ctypes.c_double()
        rc = self._lib.raster_server_wait(self._h, ctypes.c_uint64(ticket), ctypes.byref(out), ctypes.byref(lat))
        self._keep.pop(ticket, None)
        _check(rc, "raster_server_wait")
        return Result(out), lat.value

    def close(self):
        if self._h:
            self._lib.raster_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class Tuning:
    block: int = 256
    items: int = 4
    preagg_slots: int = 0
    load_factor: float = 0.6
    mode: int = 0
    group_mpoints: int = 512


def set_tuning(t: Tuning | None = None, **kw) -> None:
    lib = load()
    if t is None and not kw:
        _check(lib.raster_set_tuning(None), "raster_set_tuning")
        return
    t = t or Tuning()
    for k, v in kw.items():
        setattr(t, k, v)
    c = _Tuning(int(t.block), int(t.items), int(t.preagg_slots), float(t.load_factor), int(t.mode),
                int(t.group_mpoints))
    _check(lib.raster_set_tuning(ctypes.byref(c)), "raster_set_tuning")


def memory_stats(reset_peak: bool = False):
    """(used, cached, peak_used) device bytes of the library's pool on the
    current device; ``reset_peak`` starts a new peak window."""
    u, c, p = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    _check(load().raster_memory_stats(ctypes.byref(u), ctypes.byref(c), ctypes.byref(p), int(bool(reset_peak))),
           "raster_memory_stats")
    return u.value, c.value, p.value


def get_tuning() -> Tuning:
    c = _Tuning()
    _check(load().raster_get_tuning(ctypes.byref(c)), "raster_get_tuning")
    return Tuning(c.block, c.items, c.preagg_slots, c.load_factor, c.mode, c.group_mpoints)

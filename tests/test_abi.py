"""The C-ABI library loads and exports every symbol include/raster.h declares.

No GPU is needed: these tests only load the shared library and call the
argument checks, which return before any HIP call is made.
"""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "raster.h")
LIB = os.path.join(ROOT, "paper_1907_03620_amd", "libraster.so")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b(raster_[a-z_]+)\s*\(", src))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1907_03620_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = _declared()
    for must in ["raster_cluster", "raster_cluster_scaled", "raster_begin", "raster_feed_chunk",
                 "raster_finish", "raster_cluster_batch", "raster_server_create", "raster_server_submit",
                 "raster_server_wait", "raster_result_arrays", "raster_result_free"]:
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_library_does_not_contain_the_oracle():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    assert "oracle_" not in out
    exported = {l.split()[-1] for l in out.splitlines() if l.strip()}
    assert any(s.startswith("raster_cluster") for s in exported)


def test_argument_errors_without_gpu(lib):
    lib.raster_cluster.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_int32,
                                   ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p,
                                   ctypes.POINTER(ctypes.c_void_p)]
    lib.raster_cluster.restype = ctypes.c_int
    lib.raster_cluster_scaled.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double,
                                          ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p,
                                          ctypes.POINTER(ctypes.c_void_p)]
    lib.raster_cluster_scaled.restype = ctypes.c_int
    lib.raster_last_error.restype = ctypes.c_char_p
    lib.raster_status_string.restype = ctypes.c_char_p
    out = ctypes.c_void_p(1234)
    fake = ctypes.c_void_p(4096)
    cases = [
        dict(p=fake, n=10, dt=2, prec=2, tau=0, mu=4),     # tau 0
        dict(p=fake, n=10, dt=2, prec=2, tau=5, mu=0),     # mu 0
        dict(p=fake, n=10, dt=3, prec=2, tau=5, mu=4),     # unknown dtype
        dict(p=None, n=10, dt=2, prec=2, tau=5, mu=4),     # NULL with n > 0
        dict(p=fake, n=-1, dt=2, prec=2, tau=5, mu=4),     # negative n
        dict(p=fake, n=10, dt=2, prec=16, tau=5, mu=4),    # precision out of range
        dict(p=fake, n=10, dt=2, prec=-1, tau=5, mu=4),
        dict(p=ctypes.c_void_p(4104), n=10, dt=2, prec=2, tau=5, mu=4),  # 8-byte aligned f64
    ]
    for c in cases:
        rc = lib.raster_cluster(c["p"], c["n"], c["dt"], c["prec"], c["tau"], c["mu"], None, ctypes.byref(out))
        assert rc == -1, c
        assert out.value is None
        assert lib.raster_last_error()
    for scale in [0.0, -1.0, float("inf"), float("nan")]:
        rc = lib.raster_cluster_scaled(fake, 10, 2, scale, 5, 4, None, ctypes.byref(out))
        assert rc == -1
    assert lib.raster_status_string(-2) == b"RASTER_E_RANGE"


def test_tuning_validation(lib):
    class T(ctypes.Structure):
        _fields_ = [("block", ctypes.c_int32), ("items", ctypes.c_int32),
                    ("preagg_slots", ctypes.c_int32), ("load_factor", ctypes.c_float),
                    ("mode", ctypes.c_int32), ("group_mpoints", ctypes.c_int32)]
    lib.raster_set_tuning.argtypes = [ctypes.POINTER(T)]
    lib.raster_get_tuning.argtypes = [ctypes.POINTER(T)]
    for bad in [T(100, 4, 0, 0.5, 0, 256), T(256, 3, 0, 0.5, 0, 256), T(256, 4, 300, 0.5, 0, 256),
                T(256, 4, 0, 0.95, 0, 256), T(2048, 4, 0, 0.5, 0, 256), T(256, 4, 0, 0.5, 4, 256),
                T(256, 4, 0, 0.5, 0, 0), T(256, 4, 0, 0.5, 0, 5000)]:
        assert lib.raster_set_tuning(ctypes.byref(bad)) == -1
    good = T(512, 8, 2048, 0.4, 2, 64)
    assert lib.raster_set_tuning(ctypes.byref(good)) == 0
    got = T()
    assert lib.raster_get_tuning(ctypes.byref(got)) == 0
    assert (got.block, got.items, got.preagg_slots, got.mode, got.group_mpoints) == (512, 8, 2048, 2, 64)
    assert lib.raster_set_tuning(None) == 0
    assert lib.raster_get_tuning(ctypes.byref(got)) == 0
    assert (got.block, got.items, got.preagg_slots, got.mode, got.group_mpoints) == (256, 4, 0, 0, 512)


def test_binding_refuses_cpu_tensors():
    import torch
    import paper_1907_03620_amd as raster
    with pytest.raises(ValueError):
        raster.cluster(torch.zeros((4, 2), dtype=torch.float64), precision=1, tau=1, mu=1)

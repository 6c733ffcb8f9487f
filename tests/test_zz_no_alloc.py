"""raster_cluster_noalloc (the plain call with the library's fixed scratch and
caller-owned output rows) against raster_cluster on the same points, through
the C ABI: the same rows as a set and the same counters, on two calls in a row
(the second on a smaller input, so that it runs on scratch the first one
left behind), and the argument errors of its own.

Algorithm 1 (eight neighbours); the oracle is checked beside it.
"""
import numpy as np
import pytest

import oracle
import synth
from digest import unbias_label
from gpu_util import dev

pytestmark = pytest.mark.gpu

STATS = ("n_points", "distinct_tiles", "significant_tiles", "components", "clusters", "tiles")


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU test run without a GPU"
    return t


@pytest.fixture(scope="module")
def raster(torch):
    import paper_1907_03620_amd as r
    r.load()
    r.set_tuning(None)
    return r


def sorted_rows(kx, ky, cnt, lab):
    kx, ky, cnt, lab = (a.cpu().numpy() for a in (kx, ky, cnt, lab))
    order = np.lexsort((ky, kx))
    lx, ly = unbias_label(lab[order])
    return (kx[order].astype(np.int64), ky[order].astype(np.int64), cnt[order].astype(np.uint64), lx, ly)


def check_against_plain(raster, torch, pts, precision, tau, mu, what):
    d = dev(pts, torch)
    used0, cached0, _ = raster.memory_stats()
    kx, ky, cnt, lab, st = raster.cluster_noalloc(d, tau=tau, mu=mu, precision=precision)
    torch.cuda.synchronize()
    used1, cached1, _ = raster.memory_stats()
    assert (used1, cached1) == (used0, cached0), f"{what}: the library's device pool changed during the call"
    got = sorted_rows(kx, ky, cnt, lab)
    plain = raster.cluster(d, precision=precision, tau=tau, mu=mu)
    want = sorted_rows(*plain.tensors())
    assert got[0].shape == want[0].shape, f"{what}: {got[0].shape[0]} rows vs {want[0].shape[0]} from raster_cluster"
    for name, a, b in zip(("kx", "ky", "count", "label_x", "label_y"), got, want):
        assert np.array_equal(a, b), f"{what}: {name} differs from raster_cluster"
    for k in STATS:
        assert int(st[k]) == int(plain.stats[k]), f"{what}: {k} {st[k]} vs {plain.stats[k]}"
    ref = oracle.cluster(pts, tau=tau, mu=mu, precision=precision)
    assert int(st["clusters"]) == int(ref.stats["clusters"]) and int(st["tiles"]) == int(ref.stats["tiles"])
    assert np.array_equal(got[0], ref.kx) and np.array_equal(got[1], ref.ky), what
    assert np.array_equal(got[2], ref.count), what
    assert np.array_equal(got[3], ref.label_x) and np.array_equal(got[4], ref.label_y), what
    return int(st["tiles"])


def test_two_calls_in_a_row_second_smaller(raster, torch):
    rng = synth.rng_for(7100)
    big = synth.blobs(rng, raster.NOALLOC_MAX_POINTS, 400, 100.0, 0.05, 0.05)  # the largest input allowed
    small = synth.plain_small(1)[:150_000]
    print(f"noalloc: {big.shape[0]} points, then {small.shape[0]}", flush=True)
    t1 = check_against_plain(raster, torch, big, 1, 5, 4, "first call (maximum size)")
    t2 = check_against_plain(raster, torch, small, 1, 5, 4, "second call (smaller)")
    assert t1 > 0 and t2 > 0
    # a third, smaller still, in FP32 and at another precision: scratch left by two calls
    f32 = np.ascontiguousarray(synth.plain_small(3)[:40_000].astype(np.float32))
    check_against_plain(raster, torch, f32, 2, 3, 2, "third call (FP32)")


def test_empty_and_ragged(raster, torch):
    kx, ky, cnt, lab, st = raster.cluster_noalloc(torch.zeros((0, 2), dtype=torch.float64, device="cuda"),
                                                  tau=1, mu=1, precision=1)
    assert kx.shape[0] == 0 and st["tiles"] == 0 and st["n_points"] == 0
    rng = synth.rng_for(7101)
    for n in (1, 63, 4097):
        pts = synth.blobs(rng, n, 3, 10.0, 0.05, 0.0)
        check_against_plain(raster, torch, pts, 1, 1, 1, f"{n} points")


def test_errors(raster, torch):
    too_many = torch.zeros((raster.NOALLOC_MAX_POINTS + 1, 2), dtype=torch.float64, device="cuda")
    with pytest.raises(raster.RasterError, match="E_INVAL"):
        raster.cluster_noalloc(too_many, tau=5, mu=4, precision=1)
    pts = synth.plain_small(1)[:100_000]
    d = dev(pts, torch)
    _, _, _, _, st = raster.cluster_noalloc(d, tau=5, mu=4, precision=1)
    t = int(st["tiles"])
    assert t > 10
    with pytest.raises(raster.RasterError, match="E_INVAL") as e:
        raster.cluster_noalloc(d, tau=5, mu=4, precision=1, max_rows=t - 1)
    assert e.value.rows == t
    bad = d.clone()
    bad[17, 0] = float("nan")
    with pytest.raises(raster.RasterError, match="E_RANGE"):
        raster.cluster_noalloc(bad, tau=5, mu=4, precision=1)
    with pytest.raises(raster.RasterError, match="E_INVAL"):
        raster.cluster_noalloc(d, tau=0, mu=4, precision=1)
    # after the failures, and with exactly enough room
    kx, ky, cnt, lab, st2 = raster.cluster_noalloc(d, tau=5, mu=4, precision=1, max_rows=t)
    plain = raster.cluster(d, precision=1, tau=5, mu=4)
    for a, b in zip(sorted_rows(kx, ky, cnt, lab), sorted_rows(*plain.tensors())):
        assert np.array_equal(a, b)
    assert int(st2["tiles"]) == t

"""Helpers of the GPU parity tests: run the HIP path through the C ABI and
compare it with the oracle row by row."""
from __future__ import annotations

import numpy as np

from digest import unbias_label


def dev(a, torch):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def oracle_rows(res):
    """Oracle result as sorted (kx, ky, count, label_x, label_y) arrays."""
    return (res.kx.astype(np.int64), res.ky.astype(np.int64), res.count.astype(np.uint64),
            res.label_x.astype(np.int64), res.label_y.astype(np.int64))


def gpu_rows(res):
    """GPU result as sorted (kx, ky, count, label_x, label_y) arrays; the label
    (the biased key of the cluster's smallest tile) is decoded here, by the
    test, not by the library."""
    kx, ky, cnt, lab = res.numpy(sort=True)
    lx, ly = unbias_label(lab)
    return (kx.astype(np.int64), ky.astype(np.int64), cnt.astype(np.uint64), lx, ly)


def assert_same(gpu_res, orc_res, what=""):
    g = gpu_rows(gpu_res)
    o = oracle_rows(orc_res)
    assert g[0].shape == o[0].shape, f"{what}: {g[0].shape[0]} tiles on the GPU vs {o[0].shape[0]} in the oracle"
    for name, a, b in zip(("kx", "ky", "count", "label_x", "label_y"), g, o):
        bad = np.nonzero(a != b)[0]
        assert bad.size == 0, f"{what}: {name} differs at {bad.size} rows, first {bad[:5]}: {a[bad[:5]]} vs {b[bad[:5]]}"
    st = gpu_res.stats
    os_ = orc_res.stats
    for k_g, k_o in (("distinct_tiles", "distinct"), ("significant_tiles", "significant"),
                     ("components", "components"), ("clusters", "clusters"), ("tiles", "tiles"),
                     ("n_points", "n")):
        assert int(st[k_g]) == int(os_[k_o]), f"{what}: stat {k_g} {st[k_g]} vs {os_[k_o]}"


def same_result(a, b, what=""):
    ga, gb = gpu_rows(a), gpu_rows(b)
    assert ga[0].shape == gb[0].shape, what
    for x, y in zip(ga, gb):
        assert np.array_equal(x, y), what
    for k in ("distinct_tiles", "significant_tiles", "components", "clusters", "tiles", "n_points"):
        assert a.stats[k] == b.stats[k], (what, k)


def decode_keys(keys):
    keys = np.asarray(keys, dtype=np.uint64)
    kx = (keys >> np.uint64(32)).astype(np.int64) - (1 << 31)
    ky = (keys & np.uint64(0xFFFFFFFF)).astype(np.int64) - (1 << 31)
    return kx, ky

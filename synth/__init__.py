"""Seeded synthetic point sets shaped like the paper's GPS-canvas workloads.

The paper evaluates on data from its own generator (Section 4.2, "Data"):
cluster centres on a canvas, a few hundred points spread around each centre,
and the whole set shuffled.  Neither that generator nor its data is available,
so every workload here is a seeded stand-in with the same structure: 2-D
points around random centres, optional uniform background noise, shuffled
draw order.

This module only draws coordinates.  It holds none of the clustering
arithmetic (no projection, counting or adjacency) and is imported by both the
CPU oracle tests and the GPU path, which is the only thing they share.

Every generator uses numpy's PCG64 through ``default_rng(SeedSequence(seed))``
so that a seed names one exact point set on any machine.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "rng_for", "blobs", "blobs3d", "plain_small", "zipf_hot", "paper_scale_chunk",
    "paper_scale_centres", "batch_jobs", "served_trace", "served_parity_slice", "JobSpec",
    "PLAIN_SMALL", "ZIPF_HOT", "PAPER_SCALE",
]


def rng_for(seed) -> np.random.Generator:
    """PCG64 generator for an integer seed or a SeedSequence."""
    if isinstance(seed, np.random.SeedSequence):
        return np.random.default_rng(seed)
    return np.random.default_rng(np.random.SeedSequence(seed))


def _shuffle_rows(rng: np.random.Generator, a: np.ndarray) -> np.ndarray:
    return a[rng.permutation(a.shape[0])]


def blobs(rng: np.random.Generator, n: int, n_centres: int, box: float,
          sigma: float, noise_frac: float, dtype=np.float64) -> np.ndarray:
    """n points: a share ``noise_frac`` uniform over [0, box]^2, the rest
    around centres drawn uniformly over [0, box]^2 (each point picks its
    centre uniformly) with isotropic Gaussian spread ``sigma``.  The draw
    order is already random, so no separate shuffle is needed."""
    n = int(n)
    centres = rng.uniform(0.0, box, size=(n_centres, 2))
    is_noise = rng.random(n) < noise_frac
    n_noise = int(is_noise.sum())
    out = np.empty((n, 2), dtype=np.float64)
    idx = rng.integers(0, n_centres, size=n - n_noise)
    out[~is_noise] = centres[idx] + rng.normal(0.0, sigma, size=(n - n_noise, 2))
    out[is_noise] = rng.uniform(0.0, box, size=(n_noise, 2))
    return np.ascontiguousarray(out.astype(dtype, copy=False))


def blobs3d(seed: int, n: int, n_centres: int, box: float, sigma: float, noise_frac: float,
            dtype=np.float64) -> np.ndarray:
    """Three-dimensional version of ``blobs`` for Section 3.6's
    generalisation: n points of shape (n, 3) over [0, box]^3, a share
    ``noise_frac`` uniform, the rest Gaussian (``sigma``) around centres drawn
    uniformly.  There is no 3-D workload in the paper; this one keeps the 2-D
    workloads' structure (dense blobs in sparse noise)."""
    rng = rng_for(seed)
    n = int(n)
    centres = rng.uniform(0.0, box, size=(n_centres, 3))
    is_noise = rng.random(n) < noise_frac
    n_noise = int(is_noise.sum())
    out = np.empty((n, 3), dtype=np.float64)
    idx = rng.integers(0, n_centres, size=n - n_noise)
    out[~is_noise] = centres[idx] + rng.normal(0.0, sigma, size=(n - n_noise, 3))
    out[is_noise] = rng.uniform(0.0, box, size=(n_noise, 3))
    return np.ascontiguousarray(out.astype(dtype, copy=False))


# --------------------------------------------------------------------------
# Workload 1: 200k points, 100 centres in [0,100]^2, 1,900 points per centre
# with sigma 0.05, 10k uniform noise points; precision 1, tau 5, mu 4.
# --------------------------------------------------------------------------
PLAIN_SMALL = dict(name="plain-200k", n=200_000, precision=1, tau=5, mu=4, seed=1)


def plain_small(seed: int = 1) -> np.ndarray:
    rng = rng_for(seed)
    centres = rng.uniform(0.0, 100.0, size=(100, 2))
    clustered = np.repeat(centres, 1900, axis=0) + rng.normal(0.0, 0.05, size=(190_000, 2))
    noise = rng.uniform(0.0, 100.0, size=(10_000, 2))
    return np.ascontiguousarray(_shuffle_rows(rng, np.concatenate([clustered, noise])))


# --------------------------------------------------------------------------
# Workload 2: 50M points, 10k centres in [0,1000]^2, Zipf(1.1) mass over the
# centres (ranks randomly permuted), sigma 0.02, 5% uniform noise;
# precision 2, tau 5, mu 4.  Hot tiles stress contended counting.
# --------------------------------------------------------------------------
ZIPF_HOT = dict(name="zipf-50M", n=50_000_000, precision=2, tau=5, mu=4, seed=2)


def zipf_hot(seed: int = 2, n: int = 50_000_000, block: int = 5_000_000) -> np.ndarray:
    """Generated in fixed blocks from spawned child seeds so peak host memory
    stays near one block of temporaries; the result depends only on
    (seed, n, block)."""
    ss = np.random.SeedSequence(seed)
    head, body = ss.spawn(2)
    rng = rng_for(head)
    n_centres = 10_000
    centres = rng.uniform(0.0, 1000.0, size=(n_centres, 2))
    weight = np.arange(1, n_centres + 1, dtype=np.float64) ** -1.1
    weight = weight[rng.permutation(n_centres)]
    cdf = np.cumsum(weight)
    cdf /= cdf[-1]
    out = np.empty((n, 2), dtype=np.float64)
    n_blocks = (n + block - 1) // block
    for b, child in enumerate(body.spawn(n_blocks)):
        r = rng_for(child)
        lo, hi = b * block, min(n, (b + 1) * block)
        k = hi - lo
        is_noise = r.random(k) < 0.05
        n_noise = int(is_noise.sum())
        u = r.random(k - n_noise)
        idx = np.minimum(np.searchsorted(cdf, u, side="right"), n_centres - 1)
        seg = np.empty((k, 2), dtype=np.float64)
        seg[~is_noise] = centres[idx] + r.normal(0.0, 0.02, size=(k - n_noise, 2))
        seg[is_noise] = r.uniform(0.0, 1000.0, size=(n_noise, 2))
        out[lo:hi] = seg
    return out


# --------------------------------------------------------------------------
# Workload 3 (paper scale, Tables 3 and 4: 10^6 clusters of about 500 points):
# 500M points, 1M centres in [0,10000]^2, each point picks a centre uniformly,
# sigma 0.01, no noise; precision 2, tau 5, mu 4; ten chunks of 50M points.
# --------------------------------------------------------------------------
PAPER_SCALE = dict(name="paper-500M-stream", n=500_000_000, chunks=10,
                   chunk=50_000_000, precision=2, tau=5, mu=4, seed=3)


def _paper_scale_seeds(seed: int, n_chunks: int):
    head, *chunks = np.random.SeedSequence(seed).spawn(n_chunks + 1)
    return head, chunks


def paper_scale_centres(seed: int = 3, n_centres: int = 1_000_000) -> np.ndarray:
    head, _ = _paper_scale_seeds(seed, 10)
    return rng_for(head).uniform(0.0, 10_000.0, size=(n_centres, 2))


def paper_scale_chunk(c: int, seed: int = 3, chunk: int = 50_000_000,
                      n_chunks: int = 10, centres: np.ndarray | None = None,
                      out: np.ndarray | None = None) -> np.ndarray:
    """Chunk ``c`` of the stream.  Pass ``centres`` to skip redrawing them.
    ``chunk`` may be made smaller for a scaled-down copy of the stream."""
    if centres is None:
        centres = paper_scale_centres(seed)
    _, chunk_seeds = _paper_scale_seeds(seed, n_chunks)
    r = rng_for(chunk_seeds[c])
    idx = r.integers(0, centres.shape[0], size=chunk)
    if out is None:
        out = np.empty((chunk, 2), dtype=np.float64)
    np.add(centres[idx], r.normal(0.0, 0.01, size=(chunk, 2)), out=out)
    return out


# --------------------------------------------------------------------------
# Workloads 4 and 5: many independent jobs, each shaped like workload 1
# (100 centres in [0,100]^2, sigma 0.05, 5% uniform noise) at its own size.
# --------------------------------------------------------------------------
@dataclass(frozen=True)
class JobSpec:
    seed: int
    n: int
    precision: int
    tau: int
    mu: int
    dtype: str = "f64"
    arrival_s: float = 0.0


def job_points(spec: JobSpec) -> np.ndarray:
    dt = np.float32 if spec.dtype == "f32" else np.float64
    return blobs(rng_for(spec.seed), spec.n, 100, 100.0, 0.05, 0.05, dtype=dt)


def _draw_params(rng: np.random.Generator, k: int):
    p = rng.choice(np.array([1, 2, 3]), size=k)
    t = rng.choice(np.array([3, 5, 10]), size=k)
    m = rng.choice(np.array([2, 4, 8]), size=k)
    return p, t, m


def batch_jobs(seed: int = 4, n_jobs: int = 256, lo: float = 1e4, hi: float = 5e6,
               size_scale: float = 1.0) -> list[JobSpec]:
    """256 jobs with sizes log-uniform in [lo, hi]; ``size_scale`` shrinks
    every size for quick tests while keeping the parameter draws."""
    rng = rng_for(seed)
    sizes = np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=n_jobs)))
    p, t, m = _draw_params(rng, n_jobs)
    return [JobSpec(seed=seed * 1000 + i, n=max(1, int(sizes[i] * size_scale)),
                    precision=int(p[i]), tau=int(t[i]), mu=int(m[i]))
            for i in range(n_jobs)]


def served_trace(seed: int = 5, rate: float = 200.0, duration_s: float = 30.0,
                 lo: float = 1e3, hi: float = 2e7, size_scale: float = 1.0) -> list[JobSpec]:
    """Poisson arrivals at ``rate`` jobs/s over ``duration_s`` seconds; sizes
    log-uniform in [lo, hi]; FP32 or FP64 coordinates with probability 1/2."""
    rng = rng_for(seed)
    t, arrivals = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration_s:
            break
        arrivals.append(t)
    k = len(arrivals)
    sizes = np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=k)))
    p, tau, mu = _draw_params(rng, k)
    dts = rng.random(k) < 0.5
    return [JobSpec(seed=seed * 1_000_000 + j, n=max(1, int(sizes[j] * size_scale)),
                    precision=int(p[j]), tau=int(tau[j]), mu=int(mu[j]),
                    dtype="f32" if dts[j] else "f64", arrival_s=float(arrivals[j]))
            for j in range(k)]


def served_parity_slice(seed: int = 5, head_s: float = 0.5) -> list[JobSpec]:
    """Jobs of the served workload (200 jobs/s for 30 s) used for full-size
    parity: every job arriving in the first ``head_s`` seconds, plus the
    largest job of the whole trace, each at its full size and dtype."""
    trace = served_trace(seed=seed, rate=200.0, duration_s=30.0)
    head = [s for s in trace if s.arrival_s < head_s]
    big = max(trace, key=lambda s: s.n)
    return head + ([big] if big not in head else [])

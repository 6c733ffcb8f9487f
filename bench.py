#!/usr/bin/env python3
"""RASTER benchmark on one MI355X.

One step = the whole hot path over one batch of synthetic input: begin a
stream, feed the paper-scale workload (500M FP64 points, 1M centres in
[0, 10000]^2, sigma 0.01, precision 2, tau 5, mu 4) as ten resident 50M-point
chunks, finish (significance scan, union-find agglomeration, mu filter).

Prints one JSON line with points/s, the counting kernel's roofline (HIP-event
duration per launch against the 8 TB/s HBM peak, algorithmic bytes = 16 bytes
of FP64 coordinates per point), the whole step's algorithmic bandwidth
against the same peak, the step's kernels from the committed rocprofv3
summary, and the CPU oracle timed on the whole workload on this host (one
core), with whether its rows equal the GPU step's.  After the timed steps it also times the
per-point label pass over all 500M resident points (Section 4.1), the 256-job
batch against plain calls, and the server on a Poisson trace.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "points/s + HBM GB/s at 500M pts; batched/served vs plain, p50/p99 latency"
HBM_PEAK_GBPS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "count_kernel_traffic.txt")
KERNEL_SRC = os.path.join(ROOT, "paper_1907_03620_amd", "csrc", "raster_kernels.hip")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """Hash of the kernel source's code: comments and blank lines are dropped,
    so that editing a comment does not void the recorded counters."""
    import re
    with open(KERNEL_SRC) as f:
        src = f.read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    src = re.sub(r"//[^\n]*", "", src)
    code = "\n".join(l.rstrip() for l in src.splitlines() if l.strip())
    return hashlib.sha256(code.encode()).hexdigest()[:16]


def measured_traffic(per_launch_points: int, key: str = "hbm_bytes_per_launch"):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source with launches of
    the same size; else None.  ``key`` picks the kernel: the counting kernel
    (hbm_bytes_per_launch) or the per-point label kernel
    (labels_hbm_bytes_per_launch)."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    if int(kv.get("points_per_launch", -1)) != per_launch_points or key not in kv:
        return None
    return float(kv[key])


STEP_KERNELS_FILE = os.path.join(ROOT, "profiles", "paper500M_step_kernels.txt")

# Algorithmic bytes of each kernel of the step, per unit of the workload (n
# points, m distinct tiles, s significant tiles, t output rows): what the
# method itself must move, without probe amplification or binning scratch.
# Their sum is the step's 16 n + 24 m + 20 s + 20 t.
KERNEL_ALG_BYTES = {
    "k_bin_points": ("16 B per point (FP64 coordinates, read once)", lambda n, m, s, t: 16.0 * n),
    "k_bin_keys": ("0 (binning scratch only)", lambda n, m, s, t: 0.0),
    "k_aggregate": ("12 B per distinct tile (key and count written once)", lambda n, m, s, t: 12.0 * m),
    "k_threshold": ("12 B per distinct tile (key and count read once)", lambda n, m, s, t: 12.0 * m),
    "k_link_part": ("8 B per significant tile (its key)", lambda n, m, s, t: 8.0 * s),
    "union-find": ("12 B per significant tile (parent traffic)", lambda n, m, s, t: 12.0 * s),
    "k_filter": ("20 B per output row", lambda n, m, s, t: 20.0 * t),
}


def kernel_group(name: str):
    """The algorithmic-bytes group of a kernel name from the profile."""
    for g in ("k_bin_points", "k_bin_keys", "k_aggregate", "k_threshold", "k_link_part", "k_filter"):
        if name.startswith(g):
            return g
    if name.startswith("k_census_framed"):  # the significance scan of framed tables
        return "k_threshold"
    if name.startswith("k_link_census"):
        return "k_link_part"
    if name.startswith(("k_jump", "k_merge", "k_compress")):
        return "union-find"
    return None


def step_kernels(n: int, m: int, s: int, t: int):
    """Per-kernel figures of one step from the committed rocprofv3 summary
    (average launch time, launches per step, HBM traffic and L2 atomic
    requests per launch), with each kernel's algorithmic bytes for this run's
    n, m, s and t.  None unless the summary was taken on the current kernel
    source."""
    if not os.path.exists(STEP_KERNELS_FILE):
        return None
    kv, rows = {}, []
    for line in open(STEP_KERNELS_FILE):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line.startswith("kernel="):
            rows.append(dict(f.split("=", 1) for f in line.split(";")))
        elif "=" in line:
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    out = []
    for r in rows:
        g = kernel_group(r["kernel"])
        calls = float(r["calls_per_step"])
        alg = KERNEL_ALG_BYTES[g][1](n, m, s, t) if g else None
        out.append({"kernel": r["kernel"], "launches_per_step": calls, "avg_launch_us": float(r["avg_us"]),
                    "ms_per_step": calls * float(r["avg_us"]) / 1000.0,
                    "algorithmic_bytes_per_step": alg,
                    "algorithmic_bytes": KERNEL_ALG_BYTES[g][0] if g else None,
                    "hbm_bytes_per_step": calls * (float(r["fetch_bytes"]) + float(r["write_bytes"])),
                    "l2_atomic_requests_per_step": calls * float(r["tcc_atomic"]),
                    "memory_atomic_requests_per_step": calls * float(r["ea_atomic"])})
    return out


def gen_paper_scale(n_chunks: int, chunk: int):
    import synth
    centres = synth.paper_scale_centres(3)
    with ThreadPoolExecutor(min(16, n_chunks)) as ex:
        return list(ex.map(lambda c: synth.paper_scale_chunk(c, centres=centres, chunk=chunk,
                                                             n_chunks=n_chunks), range(n_chunks)))


def strip_sample(host_chunks, strip: float):
    """The points of every chunk whose x lies in [0, strip): a strip of the
    canvas with the full workload's density."""
    import numpy as np
    return np.concatenate([h[h[:, 0] < strip] for h in host_chunks])


def cpu_baseline(sample, strip: float, precision: int, tau: int, mu: int):
    """Times the oracle, single-threaded and pinned to one core, on the strip
    sample."""
    import oracle
    try:
        cpu = sorted(os.sched_getaffinity(0))[0]
        os.sched_setaffinity(0, {cpu})
    except (AttributeError, OSError):
        pass
    t0 = time.perf_counter()
    res = oracle.cluster(sample, tau=tau, mu=mu, precision=precision)
    dt = time.perf_counter() - t0
    try:
        os.sched_setaffinity(0, set(range(os.cpu_count() or 1)))
    except (AttributeError, OSError):
        pass
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), None)
    except OSError:
        pass
    return dict(value=sample.shape[0] / dt, unit="points/s", cores=1, kind="oracle", cpu=model,
                host_cpus=os.cpu_count(),
                sample=(f"x in [0, {strip:g}) strip of all chunks: {sample.shape[0]} points "
                        f"({res.stats['clusters']} clusters), full Algorithm 1, {dt:.1f} s"),
                seconds=dt, points=int(sample.shape[0]), clusters=int(res.stats["clusters"]))


def cpu_baseline_full(host_chunks, gpu_rows, precision: int, tau: int, mu: int):
    """Times the oracle, single-threaded and pinned to one core, on the whole
    workload (every chunk of the stream, fed as chunks), and checks that its
    rows equal those of the last timed GPU step."""
    import numpy as np
    import oracle
    try:
        cpu = sorted(os.sched_getaffinity(0))[0]
        os.sched_setaffinity(0, {cpu})
    except (AttributeError, OSError):
        pass
    t0 = time.perf_counter()
    res = oracle.cluster_chunks(host_chunks, tau=tau, mu=mu, precision=precision)
    dt = time.perf_counter() - t0
    try:
        os.sched_setaffinity(0, set(range(os.cpu_count() or 1)))
    except (AttributeError, OSError):
        pass
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), None)
    except OSError:
        pass
    kx, ky, cnt, lab = gpu_rows
    lab = lab.astype(np.uint64)
    lx = (lab >> np.uint64(32)).astype(np.int64) - (1 << 31)
    ly = (lab & np.uint64(0xFFFFFFFF)).astype(np.int64) - (1 << 31)
    same = (kx.shape[0] == res.kx.shape[0] and np.array_equal(kx.astype(np.int64), res.kx)
            and np.array_equal(ky.astype(np.int64), res.ky) and np.array_equal(cnt.astype(np.uint64), res.count)
            and np.array_equal(lx, res.label_x) and np.array_equal(ly, res.label_y))
    n = sum(int(h.shape[0]) for h in host_chunks)
    return dict(value=n / dt, unit="points/s", cores=1, kind="oracle", cpu=model, host_cpus=os.cpu_count(),
                sample=(f"the whole workload: all {len(host_chunks)} chunks ({n} points) fed to the oracle as one "
                        f"stream, full Algorithm 1, {dt:.1f} s"),
                seconds=dt, points=n, clusters=int(res.stats["clusters"]), tiles=int(res.stats["tiles"]),
                same_rows_as_gpu_step=bool(same))


def cpu_p_raster(sample, precision: int, tau: int, mu: int):
    """Times the multi-core P-RASTER baseline (Section 3.5) on the same strip
    sample, on up to 16 host threads, after one untimed run."""
    import cpu_baseline as cb
    threads = cb.default_threads()
    scale = float(10 ** precision)
    cb.cluster(sample[: min(len(sample), 1_000_000)], tau=tau, mu=mu, scale=scale, threads=threads)
    t0 = time.perf_counter()
    res = cb.cluster(sample, tau=tau, mu=mu, scale=scale, threads=threads)
    dt = time.perf_counter() - t0
    t1 = time.perf_counter()
    one = cb.cluster(sample, tau=tau, mu=mu, scale=scale, threads=1)
    dt1 = time.perf_counter() - t1
    return dict(value=sample.shape[0] / dt, unit="points/s", cores=threads, kind="P-RASTER (Algorithms 2 and 3)",
                seconds=dt, phases_s=res.stats["seconds"], clusters=res.stats["clusters"],
                one_thread_seconds=dt1, speedup_over_one_thread=dt1 / dt,
                same_clusters_one_thread=bool(one.stats["clusters"] == res.stats["clusters"]
                                              and one.num_tiles == res.num_tiles),
                sample="the same strip as cpu_baseline")


def bench_point_labels(raster, torch, res, dev, reps: int = 3):
    """Per-point labels (Section 4.1) of every resident point from one step's
    result: one call per chunk on the current stream, each bracketed by HIP
    events on that stream.  The first call builds the result's lookup table
    and is not timed.  Algorithmic bytes per point: 16 of FP64 coordinates
    read, one 16-byte table slot read, 8 bytes of label written."""
    import numpy as np
    s = torch.cuda.current_stream()
    res.point_labels(dev[0], stream=s)
    torch.cuda.synchronize()
    per_call, passes, noise = [], [], 0
    for r in range(reps):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * len(dev))]
        for k, d in enumerate(dev):
            ev[2 * k].record(s)
            lab = res.point_labels(d, stream=s)
            ev[2 * k + 1].record(s)
            if r == 0:
                noise += int((lab == -1).sum().item())
        torch.cuda.synchronize()
        calls = [ev[2 * k].elapsed_time(ev[2 * k + 1]) for k in range(len(dev))]
        per_call += calls
        passes.append(sum(calls))
    n = sum(int(d.shape[0]) for d in dev)
    ms = float(np.median(passes))
    avg_call_us = 1000.0 * float(np.mean(per_call))
    per_launch = n / len(dev)
    gbps = 40.0 * per_launch / (avg_call_us * 1e-6) / 1e9
    traffic = measured_traffic(int(per_launch), "labels_hbm_bytes_per_launch")
    # the lookup of each point's tile is one random table line: the kernel is
    # bound by that line traffic, reported beside the algorithmic rate
    traffic_gbps = traffic / (avg_call_us * 1e-6) / 1e9 if traffic else None
    return {"points": n, "ms_per_pass": ms, "points_per_s": n / (ms * 1e-3),
            "avg_launch_us": avg_call_us, "launches_per_pass": len(dev),
            "achieved": gbps, "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": gbps / HBM_PEAK_GBPS,
            "algorithmic_bytes": "40 B per point: 16 of coordinates in, one 16-byte slot, 8 of label out",
            "traffic": traffic, "traffic_bytes_per_point": traffic / per_launch if traffic else None,
            "traffic_gbps": traffic_gbps, "traffic_frac": traffic_gbps / HBM_PEAK_GBPS if traffic else None,
            "noise_points": noise}


def bench_tile_points(raster, torch, res, dev, reps: int = 3):
    """Per-tile point lists (RASTER', Section 3.4) of every resident point from
    one step's result: one call per chunk (lookup, count per row, scan,
    scatter; each call synchronises), timed with HIP events on the calling
    stream.  The first call builds the row table and is not timed."""
    import numpy as np
    s = torch.cuda.current_stream()
    res.tile_points(dev[0], stream=s)
    torch.cuda.synchronize()
    passes, kept = [], 0
    for r in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for d in dev:
            _, index = res.tile_points(d, stream=s)
            if r == 0:
                kept += int(index.shape[0])
        e1.record(s)
        torch.cuda.synchronize()
        passes.append(e0.elapsed_time(e1))
    n = sum(int(d.shape[0]) for d in dev)
    ms = float(np.median(passes))
    return {"points": n, "points_listed": kept, "ms_per_pass": ms, "points_per_s": n / (ms * 1e-3),
            "calls_per_pass": len(dev)}


def bench_neighbourhoods(raster, torch, dev, precision: int, tau: int, mu: int, steps: int = 3):
    """The same 500M-point stream with the variants of the method: other
    neighbourhoods of Section 3.2 (one pass of the link kernel per four
    backward offsets) and the 2x2 post-step of Section 3.6.  ms per step, the
    threshold and agglomeration phases, after one untimed step each."""
    import numpy as np
    out = []
    for metric, delta, square in (("manhattan", 1, False), ("chebyshev", 2, False), ("chebyshev", 3, False),
                                  ("chebyshev", 1, True)):
        def step():
            st = raster.Stream(tau=tau, mu=mu, precision=precision, metric=metric, delta=delta, square=square)
            for d in dev:
                st.feed(d)
            r = st.finish()
            st.close()
            return r
        step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rs = [step() for _ in range(steps)]
        torch.cuda.synchronize()
        ms = 1000.0 * (time.perf_counter() - t0) / steps
        out.append({"metric": metric, "delta": delta, "square_step": square, "ms_per_step": ms,
                    "us_threshold": float(np.mean([r.stats["us_threshold"] for r in rs])),
                    "us_agglomerate": float(np.mean([r.stats["us_agglomerate"] for r in rs])),
                    "clusters": int(rs[-1].stats["clusters"]), "tiles": int(rs[-1].stats["tiles"])})
    return out


def bench_3d(raster, torch, steps: int = 3, n_chunks: int = 10, chunk: int = 20_000_000):
    """Section 3.6's generalisation to three dimensions: a stream of
    n_chunks x chunk resident FP64 points; each chunk draws its own 100K
    blobs (sigma 0.01, one tile) in [0, 1000]^3 with 2% noise, so the stream
    holds 1M blobs of about 200 points; precision 2, tau 3, mu 4; ms per step
    after one untimed step."""
    import synth
    with ThreadPoolExecutor(min(16, n_chunks)) as ex:
        host = list(ex.map(lambda c: synth.blobs3d(9000 + c, n=chunk, n_centres=100_000, box=1000.0, sigma=0.01,
                                                   noise_frac=0.02), range(n_chunks)))
    dev = [torch.from_numpy(h).to("cuda") for h in host]
    del host
    torch.cuda.synchronize()

    def step():
        st = raster.Stream(tau=3, mu=4, precision=2, dims=3)
        for d in dev:
            st.feed(d)
        r = st.finish()
        st.close()
        return r

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rs = [step() for _ in range(steps)]
    torch.cuda.synchronize()
    ms = 1000.0 * (time.perf_counter() - t0) / steps
    st = rs[-1].stats
    n = n_chunks * chunk
    out = {"workload": f"3-D stream: {n} FP64 points in {n_chunks} resident chunks, 100K blobs per chunk "
                       "(1M in all, sigma 0.01) in [0,1000]^3, 2% noise, p=2, tau=3, mu=4",
           "ms_per_step": ms, "points_per_s": n / (ms * 1e-3), "distinct_tiles": st["distinct_tiles"],
           "significant_tiles": st["significant_tiles"], "clusters": st["clusters"],
           "us_count_kernel_per_launch": st["us_count_kernel"] / max(1, st["count_launches"]),
           "us_agglomerate": st["us_agglomerate"]}
    del dev, rs
    torch.cuda.empty_cache()
    return out


def bench_h2d_stream(raster, torch, host, precision: int, tau: int, mu: int, reps: int = 2):
    """Context only, never `value`: the same stream with the chunks in pinned
    host memory.  Each chunk is copied on a copy stream into one of two device
    buffers while the previous chunk is counted; the compute stream waits for
    the copy, and a copy waits until the chunk that used its buffer two steps
    earlier has been fed.  Bound by the host link."""
    import numpy as np
    pinned = [torch.from_numpy(h).pin_memory() for h in host]
    rows = max(p.shape[0] for p in pinned)
    bufs = [torch.empty((rows, 2), dtype=pinned[0].dtype, device="cuda") for _ in range(2)]
    comp = torch.cuda.current_stream()
    copy = torch.cuda.Stream()

    def run():
        free = [None, None]
        st = raster.Stream(tau=tau, mu=mu, precision=precision, stream=comp)
        for k, p in enumerate(pinned):
            b = k % 2
            buf = bufs[b][: p.shape[0]]
            with torch.cuda.stream(copy):
                if free[b] is not None:
                    copy.wait_event(free[b])
                buf.copy_(p, non_blocking=True)
                done = torch.cuda.Event()
                done.record(copy)
            comp.wait_event(done)
            st.feed(buf)
            free[b] = torch.cuda.Event()
            free[b].record(comp)
        res = st.finish()
        st.close()
        return res

    first = run()
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        t0 = time.perf_counter()
        res = run()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    n = sum(int(p.shape[0]) for p in pinned)
    nbytes = sum(p.numel() * p.element_size() for p in pinned)
    sec = float(np.median(times))
    same = all(res.stats[k] == first.stats[k] for k in ("tiles", "clusters", "distinct_tiles"))
    del pinned, bufs
    return {"ms_per_step": 1000.0 * sec, "points_per_s": n / sec, "host_to_device_gb_per_s": nbytes / sec / 1e9,
            "clusters": int(res.stats["clusters"]), "same_result_as_first_run": bool(same),
            "how": "chunks in pinned host memory, copied on a second stream into two device buffers, "
                   "overlapped with counting; median of %d runs after one warm-up" % reps}


def pct(values, q):
    import numpy as np
    return float(np.percentile(np.asarray(values), q)) if len(values) else None


def bench_batched(raster, torch, n_jobs: int, reps: int):
    """256 jobs (sizes log-uniform in [1e4, 5e6], parameters drawn per job),
    each generated from its own seed; plain per-job calls against one batch."""
    import synth
    from paper_1907_03620_amd import autotune
    specs = synth.batch_jobs(seed=4, n_jobs=n_jobs)
    log(f"batched: generating {len(specs)} jobs, {sum(s.n for s in specs)} points")
    with ThreadPoolExecutor(16) as ex:
        host = list(ex.map(synth.job_points, specs))
    dev = [torch.from_numpy(h).to("cuda") for h in host]
    del host
    args = [dict(points=d, precision=sp.precision, tau=sp.tau, mu=sp.mu) for sp, d in zip(specs, dev)]
    total = sum(sp.n for sp in specs)
    saved = raster.get_tuning()
    best = autotune.tune("batch", lambda: raster.cluster_batch(args), points=total, reps=2, log=log)

    # each form with its own settings: plain calls with the library defaults
    # (their counting path is chosen per call), the batch autotuned
    def plain():
        return [raster.cluster(**a) for a in args]

    def batched():
        return raster.cluster_batch(args)

    out = {}
    for name, fn, tuning in (("plain_per_job", plain, saved), ("batched", batched, best)):
        raster.set_tuning(tuning)
        fn()
        best_t = float("inf")
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = fn()
            torch.cuda.synchronize()
            best_t = min(best_t, time.perf_counter() - t0)
            del res
        out[name] = {"seconds": best_t, "points_per_s": total / best_t}
    raster.set_tuning(saved)
    del dev, args
    torch.cuda.empty_cache()
    return {"workload": f"{len(specs)} jobs, n log-uniform in [1e4, 5e6], {total} FP64 points, "
                        "p/tau/mu drawn per job, each job generated from its own seed",
            "jobs": len(specs), "points": total, "tuning": best.__dict__, "plain_tuning": saved.__dict__,
            "plain_per_job": out["plain_per_job"], "batched": out["batched"],
            "speedup": out["plain_per_job"]["seconds"] / out["batched"]["seconds"]}


def bench_served(raster, torch, duration_s: float, rate: float, slots: int, stress_rate: float = 0.0,
                 stress_s: float = 2.0):
    """Poisson arrivals replayed in real time: the continuous-batching server
    against a plain FIFO worker issuing one call per job; at the workload's
    rate and, if stress_rate > 0, at a rate that queues jobs."""
    import synth
    pool_n = 20_000_000
    log(f"served: pool of {pool_n} points")
    pool_h = synth.job_points(synth.JobSpec(seed=5, n=pool_n, precision=1, tau=5, mu=4))
    pool64 = torch.from_numpy(pool_h).to("cuda")
    pool32 = pool64.to(torch.float32)
    del pool_h
    out = served_run(raster, torch, pool64, pool32, duration_s, rate, slots)
    if stress_rate > 0:
        out["stress"] = served_run(raster, torch, pool64, pool32, stress_s, stress_rate, slots)
    del pool64, pool32
    torch.cuda.empty_cache()
    return out


def served_run(raster, torch, pool64, pool32, duration_s: float, rate: float, slots: int):
    import threading
    import numpy as np
    import synth
    trace = synth.served_trace(seed=5, rate=rate, duration_s=duration_s)
    pool_n = pool64.shape[0]
    log(f"served: {len(trace)} jobs over {duration_s:g} s at {rate:g} jobs/s")

    def points(j, sp):
        off = (j * 7919) % max(1, pool_n - sp.n + 1)
        src = pool32 if sp.dtype == "f32" else pool64
        return src[off:off + sp.n]

    views = [points(j, sp) for j, sp in enumerate(trace)]
    total = sum(sp.n for sp in trace)
    torch.cuda.synchronize()

    def run_server():
        srv = raster.Server(budget_bytes=64 << 30, max_slots=slots)
        lat, tickets = [], []
        done_at = [0.0]
        lock = threading.Lock()

        def waiter():
            i = 0
            while True:
                with lock:
                    if i >= len(trace):
                        return
                    ready = i < len(tickets)
                    t = tickets[i] if ready else None
                if not ready:
                    time.sleep(0.0005)
                    continue
                r, l = srv.wait(t)
                lat.append(l)
                r.free()
                done_at[0] = time.perf_counter()
                i += 1

        th = threading.Thread(target=waiter)
        th.start()
        t0 = time.perf_counter()
        for j, sp in enumerate(trace):
            d = t0 + sp.arrival_s - time.perf_counter()
            if d > 0:
                time.sleep(d)
            tk = srv.submit(views[j], tau=sp.tau, mu=sp.mu, precision=sp.precision)
            with lock:
                tickets.append(tk)
        th.join()
        srv.close()
        return lat, done_at[0] - t0

    service = []  # plain per-job call times, without waiting

    def run_fifo():
        import queue
        q = queue.Queue()
        lat = []
        done_at = [0.0]

        def worker():
            while True:
                item = q.get()
                if item is None:
                    return
                j, arrived = item
                sp = trace[j]
                start = time.perf_counter()
                r = raster.cluster(views[j], precision=sp.precision, tau=sp.tau, mu=sp.mu)
                r.free()
                now = time.perf_counter()
                lat.append(now - arrived)
                service.append(now - start)
                done_at[0] = now

        th = threading.Thread(target=worker)
        th.start()
        t0 = time.perf_counter()
        for j, sp in enumerate(trace):
            d = t0 + sp.arrival_s - time.perf_counter()
            if d > 0:
                time.sleep(d)
            q.put((j, time.perf_counter()))
        q.put(None)
        th.join()
        return lat, done_at[0] - t0

    out = {}
    big = np.array([sp.n >= 2_000_000 for sp in trace])
    for name, fn in (("server", run_server), ("plain_fifo", run_fifo)):
        lat, span = fn()
        out[name] = {"p50_ms": 1e3 * pct(lat, 50), "p99_ms": 1e3 * pct(lat, 99), "mean_ms": 1e3 * float(np.mean(lat)),
                     "points_per_s": total / span, "makespan_s": span}
        # both record latencies in arrival order: split by job size
        lat_a = np.asarray(lat)
        out[name]["p99_ms_jobs_below_2M"] = 1e3 * pct(lat_a[~big], 99)
        out[name]["p99_ms_jobs_2M_up"] = 1e3 * pct(lat_a[big], 99)
    svc = np.asarray(service)
    service_stats = {"p50_ms": 1e3 * pct(svc, 50), "p99_ms": 1e3 * pct(svc, 99),
                     "p99_ms_jobs_below_2M": 1e3 * pct(svc[~big], 99), "p99_ms_jobs_2M_up": 1e3 * pct(svc[big], 99),
                     "busy_fraction": float(svc.sum()) / duration_s}
    del views
    return {"workload": f"Poisson {rate:g} jobs/s for {duration_s:g} s ({len(trace)} jobs), n log-uniform in "
                        "[1e3, 2e7] (windows of one 20M-point set shaped like workload 1), FP32/FP64 per job, "
                        "p/tau/mu drawn per job, budget 64 GiB",
            "jobs": len(trace), "points": total, "offered_points_per_s": total / duration_s, "slots": slots,
            "server": out["server"], "plain_fifo": out["plain_fifo"],
            "plain_call_time": service_stats}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--chunks", type=int, default=10)
    ap.add_argument("--chunk", type=int, default=50_000_000)
    ap.add_argument("--tile-hint", type=int, default=0,
                    help="expected distinct tiles passed to raster_begin (0: let the table grow)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-strip", type=float, default=2000.0)
    ap.add_argument("--tuning", default="", help="JSON object of raster_tuning fields")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched (256-job) comparison")
    ap.add_argument("--no-neighbourhoods", action="store_true",
                    help="skip the steps with Manhattan 1 and Chebyshev 2 and 3 neighbourhoods and the 2x2 step")
    ap.add_argument("--no-3d", action="store_true", help="skip the three-dimensional stream")
    ap.add_argument("--no-h2d", action="store_true", help="skip the host-to-device streaming run")
    ap.add_argument("--no-point-labels", action="store_true",
                    help="skip the per-point label pass and the per-tile point lists")
    ap.add_argument("--no-served", action="store_true", help="skip the served (Poisson trace) comparison")
    ap.add_argument("--served-seconds", type=float, default=30.0)
    ap.add_argument("--served-rate", type=float, default=200.0)
    ap.add_argument("--served-slots", type=int, default=4)
    ap.add_argument("--served-stress-rate", type=float, default=2000.0,
                    help="second served run at this rate (jobs/s, 4 s), where jobs queue; 0 skips it")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (3 times), to scale HBM counters")
    args = ap.parse_args()

    if args.copy_calibration:
        import torch
        nbytes = 1 << 30
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "copies": 3}), flush=True)
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "the library has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_1907_03620_amd as raster

    raster.load()
    if args.tuning:
        raster.set_tuning(**json.loads(args.tuning))
    precision, tau, mu = 2, 5, 4
    n_total = args.chunks * args.chunk

    log(f"generating {args.chunks} x {args.chunk} points")
    host = gen_paper_scale(args.chunks, args.chunk)
    dev = [torch.from_numpy(h).to("cuda") for h in host]
    torch.cuda.synchronize()

    def step():
        st = raster.Stream(tau=tau, mu=mu, precision=precision, tile_hint=args.tile_hint)
        for d in dev:
            st.feed(d)
        res = st.finish()
        st.close()
        return res

    log(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    log(f"timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1000.0 * elapsed / args.steps
    value = n_total * args.steps / elapsed

    st = results[-1].stats
    binned = st["flushes"] > 0
    launches = sum(r.stats["count_launches"] for r in results)
    us_kernel = sum(r.stats["us_count_kernel"] for r in results)
    avg_us = us_kernel / max(1, launches)
    points_per_launch = n_total * args.steps / max(1, launches)
    bytes_per_launch = 16.0 * points_per_launch
    achieved = bytes_per_launch / (avg_us * 1e-6) / 1e9
    traffic = measured_traffic(int(points_per_launch))
    m, s, t = st["distinct_tiles"], st["significant_tiles"], st["tiles"]
    alg_bytes = 16.0 * n_total + 2 * 12.0 * m + 20.0 * s + 20.0 * t
    step_gbps = alg_bytes / (ms_per_step * 1e-3) / 1e9
    phases = {k: round(float(np.mean([r.stats[k] for r in results])), 1)
              for k in ("us_contract", "us_threshold", "us_agglomerate", "us_filter",
                        "us_count_kernel", "us_bin_keys", "us_aggregate")}

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": (f"paper-scale stream: {n_total} FP64 points, 1M centres in [0,10000]^2, "
                         f"sigma 0.01, p=2, tau=5, mu=4, {args.chunks} resident chunks of {args.chunk} "
                         "through begin/feed_chunk/finish"),
            "points": n_total, "chunks": args.chunks, "precision": precision, "tau": tau, "mu": mu,
            "tile_hint": args.tile_hint, "tuning": raster.get_tuning().__dict__,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": ("k_bin_points_f (projection + level-1 binning of 4-byte entries)" if st["key_frame"]
                       else "k_bin_points (projection + level-1 binning)") if binned
                      else "k_count_direct (projection + device-table count)",
            "achieved": achieved,
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBPS,
            "traffic": traffic,
            "avg_launch_us": avg_us,
            "bytes_per_launch": bytes_per_launch,
            "algorithmic_bytes": "16 B of FP64 coordinates per point, read once",
            "step_achieved": step_gbps,
            "step_frac": step_gbps / HBM_PEAK_GBPS,
            "step_algorithmic_bytes": alg_bytes,
            "step_algorithmic_bytes_formula": "16 n + 24 m + 20 s + 20 t (n points, m distinct tiles, "
                                              "s significant tiles, t output rows)",
        },
        "kernels": step_kernels(n_total, m, s, t),
        "hbm_gbps_algorithmic_step": step_gbps,
        "phases_us": phases,
        "result": {"distinct_tiles": m, "significant_tiles": s, "clusters": st["clusters"], "tiles": t,
                   "table_capacity": st["table_capacity"], "grow_events": st["grow_events"]},
        "cpu_baseline": None,
    }
    gpu_rows = results[-1].numpy(sort=True) if not args.no_cpu_baseline else None
    line["point_labels"] = None if args.no_point_labels else bench_point_labels(raster, torch, results[-1], dev)
    line["tile_points"] = None if args.no_point_labels else bench_tile_points(raster, torch, results[-1], dev)
    line["neighbourhoods"] = None
    if not args.no_neighbourhoods:
        log("other neighbourhoods")
        line["neighbourhoods"] = bench_neighbourhoods(raster, torch, dev, precision, tau, mu)
        line["neighbourhoods"].insert(0, {"metric": "chebyshev", "delta": 1, "square_step": False,
                                          "ms_per_step": ms_per_step, "us_threshold": phases["us_threshold"],
                                          "us_agglomerate": phases["us_agglomerate"], "clusters": st["clusters"],
                                          "tiles": st["tiles"]})
    del dev, results
    torch.cuda.empty_cache()
    line["three_d"] = None
    if not args.no_3d:
        log("three-dimensional stream")
        line["three_d"] = bench_3d(raster, torch)
    line["h2d_stream"] = None
    if not args.no_h2d:
        log("host-to-device stream (pinned chunks, two buffers)")
        line["h2d_stream"] = bench_h2d_stream(raster, torch, host, precision, tau, mu)
        line["h2d_stream"]["resident_clusters"] = st["clusters"]
        torch.cuda.empty_cache()
    line["batched"] = None if args.no_batched else bench_batched(raster, torch, 256, 3)
    line["served"] = None if args.no_served else bench_served(raster, torch, args.served_seconds, args.served_rate,
                                                              args.served_slots, args.served_stress_rate)
    line["cpu_p_raster"] = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle, one core, the whole stream)")
        line["cpu_baseline"] = cpu_baseline_full(host, gpu_rows, precision, tau, mu)
        del gpu_rows
        sample = strip_sample(host, args.cpu_strip)
        log("cpu P-RASTER (host threads) and the oracle on a strip")
        strip = cpu_baseline(sample, args.cpu_strip, precision, tau, mu)
        line["cpu_p_raster"] = cpu_p_raster(sample, precision, tau, mu)
        line["cpu_p_raster"]["oracle_on_the_strip"] = strip
        line["cpu_p_raster"]["same_clusters_as_oracle"] = line["cpu_p_raster"]["clusters"] == strip["clusters"]
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

#!/usr/bin/env python3
"""Writes tests/golden/full_size_digests.json: the oracle's results on the
full-size workloads, as canonical digests (tests/digest.py) with their
statistics, so that the GPU tests can compare every row of a full-size run
without running the single-threaded oracle for minutes each time.

Calls only the seeded generators (synth) and the CPU oracle (oracle); the
HIP library is not loaded.  Workloads:

* paper-500M: 500M FP64 points in ten 50M chunks (1M centres in
  [0, 10000]^2, sigma 0.01), precision 2, tau 5, mu 4, fed chunk by chunk
  (Section 3.6);
* batch-256: the 256 jobs of the batched workload, each clustered alone;
* served-slice: the served workload's jobs of the first half second plus its
  largest job, each clustered alone.

Usage: python tests/golden/make_full_size_digests.py [paper] [batch] [served]
(no argument: all three; existing entries of the others are kept).
"""
from __future__ import annotations

import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import oracle  # noqa: E402
import synth  # noqa: E402
from digest import STAT_KEYS, points_digest, rows_digest  # noqa: E402

OUT = os.path.join(HERE, "full_size_digests.json")


def summary(res) -> dict:
    d = {k: int(res.stats[k]) for k in STAT_KEYS}
    d["rows"] = rows_digest(res.kx, res.ky, res.count, res.label_x, res.label_y)
    return d


def paper():
    cfg = synth.PAPER_SCALE
    centres = synth.paper_scale_centres(cfg["seed"])
    st = oracle.OracleStream(oracle.scale_for_precision(cfg["precision"]), cfg["tau"], cfg["mu"])
    inputs = []
    t0 = time.time()
    for c in range(cfg["chunks"]):
        h = synth.paper_scale_chunk(c, seed=cfg["seed"], chunk=cfg["chunk"], n_chunks=cfg["chunks"],
                                    centres=centres)
        inputs.append(points_digest(h))
        st.feed(h)
        print(f"paper-500M: chunk {c} fed ({time.time() - t0:.0f} s)", flush=True)
        del h
    res = st.finish()
    st.close()
    print(f"paper-500M: oracle done ({time.time() - t0:.0f} s)", flush=True)
    return {"workload": "paper-500M stream, 10 x 50M FP64, p=2 tau=5 mu=4", "inputs": inputs, **summary(res)}


def _jobs(specs, name):
    out = []
    t0 = time.time()
    with ThreadPoolExecutor(8) as ex:
        for i, (sp, pts) in enumerate(zip(specs, ex.map(synth.job_points, specs))):
            res = oracle.cluster(pts, tau=sp.tau, mu=sp.mu, precision=sp.precision)
            out.append({"seed": sp.seed, "n": sp.n, "dtype": sp.dtype, "precision": sp.precision, "tau": sp.tau,
                        "mu": sp.mu, "input": points_digest(pts), **summary(res)})
            if i % 32 == 0:
                print(f"{name}: job {i}/{len(specs)} ({time.time() - t0:.0f} s)", flush=True)
    return out


def batch():
    return {"workload": "batch-256 (seed 4), each job alone", "jobs": _jobs(synth.batch_jobs(4), "batch-256")}


def served():
    return {"workload": "served slice (seed 5: arrivals before 0.5 s and the largest job), each job alone",
            "jobs": _jobs(synth.served_parity_slice(5), "served-slice")}


def main():
    want = set(sys.argv[1:]) or {"paper", "batch", "served"}
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name, fn in (("paper", paper), ("batch", batch), ("served", served)):
        if name in want:
            data[name] = fn()
            with open(OUT, "w") as f:
                json.dump(data, f, indent=1, sort_keys=True)
                f.write("\n")
    print("wrote", OUT)


if __name__ == "__main__":
    main()

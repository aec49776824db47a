#!/usr/bin/env python3
"""Throughput of the MI355X lattice Boltzmann hot path.

Workload (default): D3Q19 BGK lid-driven cavity, 256^3 cells, FP32 storage
(deviation form) and arithmetic, tau = 0.55, halfway bounce-back on five static
walls and a lid (+z face) moving at u = (0.05, 0, 0), start at rest, in-place
(AA) streaming -- the 3-D cavity the paper benchmarks in Sec. 5.  One "step"
is one lattice Boltzmann time step over the whole grid (stream + collide +
boundary fill, one kernel launch); MLUPS = cells * steps / time / 1e6.

Printed: one JSON line with the metric, a roofline object for the step kernel
(algorithmic bytes 2*Q*sizeof per cell update / measured kernel time), the
HBM counter traffic from the committed rocprofv3 summary when it matches the
current kernel source, and the FP64 CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBPS = 8000.0
COUNTERS = os.path.join(ROOT, "profiles", "hbm_counters_d3q19_f32_256.json")
KERNEL_SOURCES = ["core.hpp", "kernels_impl.hpp", "lattice.hpp"]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2311_16080_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counter_traffic(bytes_alg_per_launch: float):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source."""
    try:
        with open(COUNTERS) as fh:
            c = json.load(fh)
    except (OSError, ValueError):
        return None
    if c.get("kernel_source_hash") != kernel_source_hash():
        return None
    return c.get("hbm_bytes_per_launch")


def cavity_faces(lbm, U=0.05):
    return [(lbm.WALL,)] * 5 + [(lbm.WALL, (U, 0.0, 0.0))]


def cpu_baseline(n: int, tau: float, target_s: float = 15.0):
    """FP64 oracle on the same cavity, timed on the host for a bounded number
    of steps (about target_s seconds of work)."""
    import oracle
    faces = [oracle.Face(oracle.WALL) for _ in range(6)]
    faces[5] = oracle.Face(oracle.WALL, (0.05, 0.0, 0.0))
    S = oracle.Sim(q=19, nx=n, ny=n, nz=n, tau=tau, faces=faces)
    f = S.equilibrium_state()
    t0 = time.perf_counter()
    S.run(f, 1)
    dt1 = time.perf_counter() - t0
    k = max(1, min(50, int(target_s / max(dt1, 1e-3))))
    t0 = time.perf_counter()
    S.run(f, k)
    dt = time.perf_counter() - t0
    mlups = n ** 3 * k / dt / 1e6
    return {"value": round(mlups, 3), "unit": "MLUPS", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"D3Q19 FP64 cavity {n}^3, {k} steps after 1 warm-up step ({dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--storage", default="f32", choices=["f32", "f16", "bf16", "f64"])
    ap.add_argument("--lattice", default="D3Q19", choices=["D2Q9", "D3Q19", "D3Q27"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extras", action="store_true", help="skip the copy probe and extra figures")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch
    from paper_2311_16080_amd import lbm

    n = args.n
    tau = 0.55
    lat = args.lattice
    Q = lbm.Q_OF[lbm.LATTICES[lat]]
    shape = (n, n) if lat == "D2Q9" else (n, n, n)
    faces = cavity_faces(lbm) if lat != "D2Q9" else [(lbm.WALL,), (lbm.WALL,), (lbm.WALL,),
                                                      (lbm.WALL, (0.05, 0.0)), (lbm.PERIODIC,), (lbm.PERIODIC,)]
    N = int(np.prod(shape))
    sim = lbm.Sim(lat, shape, tau, faces=faces, storage=args.storage, pattern="inplace")
    sim.use_current_stream()
    sim.init_equilibrium()
    stream = torch.cuda.current_stream()

    sim.step(args.warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    sim.step(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    ms_per_step = ms / args.steps
    mlups = N * args.steps / (ms / 1e3) / 1e6

    esize = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2}[args.storage]
    bytes_per_launch = 2.0 * Q * esize * N
    achieved = bytes_per_launch / (ms_per_step / 1e3) / 1e9
    traffic = counter_traffic(bytes_per_launch) if (lat == "D3Q19" and n == 256 and args.storage == "f32") else None

    out = {
        "metric": f"MLUPS, {lat} {args.storage} {n}^{len(shape)} lid-driven cavity (and % of HBM roofline)",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.storage,
        "data": "synthetic",
        "config": {"workload": f"{lat} BGK lid-driven cavity {'x'.join(map(str, shape))}, tau={tau}, "
                               f"halfway bounce-back walls, lid u=(0.05,0,0), rest start, in-place AA streaming",
                   "cells": N, "pattern": "inplace"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBPS, 4), "traffic": traffic,
                     "bytes_per_lattice_update": 2 * Q * esize},
    }

    if not args.no_extras:
        # achievable HBM copy bandwidth (bandwidth probe), same stream
        nb = 2 * 1024 ** 3
        src = torch.empty(nb // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            lbm.copy_probe(dst, src, nb)
        torch.cuda.synchronize()
        e0.record(stream)
        reps = 20
        for _ in range(reps):
            lbm.copy_probe(dst, src, nb)
        e1.record(stream)
        torch.cuda.synchronize()
        copy_gbps = 2.0 * nb * reps / (e0.elapsed_time(e1) / 1e3) / 1e9
        out["copy_probe_GBps"] = round(copy_gbps, 1)
        out["frac_of_copy"] = round(achieved / copy_gbps, 4)
        del src, dst
        torch.cuda.empty_cache()

    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(n if lat == "D3Q19" else 128, tau)

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

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
import platform
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


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(n: int, tau: float, target_s: float = 10.0, n_one: int = 128):
    """FP64 oracle on the same cavity, timed on the host for a bounded number
    of steps (about target_s seconds of work): once with every OpenMP thread
    the process may use (`value`, `cores`), once on one thread (a 128^3 cavity,
    whose state is still far beyond the caches)."""
    import oracle
    faces = [oracle.Face(oracle.WALL) for _ in range(6)]
    faces[5] = oracle.Face(oracle.WALL, (0.05, 0.0, 0.0))

    def timed(m, threads):
        oracle.set_num_threads(threads)
        S = oracle.Sim(q=19, nx=m, ny=m, nz=m, tau=tau, faces=faces)
        f = S.equilibrium_state()
        t0 = time.perf_counter()
        S.run(f, 1)
        dt1 = time.perf_counter() - t0
        k = max(1, min(50, int(target_s / max(dt1, 1e-3))))
        t0 = time.perf_counter()
        S.run(f, k)
        dt = time.perf_counter() - t0
        return m ** 3 * k / dt / 1e6, k, dt, oracle.num_threads()

    threads = oracle.num_threads()
    v_all, k_all, dt_all, used = timed(n, threads)
    v_one, k_one, dt_one, _ = timed(n_one, 1)
    oracle.set_num_threads(threads)
    try:
        affinity = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        affinity = None
    return {"value": round(v_all, 3), "unit": "MLUPS", "cores": used, "kind": "oracle",
            "sample": f"D3Q19 FP64 cavity {n}^3, {k_all} steps after 1 warm-up step ({dt_all:.1f} s) on "
                      f"{used} OpenMP threads; one-thread figure: {n_one}^3, {k_one} steps ({dt_one:.1f} s)",
            "one_core_MLUPS": round(v_one, 3), "nproc": os.cpu_count(), "affinity_cpus": affinity,
            "cpu_model": _cpu_model()}


GOLDEN = os.path.join(ROOT, "tests", "golden")


def _golden(name):
    """Stored oracle results (written by tests/golden/make_golden.py), or None."""
    path = os.path.join(GOLDEN, name)
    return np.load(path) if os.path.exists(path) else None


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def cavity_error_vs_oracle(torch, lbm, storage, n=256, steps=1000, pattern="inplace"):
    """u after 1000 steps of the cavity from rest against the stored FP64
    oracle run: rel-L2 over the whole planes y = n/2 and x = n/2 and over a
    uniform random sample of cells (the whole-field estimate)."""
    ref = _golden("cavity256_d3q19_1000.npz")
    if ref is None or n != 256:
        return None
    sim = lbm.Sim("D3Q19", (n, n, n), 0.55, faces=cavity_faces(lbm), storage=storage, pattern=pattern)
    sim.use_current_stream()
    sim.init_equilibrium()
    sim.step(steps)
    _, u = sim.moments(dtype=torch.float64)
    st = int(ref["stride"])
    out = {"steps": steps}
    py = torch.stack([u[a, ::st, n // 2, ::st] for a in range(3)], -1).cpu().numpy()
    out["u_rel_l2_y128"] = _rel(py, ref["u_y128"])
    if "u_x128" in ref.files:
        px = torch.stack([u[a, n // 2, :, :] for a in range(3)], -1).cpu().numpy()
        out["u_rel_l2_x128"] = _rel(px, ref["u_x128"])
    if "u_sample" in ref.files:
        idx = torch.tensor(ref["sample_cells"], device=u.device)
        us = u.reshape(3, -1)[:, idx].T.cpu().numpy()
        out["u_rel_l2_cell_sample"] = _rel(us, ref["u_sample"])
    del sim
    return out


class Timer:
    """HIP events on the torch current stream (the stream the library launches on)."""

    def __init__(self, torch):
        self.torch = torch
        self.s = torch.cuda.current_stream()
        self.e0 = torch.cuda.Event(enable_timing=True)
        self.e1 = torch.cuda.Event(enable_timing=True)

    def __enter__(self):
        self.torch.cuda.synchronize()
        self.e0.record(self.s)
        return self

    def __exit__(self, *exc):
        self.e1.record(self.s)
        self.torch.cuda.synchronize()
        self.ms = self.e0.elapsed_time(self.e1)


def storage_variants(torch, lbm, n, tau, steps=200):
    """The same cavity with FP16 / BF16 deviation storage (FP32 arithmetic),
    timed over a fixed 200 steps after 20 warm-up steps, in place and with the
    pull pattern.  Both keep the box's X-halves in split pairs (two cells per
    32-bit word); the figure is the pull pattern (two buffers, 1.3 GB), whose
    stores are all aligned, with the in-place figure (one buffer) beside it."""
    out = {}
    for st, es in (("f16", 2), ("bf16", 2)):
        rate = {}
        for pattern in ("inplace", "pull"):
            sim = lbm.Sim("D3Q19", (n, n, n), tau, faces=cavity_faces(lbm), storage=st, pattern=pattern)
            sim.use_current_stream()
            sim.init_equilibrium()
            sim.step(20)
            with Timer(torch) as T:
                sim.step(steps)
            rate[pattern] = n ** 3 * steps / (T.ms / 1e3) / 1e6
            del sim
            torch.cuda.empty_cache()
        mlups = rate["pull"]
        gbps = mlups * 1e6 * 2 * 19 * es / 1e9
        out[st] = {"pattern": "pull", "MLUPS": round(mlups, 1), "GBps": round(gbps, 1),
                   "frac": round(gbps / PEAK_HBM_GBPS, 4), "bytes_per_lattice_update": 2 * 19 * es, "steps": steps,
                   "inplace": {"MLUPS": round(rate["inplace"], 1),
                               "frac": round(rate["inplace"] * 1e6 * 2 * 19 * es / 1e9 / PEAK_HBM_GBPS, 4)}}
        out[st]["error_vs_oracle"] = cavity_error_vs_oracle(torch, lbm, st, n, pattern="pull")
    return out


def _ke_seed(torch, rho, u, n_cells):
    return 0.5 * (u * u).sum(0) / n_cells, rho * u / n_cells


def adjoint_ratio(torch, lbm, name, make_sim, nsteps, K, loss):
    """(time of lbm_backward over nsteps, checkpoint restores and recompute
    included) / (time of lbm_step(nsteps) without a tape).  One untimed
    forward + backward first, so that neither side is charged with the
    one-time loading of its kernels (the paper likewise drops the first,
    compiling iteration, Sec. 5)."""
    sim = make_sim()
    sim.use_current_stream()
    want_s = getattr(sim, "_has_s", False)
    sim.init_equilibrium()
    sim.tape_begin(K, nsteps)
    sim.step(nsteps)
    sim.tape_end()
    rho, u = sim.moments(dtype=torch.float32)
    sim.backward(*loss(rho, u), want_s=want_s)
    sim.init_equilibrium()
    sim.step(2)
    with Timer(torch) as F:
        sim.step(nsteps)
    sim.init_equilibrium()
    sim.tape_begin(K, nsteps)
    with Timer(torch) as R:
        sim.step(nsteps)
    sim.tape_end()
    rho, u = sim.moments(dtype=torch.float32)
    g_rho, g_u = loss(rho, u)
    with Timer(torch) as B:
        ds, dtau, _ = sim.backward(g_rho, g_u, want_s=want_s)
    sim.tape_free()
    del sim
    out = {"workload": name, "steps": nsteps, "K": K, "forward_ms": round(F.ms, 3),
           "forward_taped_ms": round(R.ms, 3), "backward_ms": round(B.ms, 3),
           "ratio": round(B.ms / F.ms, 3), "dL_dtau": float(dtau[0])}
    if ds is not None:
        out["dL_ds"] = ds.double().cpu().numpy()
    return out


def c4_faces(lbm):
    return [(lbm.ZOUHE_VELOCITY, (0.04, 0.0)), (lbm.EQ_OUTFLOW, (0.0, 0.0), 1.0), (lbm.WALL,), (lbm.WALL,),
            (lbm.PERIODIC,), (lbm.PERIODIC,)]


def c4_target(torch, lbm):
    """u_T = u(500) of the channel with the solid fraction from seed 40 (FP64 run on the GPU)."""
    from paper_2311_16080_amd import inputs
    sim = lbm.Sim("D2Q9", (512, 256), 0.6, faces=c4_faces(lbm), storage="f64")
    sim.use_current_stream()
    sim.set_solid_fraction(inputs.smooth_solid_fraction(512, 256, seed=40))
    sim.init_equilibrium()
    sim.step(500)
    _, u = sim.moments(dtype=torch.float32)
    del sim
    return u


def adjoint_figures(torch, lbm):
    from paper_2311_16080_amd import inputs
    res = []

    def c4():
        sim = lbm.Sim("D2Q9", (512, 256), 0.6, faces=c4_faces(lbm), storage="f32")
        sim.set_solid_fraction(inputs.smooth_solid_fraction(512, 256, seed=4))
        sim._has_s = True
        return sim

    tgt = c4_target(torch, lbm)

    def l2(rho, u):
        return None, 2.0 * (u - tgt)

    r = adjoint_ratio(torch, lbm, "D2Q9 FP32 512x256 channel, partial bounce-back s field, u-mismatch loss "
                                  "against the seed-40 run (C4)", c4, 500, 50, l2)
    ref = _golden("c4_adjoint_d2q9_512x256.npz")
    if ref is not None and "dL_ds" in r:
        r["error_vs_oracle"] = {"dL_ds_rel_l2": _rel(r.pop("dL_ds"), ref["dlds"].astype(np.float64)),
                                "dL_dtau_rel": abs(r["dL_dtau"] - float(ref["dtau"])) / abs(float(ref["dtau"]))}
    r.pop("dL_ds", None)
    res.append(r)

    def cav3():
        return lbm.Sim("D3Q19", (256, 256, 256), 0.55, faces=cavity_faces(lbm), storage="f32")

    res.append(adjoint_ratio(torch, lbm, "D3Q19 FP32 256^3 cavity, mean kinetic energy loss", cav3, 100, 10,
                             lambda r, u: _ke_seed(torch, r, u, 256.0 ** 3)))

    def cav2():
        return lbm.Sim("D2Q9", (8192, 8192), 0.6, faces=[(lbm.WALL,), (lbm.WALL,), (lbm.WALL,),
                                                         (lbm.WALL, (0.05, 0.0)), (lbm.PERIODIC,), (lbm.PERIODIC,)],
                       storage="f32")

    res.append(adjoint_ratio(torch, lbm, "D2Q9 FP32 8192^2 cavity, mean kinetic energy loss", cav2, 50, 10,
                             lambda r, u: _ke_seed(torch, r, u, 8192.0 ** 2)))

    def kbc3():
        sim = lbm.Sim("D3Q27", (256, 256, 256), 0.5005, faces=cavity_faces(lbm), storage="f32")
        sim.set_collision("KBC")
        return sim

    res.append(adjoint_ratio(torch, lbm, "D3Q27 FP32 256^3 KBC cavity at tau = 0.5005, mean kinetic energy loss",
                             kbc3, 40, 10, lambda r, u: _ke_seed(torch, r, u, 256.0 ** 3)))
    return res


def batch_figures(torch, lbm, steps=2000):
    """256 D2Q9 cavities (side lengths 64..256, tau in [0.52, 1), lid 0.05..0.1)
    advanced by one captured graph; against one launch per domain and the
    plain single-domain FP32 rate; then forward + adjoint of the summed
    per-domain mean kinetic energy."""
    from paper_2311_16080_amd import inputs
    L, tau, U = inputs.batch_cavities(256, seed=5)
    shapes = [(int(l), int(l)) for l in L]
    faces = [[(lbm.WALL,), (lbm.WALL,), (lbm.WALL,), (lbm.WALL, (float(U[d]), 0.0)), (lbm.PERIODIC,),
              (lbm.PERIODIC,)] for d in range(256)]
    out = {"domains": 256, "cells": int(sum(l * l for l in L)), "steps": steps}
    bs = lbm.BatchSim("D2Q9", shapes, tau, faces, storage="f32")
    bs.use_current_stream()
    bs.init_equilibrium()
    bs.step(2)                       # runs the autotuner on a copy of the state
    bs.capture_graph(steps)
    bs.graph_launch()                # warm-up replay
    with Timer(torch) as G:
        bs.graph_launch()
    N = out["cells"]
    tile, pers = bs.config()
    out["graph_MLUPS"] = round(N * steps / (G.ms / 1e3) / 1e6, 1)
    out["graph_ms"] = round(G.ms, 2)
    out["tile"] = tile
    out["persistent"] = pers
    out["effective_GBps"] = round(out["graph_MLUPS"] * 1e6 * 72 / 1e9, 1)
    # both launch modes at the chosen tile, each captured as one graph of all steps
    modes = {}
    for mode in (1, 0):
        bs.tuning(tile, mode)
        bs.init_equilibrium()
        bs.capture_graph(steps)
        bs.graph_launch()
        with Timer(torch) as M:
            bs.graph_launch()
        modes["persistent_one_launch" if mode else "one_launch_per_step"] = {
            "MLUPS": round(N * steps / (M.ms / 1e3) / 1e6, 1), "graph_ms": round(M.ms, 2)}
    out["launch_modes"] = modes
    bs.tuning(tile, pers)
    bs.init_equilibrium()
    bs.capture_graph(steps)
    bs.graph_launch()
    # unstable domains: non-finite or |u| above 0.3 anywhere
    rho, u = bs.moments(dtype=torch.float32)
    speed = torch.sqrt((u * u).sum(0))
    bad = []
    for d in range(256):
        a, b = int(bs.offsets[d]), int(bs.offsets[d + 1])
        m = float(speed[a:b].max())
        if not np.isfinite(m) or m > 0.3:
            bad.append(d)
    out["unstable_domains"] = bad
    # one launch per domain (separate contexts), fewer steps
    sims = []
    for d in range(256):
        s = lbm.Sim("D2Q9", shapes[d], float(tau[d]), faces=faces[d], storage="f32")
        s.use_current_stream()
        s.init_equilibrium()
        sims.append(s)
    k = 50
    for s in sims:
        s.step(2)
    with Timer(torch) as P:
        for s in sims:
            s.step(k)
    out["per_domain_launch_MLUPS"] = round(N * k / (P.ms / 1e3) / 1e6, 1)
    del sims
    big = lbm.Sim("D2Q9", (4096, 4096), 0.6, faces=faces[0], storage="f32")
    big.use_current_stream()
    big.init_equilibrium()
    big.step(10)
    with Timer(torch) as S:
        big.step(100)
    out["single_domain_4096sq_MLUPS"] = round(4096 ** 2 * 100 / (S.ms / 1e3) / 1e6, 1)
    del big
    # forward + adjoint of sum_d mean KE_d over the same steps (after one
    # untimed forward + backward, which loads the adjoint kernels)
    K = 50
    ncell = None
    for timed in (False, True):
        bs.init_equilibrium()
        bs.tape_begin(K, steps)
        with Timer(torch) as R:
            bs.step(steps)
        bs.tape_end()
        rho, u = bs.moments(dtype=torch.float32)
        if ncell is None:
            ncell = torch.empty_like(rho)
            for d in range(256):
                ncell[int(bs.offsets[d]):int(bs.offsets[d + 1])] = float(L[d]) ** 2
        g_rho, g_u = _ke_seed(torch, rho, u, ncell)
        with Timer(torch) as B:
            dtau, duw = bs.backward(g_rho, g_u)
    out["adjoint"] = {"K": K, "forward_taped_ms": round(R.ms, 2), "backward_ms": round(B.ms, 2),
                      "ratio_vs_graph_forward": round(B.ms / G.ms, 3),
                      "dE_dtau_first4": [float(v) for v in dtau[:4]],
                      "dE_dU_first4": [float(duw[d, 3, 0]) for d in range(4)]}
    ref = _golden("c5_gradients_d2q9.npz")
    if ref is not None and int(ref["steps"]) == steps:
        pick = [int(d) for d in ref["domains"]]
        e_tau = max(abs(float(dtau[d]) - float(ref["dtau"][k])) / abs(float(ref["dtau"][k]))
                    for k, d in enumerate(pick))
        e_u = max(abs(float(duw[d, 3, 0]) - float(ref["dU"][k])) / abs(float(ref["dU"][k]))
                  for k, d in enumerate(pick))
        out["adjoint"]["error_vs_oracle"] = {"domains": pick, "dE_dtau_max_rel": e_tau, "dE_dU_max_rel": e_u}
    return out


def channel_spheres_figures(torch, lbm, steps=50):
    """D3Q27 1024x512x512 FP32 channel with random spheres (5% solid), Zou-He
    inlet u = 0.04, equilibrium outflow, bounce-back walls.  The figure is the
    pull pattern (two buffers, 58 GB: at this size its aligned cell-local
    stores beat the in-place pattern, whose neighbour step stores Z-shifted
    addresses); the in-place figure (one buffer, 29 GB) is reported beside it."""
    from paper_2311_16080_amd import inputs
    shape = (1024, 512, 512)
    t0 = time.perf_counter()
    solid = inputs.sphere_obstacles(*shape, seed=3)
    gen_s = time.perf_counter() - t0
    faces = [(lbm.ZOUHE_VELOCITY, (0.04, 0.0, 0.0)), (lbm.EQ_OUTFLOW, (0.0, 0.0, 0.0), 1.0), (lbm.WALL,),
             (lbm.WALL,), (lbm.WALL,), (lbm.WALL,)]
    N = int(np.prod(shape))
    rate = {}
    for pattern in ("inplace", "pull"):
        sim = lbm.Sim("D3Q27", shape, 0.6, faces=faces, storage="f32", pattern=pattern)
        sim.use_current_stream()
        sim.set_solid(solid)
        sim.init_equilibrium()
        sim.step(10)
        with Timer(torch) as T:
            sim.step(steps)
        rate[pattern] = N * steps / (T.ms / 1e3) / 1e6
        if pattern == "pull":
            # momentum-exchange force of the last step (drag / lift on the spheres, force on the walls)
            with Timer(torch) as FT:
                Fs, Ff = sim.forces()
        del sim
        torch.cuda.empty_cache()
    mlups = rate["pull"]
    gbps = mlups * 1e6 * 216 / 1e9
    res = {"cells": N, "solid_fraction": round(float(solid.mean()), 4), "steps": steps, "pattern": "pull",
           "MLUPS": round(mlups, 1), "GBps_at_216B": round(gbps, 1), "frac": round(gbps / PEAK_HBM_GBPS, 4),
           "inplace": {"MLUPS": round(rate["inplace"], 1),
                       "frac": round(rate["inplace"] * 1e6 * 216 / 1e9 / PEAK_HBM_GBPS, 4)},
           "sphere_generation_s": round(gen_s, 1), "forces_ms": round(FT.ms, 3),
           "sphere_force": [float(v) for v in Fs]}
    # the same generator at 256 x 128 x 128 (radii 2..8), 300 steps, against the stored oracle plane z = 64
    ref = _golden("channel_spheres_d3q27_300.npz")
    if ref is not None:
        rs = (256, 128, 128)
        sol = inputs.sphere_obstacles(*rs, seed=3, rmin=2.0, rmax=8.0, xlo=16, xhi=240, fraction=0.05)
        sim = lbm.Sim("D3Q27", rs, 0.6, faces=faces, storage="f32", pattern="pull")
        sim.use_current_stream()
        sim.set_solid(sol)
        sim.init_equilibrium()
        sim.step(int(ref["steps"]))
        _, u = sim.moments(dtype=torch.float64)
        st = int(ref["stride"])
        pl = torch.stack([u[a, ::st, ::st, rs[2] // 2] for a in range(3)], -1).cpu().numpy()
        m = ~ref["solid_z64"].astype(bool)
        res["error_vs_oracle"] = {"shape": list(rs), "steps": int(ref["steps"]),
                                  "u_rel_l2_z64": _rel(pl[m], ref["u_z64"][m])}
        del sim
    return res


def forced_channel_figures(torch, lbm, steps=100, adj_steps=40, K=10):
    """Force-driven channel (the paper's turbulent-channel setup, Sec. 4.4):
    D3Q19 FP32, walls 2h apart in y, periodic streamwise (6h) and spanwise (3h),
    h = 128 (768 x 256 x 384 cells), driven by F_x = Re_tau^2 nu^2 / h^3 at
    Re_tau = 180 through the exact-difference method; once as a uniform force,
    once as a per-cell field (3 more FP32 reads per cell), plus the adjoint /
    forward time ratio with the field gradient requested; the forced runs also
    with the pull pattern."""
    from paper_2311_16080_amd import inputs
    h = 128
    shape = (6 * h, 2 * h, 3 * h)
    N = int(np.prod(shape))
    nu = 0.01 * h / 180.0            # u_tau = Re_tau nu / h = 0.01
    tau = 0.5 + 3.0 * nu
    Fx = 180.0 ** 2 * nu ** 2 / h ** 3
    faces = [(lbm.PERIODIC,), (lbm.PERIODIC,), (lbm.WALL,), (lbm.WALL,), (lbm.PERIODIC,), (lbm.PERIODIC,)]
    res = {"shape": list(shape), "tau": round(tau, 6), "Fx": Fx}
    field = torch.tensor(np.moveaxis(inputs.random_velocity(shape, 3, 90, amp=0.1 * Fx), -1, 0).copy(),
                         dtype=torch.float32, device="cuda")
    for kind, bpc in (("none", 152), ("uniform", 152), ("field", 164)):
        sim = lbm.Sim("D3Q19", shape, tau, faces=faces, storage="f32")
        sim.use_current_stream()
        sim.init_equilibrium()
        if kind == "uniform":
            sim.set_force([Fx, 0.0, 0.0])
        elif kind == "field":
            sim.set_force([Fx, 0.0, 0.0], field)
        sim.step(10)
        with Timer(torch) as T:
            sim.step(steps)
        mlups = N * steps / (T.ms / 1e3) / 1e6
        gbps = mlups * 1e6 * bpc / 1e9
        res[kind] = {"MLUPS": round(mlups, 1), "GBps": round(gbps, 1), "frac": round(gbps / PEAK_HBM_GBPS, 4),
                     "bytes_per_lattice_update": bpc}
        if kind == "field":
            # adjoint / forward ratio with dL/dfield requested (mean kinetic energy loss)
            sim.init_equilibrium()
            sim.step(2)
            with Timer(torch) as F:
                sim.step(adj_steps)
            for timed in (False, True):       # the first pass loads the adjoint kernels
                sim.init_equilibrium()
                sim.tape_begin(K, adj_steps)
                sim.step(adj_steps)
                sim.tape_end()
                rho, u = sim.moments(dtype=torch.float32)
                g_rho, g_u = _ke_seed(torch, rho, u, float(N))
                with Timer(torch) as B:
                    _, _, _, dfield, dforce = sim.backward_force(g_rho, g_u)
            res["adjoint_with_force"] = {"steps": adj_steps, "K": K, "forward_ms": round(F.ms, 3),
                                         "backward_ms": round(B.ms, 3), "ratio": round(B.ms / F.ms, 3),
                                         "dL_dforce": [float(v) for v in dforce]}
            del dfield
            sim.tape_free()
        del sim
        torch.cuda.empty_cache()
    # the pull pattern (two buffers, 5.7 GB): cell-local aligned stores
    res["pull"] = {}
    for kind, bpc in (("uniform", 152), ("field", 164)):
        sim = lbm.Sim("D3Q19", shape, tau, faces=faces, storage="f32", pattern="pull")
        sim.use_current_stream()
        sim.init_equilibrium()
        sim.set_force([Fx, 0.0, 0.0], field if kind == "field" else None)
        sim.step(10)
        with Timer(torch) as T:
            sim.step(steps)
        mlups = N * steps / (T.ms / 1e3) / 1e6
        gbps = mlups * 1e6 * bpc / 1e9
        res["pull"][kind] = {"MLUPS": round(mlups, 1), "GBps": round(gbps, 1), "frac": round(gbps / PEAK_HBM_GBPS, 4)}
        del sim
        torch.cuda.empty_cache()
    return res


def regularized_channel_figures(torch, lbm, steps=100):
    """D3Q19 FP32 512 x 256 x 256 channel, velocity inlet u = 0.04 on -x and
    pressure outlet rho = 1 on +x, walls on y and z: the same run with
    Zou-He faces and with regularized faces (the closure runs on the two
    open face planes only)."""
    shape = (512, 256, 256)
    N = int(np.prod(shape))
    res = {"shape": list(shape)}
    for name, vel, pres in (("zouhe", lbm.ZOUHE_VELOCITY, lbm.ZOUHE_PRESSURE),
                            ("regularized", lbm.REG_VELOCITY, lbm.REG_PRESSURE)):
        faces = [(vel, (0.04, 0.0, 0.0)), (pres, (0.0, 0.0, 0.0), 1.0), (lbm.WALL,), (lbm.WALL,), (lbm.WALL,),
                 (lbm.WALL,)]
        sim = lbm.Sim("D3Q19", shape, 0.6, faces=faces, storage="f32")
        sim.use_current_stream()
        sim.init_equilibrium()
        sim.step(10)
        with Timer(torch) as T:
            sim.step(steps)
        mlups = N * steps / (T.ms / 1e3) / 1e6
        gbps = mlups * 1e6 * 152 / 1e9
        res[name] = {"MLUPS": round(mlups, 1), "GBps": round(gbps, 1), "frac": round(gbps / PEAK_HBM_GBPS, 4)}
        del sim
    return res


def kbc_figures(torch, lbm, steps=60):
    """KBC vs BGK step rate: D3Q27 FP32 256^3 and D2Q9 FP32 4096^2 lid-driven
    cavities at tau = 0.5005 (KBC's use: nearly inviscid flow), in place (the
    top-level figures) and with the pull pattern."""
    res = {}
    for lat, shape, bpc in (("D3Q27", (256, 256, 256), 216), ("D2Q9", (4096, 4096), 72)):
        faces = cavity_faces(lbm) if lat == "D3Q27" else [(lbm.WALL,), (lbm.WALL,), (lbm.WALL,),
                                                           (lbm.WALL, (0.05, 0.0)), (lbm.PERIODIC,), (lbm.PERIODIC,)]
        N = int(np.prod(shape))
        for model in ("BGK", "KBC"):
            fig = {}
            for pattern in ("inplace", "pull"):
                sim = lbm.Sim(lat, shape, 0.5005, faces=faces, storage="f32", pattern=pattern)
                sim.use_current_stream()
                sim.set_collision(model)
                sim.init_equilibrium()
                sim.step(4)
                with Timer(torch) as T:
                    sim.step(steps)
                mlups = N * steps / (T.ms / 1e3) / 1e6
                gbps = mlups * 1e6 * bpc / 1e9
                fig[pattern] = {"MLUPS": round(mlups, 1), "GBps": round(gbps, 1),
                                "frac": round(gbps / PEAK_HBM_GBPS, 4)}
                del sim
                torch.cuda.empty_cache()
            res[f"{lat}_{model}"] = dict(fig["inplace"], pull=fig["pull"])
    return res


def pattern_size_figures(torch, lbm, steps=10):
    """In-place vs pull pattern on D3Q19 FP32 walls-only cavities from 4M to
    268M cells: the in-place neighbour step stores Z-shifted addresses, whose
    cost shows once the state outgrows the 256 MB Infinity Cache; the pull
    pattern stores only aligned cell-local slots."""
    res = {}
    for shape in ((64, 256, 256), (256, 256, 256), (1024, 256, 256), (4096, 256, 256), (1024, 512, 512)):
        N = int(np.prod(shape))
        row = {"GB_state": round(N * 76 / 1e9, 2)}
        for pattern in ("inplace", "pull"):
            sim = lbm.Sim("D3Q19", shape, 0.6, faces=cavity_faces(lbm), storage="f32", pattern=pattern)
            sim.use_current_stream()
            sim.init_equilibrium()
            sim.step(4)
            with Timer(torch) as T:
                sim.step(steps)
            mlups = N * steps / (T.ms / 1e3) / 1e6
            row[pattern] = {"MLUPS": round(mlups, 1), "frac": round(mlups * 152 / 1e3 / PEAK_HBM_GBPS, 4)}
            del sim
            torch.cuda.empty_cache()
        res["x".join(str(v) for v in shape)] = row
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--storage", default="f32", choices=["f32", "f16", "bf16", "f64"])
    ap.add_argument("--lattice", default="D3Q19", choices=["D2Q9", "D3Q19", "D3Q27"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-copy", action="store_true", help="skip the HBM copy probe")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the FP16/BF16, adjoint, batched and D3Q27 channel figures")
    ap.add_argument("--extra", default=None,
                    choices=["storage_f16_bf16", "adjoint_forward_ratio", "batched_cavities", "d3q27_channel_spheres",
                             "d3q19_forced_channel", "d3q19_regularized_channel", "kbc_cavities",
                             "pattern_sizes"],
                    help="run only this secondary figure and print it as one JSON line (for profiling)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch
    from paper_2311_16080_amd import lbm

    if args.extra:
        fns = {"storage_f16_bf16": lambda: storage_variants(torch, lbm, args.n, 0.55),
               "adjoint_forward_ratio": lambda: adjoint_figures(torch, lbm),
               "batched_cavities": lambda: batch_figures(torch, lbm),
               "d3q27_channel_spheres": lambda: channel_spheres_figures(torch, lbm),
               "d3q19_forced_channel": lambda: forced_channel_figures(torch, lbm),
               "d3q19_regularized_channel": lambda: regularized_channel_figures(torch, lbm),
               "kbc_cavities": lambda: kbc_figures(torch, lbm),
               "pattern_sizes": lambda: pattern_size_figures(torch, lbm)}
        print(json.dumps({"extra": args.extra, "result": fns[args.extra]()}), flush=True)
        return

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

    if lat == "D3Q19" and n == 256:
        out["error_vs_oracle"] = cavity_error_vs_oracle(torch, lbm, args.storage, n)

    if not args.no_copy:
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

    if not args.no_extras:
        del sim
        extras = {}
        for key, fn in (("storage_f16_bf16", lambda: storage_variants(torch, lbm, n, tau)),
                        ("adjoint_forward_ratio", lambda: adjoint_figures(torch, lbm)),
                        ("batched_cavities", lambda: batch_figures(torch, lbm)),
                        ("d3q27_channel_spheres", lambda: channel_spheres_figures(torch, lbm)),
                        ("d3q19_forced_channel", lambda: forced_channel_figures(torch, lbm)),
                        ("d3q19_regularized_channel", lambda: regularized_channel_figures(torch, lbm)),
                        ("kbc_cavities", lambda: kbc_figures(torch, lbm)),
                        ("pattern_sizes", lambda: pattern_size_figures(torch, lbm))):
            t0 = time.perf_counter()
            try:
                extras[key] = fn()
            except Exception as exc:  # reported, never hides the headline figure
                extras[key] = {"error": f"{type(exc).__name__}: {exc}"}
            print(f"[bench] {key} done in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
        out["extras"] = extras

    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(n if lat == "D3Q19" else 128, tau)

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

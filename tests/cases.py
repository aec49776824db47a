"""Shared helpers for GPU-vs-oracle parity tests: one case description builds
both the oracle problem and the GPU context from the same seeded inputs."""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

import oracle
from paper_2311_16080_amd import inputs, lbm

LAT = {9: "D2Q9", 19: "D3Q19", 27: "D3Q27"}


@dataclass
class Case:
    q: int
    shape: tuple                       # (nx, ny) or (nx, ny, nz)
    tau: float
    faces: list = field(default_factory=lambda: [(0,)] * 6)   # (type, u, rho) per face, caller axes
    steps: int = 10
    storage: str = "f64"
    pattern: str = "inplace"
    solid: Optional[np.ndarray] = None
    s: Optional[np.ndarray] = None
    init_seed: Optional[int] = None    # random (rho, u) init; None = rest
    init_u: Optional[np.ndarray] = None  # explicit velocity (*shape, D)
    amp: float = 0.03
    links: Optional[tuple] = None      # curved-wall links (cells, dirs, q), flat caller order
    bz_order: int = 1                  # interpolated bounce-back: 1 linear, 2 quadratic

    @property
    def D(self):
        return 2 if self.q == 9 else 3

    @property
    def oshape(self):
        return tuple(self.shape) + ((1,) if self.q == 9 else ())

    def init_fields(self):
        """(rho [shape] or None, u [*shape, D] or None) in FP64."""
        if self.init_u is not None:
            return None, np.asarray(self.init_u, dtype=np.float64)
        if self.init_seed is None:
            return None, None
        rho = inputs.random_density(self.shape, self.init_seed, amp=0.01)
        u = inputs.random_velocity(self.shape, self.D, self.init_seed + 1000, amp=self.amp)
        return rho, u


def _oface(F):
    t = int(F[0])
    u = tuple(F[1]) if len(F) > 1 else (0.0, 0.0, 0.0)
    u = tuple(u) + (0.0,) * (3 - len(u))
    rho = float(F[2]) if len(F) > 2 else 1.0
    return oracle.Face(t, u, rho)


def oracle_run(case: Case, steps: Optional[int] = None):
    """Oracle rho [oshape], u [oshape + (3,)] after `steps` steps."""
    faces = [_oface(F) for F in case.faces]
    if case.q == 9:
        faces[4] = faces[5] = oracle.Face()
    sol = None if case.solid is None else case.solid.reshape(case.oshape).astype(np.uint8)
    # the C-ABI takes the solid fraction as float32: both sides get the same rounded values
    sv = None if case.s is None else case.s.reshape(case.oshape).astype(np.float32).astype(np.float64)
    S = oracle.Sim(q=case.q, nx=case.oshape[0], ny=case.oshape[1], nz=case.oshape[2], tau=case.tau,
                   faces=faces, solid=sol, s=sv, bouzidi_order=case.bz_order)
    if case.links is not None:
        S.qlink = S.links_to_qlink(*case.links)
    rho, u = case.init_fields()
    if u is not None:
        u = u.reshape(case.oshape + (case.D,))
    if rho is not None:
        rho = rho.reshape(case.oshape)
    f = S.equilibrium_state(rho=rho, u=u)
    S.run(f, case.steps if steps is None else steps)
    r, v = S.moments(f)
    return r, v, S.sums(f), S, f


def gpu_sim(case: Case):
    import torch
    sim = lbm.Sim(LAT[case.q], case.shape, case.tau, faces=case.faces, storage=case.storage,
                  pattern=case.pattern)
    if case.solid is not None:
        sim.set_solid(case.solid)
    if case.links is not None:
        sim.set_curved_links(*case.links, order=case.bz_order)
    if case.s is not None:
        sim.set_solid_fraction(case.s.astype(np.float32))
    rho, u = case.init_fields()
    rt = None if rho is None else torch.tensor(rho, dtype=torch.float64, device="cuda")
    ut = None if u is None else torch.tensor(np.moveaxis(u, -1, 0).copy(), dtype=torch.float64, device="cuda")
    sim.init_equilibrium(rt, ut)
    return sim


def gpu_run(case: Case, steps: Optional[int] = None):
    """GPU rho [oshape], u [oshape + (3,)] (numpy FP64), sums, sim."""
    import torch
    sim = gpu_sim(case)
    sim.step(case.steps if steps is None else steps)
    rho, u, sums = sim.moments(dtype=torch.float64, sums=True)
    torch.cuda.synchronize()
    r = rho.cpu().numpy().reshape(case.oshape)
    v = np.zeros(case.oshape + (3,))
    uu = u.cpu().numpy()
    for a in range(case.D):
        v[..., a] = uu[a].reshape(case.oshape)
    return r, v, sums, sim


def fluid_mask(case: Case):
    if case.solid is None:
        return np.ones(case.oshape, bool)
    return ~case.solid.reshape(case.oshape).astype(bool)


def rel_l2(a, b, mask):
    d = (a - b)[mask]
    n = np.linalg.norm(b[mask])
    return float(np.linalg.norm(d) / n) if n > 0 else float(np.linalg.norm(d))


def compare(case: Case, g, o):
    """(u rel-L2, max |rho - rho_oracle|) over fluid cells."""
    m = fluid_mask(case)
    return rel_l2(g[1], o[1], m), float(np.max(np.abs(g[0] - o[0])[m]))


def cone_oracle(q: int, shape, tau: float, faces, center, nsteps: int, init_seed: int, solid=None,
                margin: int = 2, amp: float = 0.03, force=None, collision: int = 0):
    """Oracle (rho, u[3]) at one cell after `nsteps` steps of a run on the full
    grid `shape`, computed on the cell's light cone only: a step moves
    information one cell, so a sub-box reaching nsteps + margin cells around
    the cell gives the full-grid result at its centre.  The sub-box keeps the
    grid's own faces where it reaches them, wraps around periodic axes, and
    has static walls on its cut faces.  The initial state is the seeded wave
    field (inputs.wave_field, periodic on the full grid) on the sub-box.
    force: a uniform body force (exact-difference method); collision: the
    oracle's collision model."""
    D = 2 if q == 9 else 3
    r = nsteps + margin
    lo, sub, of = [], [], []
    for a in range(D):
        c, n = int(center[a]), int(shape[a])
        periodic = int(faces[2 * a][0]) == lbm.PERIODIC
        if periodic and 2 * r + 1 < n:
            lo.append(c - r)
            sub.append(2 * r + 1)
            of += [oracle.Face(oracle.WALL), oracle.Face(oracle.WALL)]
            continue
        l, h = max(c - r, 0), min(c + r + 1, n)
        if periodic:
            l, h = 0, n
        lo.append(l)
        sub.append(h - l)
        of.append(_oface(faces[2 * a]) if l == 0 else oracle.Face(oracle.WALL))
        of.append(_oface(faces[2 * a + 1]) if h == n else oracle.Face(oracle.WALL))
    if q == 9:
        of += [oracle.Face(), oracle.Face()]
    osub = tuple(sub) + ((1,) if q == 9 else ())
    sol = None
    if solid is not None:
        sol = np.asarray(solid)
        for a in range(D):
            sol = np.take(sol, np.arange(lo[a], lo[a] + sub[a]), axis=a, mode="wrap")
        sol = np.ascontiguousarray(sol).reshape(osub).astype(np.uint8)
    edm = None
    if force is not None:
        edm = np.zeros(osub + (3,))
        edm[...] = np.asarray(list(force) + [0.0] * (3 - len(force)))
    S = oracle.Sim(q=q, nx=osub[0], ny=osub[1], nz=osub[2], tau=tau, faces=of, solid=sol, edm=edm,
                   collision=collision)
    rho, u = inputs.wave_field(tuple(shape), init_seed, lo=lo, sub=sub, amp=amp)
    f = S.equilibrium_state(rho=rho.reshape(osub), u=u.reshape(osub + (D,)))
    S.run(f, nsteps)
    R, U = S.moments(f)
    idx = tuple(int(c) - l for c, l in zip(center, lo)) + ((0,) if q == 9 else ())
    return float(R[idx]), U[idx].copy()

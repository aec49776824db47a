"""Seeded synthetic inputs shared by the GPU path's tests/benchmark and the oracle.

This module holds no lattice Boltzmann arithmetic: it only produces the
workload inputs (initial velocity fields, obstacle masks, solid-fraction
fields, batch parameters) from fixed seeds, in FP64 on the host.  Both sides
receive the same arrays; each side turns them into populations with its own
code.

Workloads (shapes follow the paper's test problems):
* Taylor-Green vortex, Sec. 4.1: u = U0 (sin kx cos ky, -cos kx sin ky).
* 3-D lid-driven cavity, Sec. 4.2 and Sec. 5: starts at rest (no generator).
* channel with random spheres: a 3-D obstacle field standing in for the
  paper's channel/obstacle flows (Sec. 4.3/4.4); centres and radii from
  numpy's default_rng(3), added until the solid fraction reaches the target.
* partial bounce-back solid fraction: periodic Gaussian-filtered white noise
  (default_rng(4) for the design field, 40 for the target run), s = (1 + tanh z)/2,
  s = 0 in the first and last 16 columns.
* batched cavities: side lengths, relaxation times and lid speeds from
  default_rng(5).
"""
from __future__ import annotations

import numpy as np


def taylor_green_velocity(nx: int, ny: int, u0: float = 0.01) -> np.ndarray:
    """(nx, ny, 2) float64 Taylor-Green velocity at t = 0 with x_i = i, y_j = j."""
    kx = 2.0 * np.pi / nx
    ky = 2.0 * np.pi / ny
    x = np.arange(nx, dtype=np.float64)[:, None]
    y = np.arange(ny, dtype=np.float64)[None, :]
    u = np.empty((nx, ny, 2))
    u[..., 0] = u0 * np.sin(kx * x) * np.cos(ky * y)
    u[..., 1] = -u0 * np.cos(kx * x) * np.sin(ky * y)
    return u


def random_velocity(shape, dim: int, seed: int, amp: float = 0.03) -> np.ndarray:
    """Seeded smooth-free random velocity (shape + (dim,)), for parity cases."""
    rng = np.random.default_rng(seed)
    return amp * rng.standard_normal(tuple(shape) + (dim,))


def wave_field(shape, seed: int, lo=None, sub=None, amp: float = 0.03, rho_amp: float = 0.01,
               modes: int = 4, xp=None, device=None):
    """Seeded smooth (rho, u) over the box [lo, lo + sub) of a grid of `shape`:
    a sum of `modes` plane waves per component with integer wave numbers in
    [1, 3] per axis (periodic on the full grid), random phases and amplitudes.
    Values depend only on the global cell coordinates, so any sub-box of the
    full field is reproduced exactly.  xp = numpy (default) or torch
    (device tensors for the full-size GPU runs).  Returns rho `sub` and u
    `sub + (D,)` in FP64."""
    rng = np.random.default_rng(seed)
    D = len(shape)
    lo = [0] * D if lo is None else list(lo)
    sub = list(shape) if sub is None else list(sub)
    xp = np if xp is None else xp
    kw = {} if xp is np else {"device": device}
    coords = []
    for a in range(D):
        c = xp.arange(lo[a], lo[a] + sub[a], dtype=xp.float64, **kw)
        coords.append(c.reshape([-1 if b == a else 1 for b in range(D)]))

    def waves(scale):
        out = None
        for _ in range(modes):
            k = rng.integers(1, 4, size=D)
            ph = rng.uniform(0.0, 2.0 * np.pi)
            a = scale * rng.uniform(0.3, 1.0) / modes
            arg = ph
            for d in range(D):
                arg = arg + (2.0 * np.pi * float(k[d]) / shape[d]) * coords[d]
            term = a * xp.sin(arg)
            out = term if out is None else out + term
        return out

    rho = 1.0 + waves(rho_amp)
    u = [waves(amp) for _ in range(D)]
    full = tuple(sub)
    rho = rho + xp.zeros(full, dtype=xp.float64, **kw)
    u = xp.stack([c + xp.zeros(full, dtype=xp.float64, **kw) for c in u], -1)
    return rho, u


def random_density(shape, seed: int, amp: float = 0.01, rho0: float = 1.0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rho0 + amp * rng.standard_normal(tuple(shape))


def sphere_obstacles(nx: int, ny: int, nz: int, seed: int = 3, rmin: float = 8.0, rmax: float = 32.0,
                     xlo: int = 64, xhi: int = 960, fraction: float = 0.05, max_spheres: int = 100000,
                     return_spheres: bool = False):
    """(nx, ny, nz) uint8 obstacle mask: spheres with centres uniform in
    [xlo, xhi) x [0, ny) x [0, nz) and radii uniform in [rmin, rmax], added
    until at least `fraction` of all cells are solid (overlaps allowed).
    Rasterised in FP64: a cell is solid when its centre lies inside a sphere.
    return_spheres: also return the rasterised spheres as rows (cx, cy, cz, r)."""
    rng = np.random.default_rng(seed)
    solid = np.zeros((nx, ny, nz), dtype=np.uint8)
    target = fraction * nx * ny * nz
    count = 0
    balls = []
    for _ in range(max_spheres):
        cx = rng.uniform(xlo, xhi)
        cy = rng.uniform(0, ny)
        cz = rng.uniform(0, nz)
        r = rng.uniform(rmin, rmax)
        x0, x1 = max(int(np.floor(cx - r)), 0), min(int(np.ceil(cx + r)) + 1, nx)
        y0, y1 = max(int(np.floor(cy - r)), 0), min(int(np.ceil(cy + r)) + 1, ny)
        z0, z1 = max(int(np.floor(cz - r)), 0), min(int(np.ceil(cz + r)) + 1, nz)
        if x0 >= x1 or y0 >= y1 or z0 >= z1:
            continue
        X = np.arange(x0, x1, dtype=np.float64)[:, None, None]
        Y = np.arange(y0, y1, dtype=np.float64)[None, :, None]
        Z = np.arange(z0, z1, dtype=np.float64)[None, None, :]
        inside = (X - cx) ** 2 + (Y - cy) ** 2 + (Z - cz) ** 2 <= r * r
        block = solid[x0:x1, y0:y1, z0:z1]
        count += int(np.count_nonzero(inside & (block == 0)))
        block[inside] = 1
        balls.append((cx, cy, cz, r))
        if count >= target:
            break
    if return_spheres:
        return solid, np.array(balls, dtype=np.float64).reshape(-1, 4)
    return solid


def cylinder_obstacle(nx: int, ny: int, cx: float, cy: float, r: float) -> np.ndarray:
    """(nx, ny) uint8 mask of one circular cylinder (the obstacle of the
    paper's flow past a cylinder, Sec. 4.3): cell (i, j) is solid when its
    centre lies within r of (cx, cy)."""
    X = np.arange(nx, dtype=np.float64)[:, None]
    Y = np.arange(ny, dtype=np.float64)[None, :]
    return ((X - cx) ** 2 + (Y - cy) ** 2 <= r * r).astype(np.uint8)


def ball_wall_fractions(solid: np.ndarray, balls: np.ndarray, c: np.ndarray):
    """Curved-wall links of an obstacle mask made of balls (circles in 2-D,
    spheres in 3-D): for every fluid cell x and every direction i >= 1 of the
    caller's velocity set c (Q x D integer rows) whose neighbour x + c_i lies
    in the grid and is solid, the fraction q in (0, 1] of the segment
    x -> x + c_i at which it first enters one of the balls (rows (centre...,
    r)).  Returns (cells, dirs, q): flat C-order cell indices, direction
    indices and fractions, in cell-then-direction order.  Pure geometry in
    FP64 (segment-sphere intersection)."""
    solid = np.asarray(solid).astype(bool)
    shape = solid.shape
    D = solid.ndim
    c = np.asarray(c, dtype=np.int64)[:, :D]
    Q = c.shape[0]
    N = solid.size
    qarr = np.full(N * Q, np.inf)
    coords = np.indices(shape).reshape(D, -1).T.astype(np.float64)   # cell centres, flat order
    for row in np.asarray(balls, dtype=np.float64).reshape(-1, D + 1):
        ctr, r = row[:D], row[D]
        lo = [max(int(np.floor(ctr[a] - r)) - 2, 0) for a in range(D)]
        hi = [min(int(np.ceil(ctr[a] + r)) + 3, shape[a]) for a in range(D)]
        if any(lo[a] >= hi[a] for a in range(D)):
            continue
        box = np.zeros(shape, dtype=bool)
        box[tuple(slice(lo[a], hi[a]) for a in range(D))] = True
        cand = np.flatnonzero(box.reshape(-1) & ~solid.reshape(-1))
        p0 = coords[cand] - ctr
        c0 = np.sum(p0 * p0, axis=1) - r * r
        for i in range(1, Q):
            d = c[i].astype(np.float64)
            a2 = float(d @ d)
            b = p0 @ d
            disc = b * b - a2 * c0
            ok = disc >= 0.0
            t = np.full(cand.size, np.inf)
            t[ok] = (-b[ok] - np.sqrt(disc[ok])) / a2
            hit = ok & (t > 0.0) & (t <= 1.0)
            idx = cand[hit] * Q + i
            qarr[idx] = np.minimum(qarr[idx], t[hit])
    cells, dirs, qs = [], [], []
    flat_solid = solid.reshape(-1)
    for i in range(1, Q):
        src = np.indices(shape).reshape(D, -1)
        dst = src + c[i][:, None]
        inb = np.all((dst >= 0) & (dst < np.array(shape)[:, None]), axis=0)
        k = np.flatnonzero(inb & ~flat_solid)
        dflat = np.ravel_multi_index(tuple(dst[:, k]), shape)
        k = k[flat_solid[dflat]]
        qv = qarr[k * Q + i]
        qv = np.where(np.isfinite(qv), qv, 0.5)
        cells.append(k)
        dirs.append(np.full(k.size, i, dtype=np.int64))
        qs.append(qv)
    cells = np.concatenate(cells) if cells else np.zeros(0, np.int64)
    dirs = np.concatenate(dirs) if dirs else np.zeros(0, np.int64)
    qs = np.concatenate(qs) if qs else np.zeros(0)
    order = np.lexsort((dirs, cells))
    return cells[order], dirs[order], qs[order]


def smooth_solid_fraction(nx: int, ny: int, seed: int = 4, sigma: float = 8.0, edge: int = 16) -> np.ndarray:
    """(nx, ny) float64 field in [0, 1]: periodic Gaussian-filtered (sigma
    cells) white noise normalised to unit std, mapped by (1 + tanh z)/2;
    zero in the first and last `edge` columns of x."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((nx, ny))
    kx = np.fft.fftfreq(nx)[:, None]
    ky = np.fft.fftfreq(ny)[None, :]
    g = np.exp(-2.0 * (np.pi * sigma) ** 2 * (kx * kx + ky * ky))
    z = np.real(np.fft.ifft2(np.fft.fft2(z) * g))
    z = (z - z.mean()) / z.std()
    s = 0.5 * (1.0 + np.tanh(z))
    s[:edge, :] = 0.0
    s[nx - edge:, :] = 0.0
    return s


def batch_cavities(n: int = 256, seed: int = 5, lmin: int = 64, lmax: int = 256,
                   tau_lo: float = 0.52, tau_hi: float = 1.0, u_lo: float = 0.05, u_hi: float = 0.1):
    """Side lengths L_d in [lmin, lmax], tau_d in [tau_lo, tau_hi), lid speeds U_d in [u_lo, u_hi)."""
    rng = np.random.default_rng(seed)
    L = rng.integers(lmin, lmax + 1, size=n)
    tau = rng.uniform(tau_lo, tau_hi, size=n)
    U = rng.uniform(u_lo, u_hi, size=n)
    return L.astype(np.int64), tau, U


def sample_cells(shape, count: int, seed: int) -> np.ndarray:
    """`count` distinct flat cell indices of a grid of `shape`, seeded."""
    rng = np.random.default_rng(seed)
    n = int(np.prod(shape))
    return np.sort(rng.choice(n, size=min(count, n), replace=False))

"""Full-size checks of the body force, the regularized faces and KBC, on the
grids and launches the benchmark times: sampled cells after a few steps from a
seeded wave field against the FP64 oracle on their light cones (faces,
edges, periodic seams, random cells)."""
import sys

import numpy as np
import pytest

from cases import cone_oracle
from paper_2311_16080_amd import inputs, lbm

pytestmark = pytest.mark.gpu
W, P = lbm.WALL, lbm.PERIODIC


def _announce(name):
    print(f"\n[case] {name}", flush=True)
    sys.stdout.flush()


def _run(lattice, shape, tau, faces, steps, seed, amp, setup=None):
    import torch
    sim = lbm.Sim(lattice, shape, tau, faces=faces, storage="f32", pattern="inplace")
    if setup:
        setup(sim)
    rho0, u0 = inputs.wave_field(shape, seed, amp=amp, xp=torch, device="cuda")
    sim.init_equilibrium(rho0, u0.permute(3, 0, 1, 2).contiguous())
    del rho0, u0
    torch.cuda.empty_cache()
    sim.step(steps)
    rho, u = sim.moments(dtype=torch.float32)
    out = (rho.cpu().numpy(), u.cpu().numpy())
    del sim, rho, u
    torch.cuda.empty_cache()
    return out


def _samples(shape, extra, seed=19, n=8):
    rng = np.random.default_rng(seed)
    return list(extra) + [tuple(int(rng.integers(0, m)) for m in shape) for _ in range(n)]


def _compare(q, shape, tau, faces, cells, steps, seed, amp, got, **kw):
    rho, u = got
    worst_u, worst_r = 0.0, 0.0
    for c in cells:
        r_o, u_o = cone_oracle(q, shape, tau, faces, c, steps, seed, amp=amp, **kw)
        u_g = np.array([float(u[a][c]) for a in range(3)])
        worst_u = max(worst_u, float(np.max(np.abs(u_g - u_o))))
        worst_r = max(worst_r, abs(float(rho[c]) - r_o))
    return worst_u, worst_r


def test_forced_channel_full_size_light_cone_samples():
    """768 x 256 x 384 D3Q19 FP32, walls on y, periodic x and z, uniform force."""
    _announce("forced channel 768x256x384 light-cone samples")
    shape, tau, steps, seed, amp = (768, 256, 384), 0.521333, 6, 41, 0.03
    F = (2e-4, -5e-5, 1e-4)
    faces = [(P,), (P,), (W,), (W,), (P,), (P,)]
    got = _run("D3Q19", shape, tau, faces, steps, seed, amp, setup=lambda s: s.set_force(F))
    cells = _samples(shape, [(0, 0, 0), (767, 255, 383), (0, 128, 383), (767, 0, 0), (400, 1, 200), (5, 254, 1)])
    wu, wr = _compare(19, shape, tau, faces, cells, steps, seed, amp, got, force=F)
    print(f"[case] forced channel: max |du| {wu:.3e} (u scale {amp}), max |drho| {wr:.3e}", flush=True)
    assert wu <= 3e-6 and wr <= 1e-6


def test_regularized_channel_full_size_light_cone_samples():
    """512 x 256 x 256 D3Q19 FP32, regularized velocity inlet and pressure outlet, walls."""
    _announce("regularized channel 512x256x256 light-cone samples")
    shape, tau, steps, seed, amp = (512, 256, 256), 0.6, 6, 43, 0.03
    faces = [(lbm.REG_VELOCITY, (0.04, 0.0, 0.0)), (lbm.REG_PRESSURE, (0.0, 0.0, 0.0), 1.0), (W,), (W,), (W,), (W,)]
    got = _run("D3Q19", shape, tau, faces, steps, seed, amp)
    cells = _samples(shape, [(0, 0, 0), (0, 100, 200), (511, 255, 255), (511, 128, 3), (1, 50, 0), (510, 0, 100),
                             (256, 128, 128)])
    wu, wr = _compare(19, shape, tau, faces, cells, steps, seed, amp, got)
    print(f"[case] regularized channel: max |du| {wu:.3e} (u scale {amp}), max |drho| {wr:.3e}", flush=True)
    assert wu <= 3e-6 and wr <= 1e-6


def test_kbc_cavity_full_size_light_cone_samples():
    """256^3 D3Q27 FP32 KBC cavity at tau = 0.5005 (the benchmarked grid)."""
    import oracle
    _announce("kbc cavity 256^3 light-cone samples")
    shape, tau, steps, seed, amp = (256, 256, 256), 0.5005, 6, 47, 0.03
    faces = [(W,)] * 5 + [(W, (0.05, 0.0, 0.0))]
    got = _run("D3Q27", shape, tau, faces, steps, seed, amp, setup=lambda s: s.set_collision("KBC"))
    cells = _samples(shape, [(0, 0, 0), (255, 255, 255), (128, 128, 255), (0, 200, 255), (255, 0, 17), (64, 64, 64)])
    wu, wr = _compare(27, shape, tau, faces, cells, steps, seed, amp, got, collision=oracle.KBC)
    print(f"[case] kbc cavity: max |du| {wu:.3e} (u scale {amp}), max |drho| {wr:.3e}", flush=True)
    assert wu <= 3e-6 and wr <= 1e-6

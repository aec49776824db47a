"""lbm_forces_noalloc (the entry point for callers that cannot allocate)
against lbm_forces, through the C ABI: two calls in a row on one GPU, the
first on a grid whose force rows span two scratch passes (with curved links),
the second on a smaller grid, so a stale scratch from the first call would
show.  FP64 sums in another fixed order: <= 1e-12 of the largest component;
entries that lbm_forces reports as exactly zero stay exactly zero."""
import ctypes
import sys

import numpy as np
import pytest

from cases import Case, gpu_sim
from paper_2311_16080_amd import inputs, lbm

pytestmark = pytest.mark.gpu
W, P, ZV, OUT = lbm.WALL, lbm.PERIODIC, lbm.ZOUHE_VELOCITY, lbm.EQ_OUTFLOW


def _announce(name):
    print(f"\n[case] {name}", flush=True)
    sys.stdout.flush()


def _compare(sim):
    import torch
    ref = np.zeros(21)
    lbm.check(lbm.lib().lbm_forces(sim.h, ref.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    out = torch.full((21,), float("nan"), dtype=torch.float64, device="cuda")
    lbm.check(lbm.lib().lbm_forces_noalloc(sim.h, ctypes.c_void_p(out.data_ptr())))
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    scale = np.max(np.abs(ref))
    assert scale > 0
    assert np.all(np.isfinite(got))
    assert np.max(np.abs(got - ref)) <= 1e-12 * scale, (got, ref)
    assert np.all(got[ref == 0.0] == 0.0)
    return ref


def test_noalloc_forces_match_lbm_forces_two_calls():
    # 1) D3Q19 130 x 130 x 64 channel with spheres and curved links: 16900
    #    step-kernel workgroups + link blocks, two scratch passes
    _announce("noalloc forces, call 1: 130x130x64 spheres with curved links")
    shape = (130, 130, 64)
    solid, balls = inputs.sphere_obstacles(*shape, seed=12, rmin=3.0, rmax=6.0, xlo=8, xhi=120, fraction=0.03,
                                           return_spheres=True)
    c, _ = lbm.lattice_info("D3Q19")
    links = inputs.ball_wall_fractions(solid, balls, c)
    big = Case(19, shape, 0.6, [(ZV, (0.03, 0.0, 0.0)), (OUT, (0, 0, 0), 1.0), (W,), (W, (0.02, 0.0, 0.01)),
                                (W,), (W,)], storage="f64", solid=solid, init_seed=41, links=links, bz_order=2)
    sim = gpu_sim(big)
    sim.step(7)
    _compare(sim)
    del sim
    # 2) a smaller D2Q9 cavity (one pass, no links)
    _announce("noalloc forces, call 2: D2Q9 40x70 cavity")
    small = Case(9, (40, 70), 0.7, [(W,), (W,), (W,), (W, (0.05, 0.0)), (P,), (P,)], storage="f32", init_seed=42)
    sim = gpu_sim(small)
    sim.step(5)
    _compare(sim)


def test_noalloc_forces_argument_checks():
    import torch
    _announce("noalloc forces argument checks")
    sim = gpu_sim(Case(9, (16, 20), 0.7, [(W,), (W,), (W,), (W, (0.05, 0.0)), (P,), (P,)], storage="f32"))
    out = torch.zeros(21, dtype=torch.float64, device="cuda")
    L = lbm.lib()
    assert L.lbm_forces_noalloc(sim.h, ctypes.c_void_p(out.data_ptr())) == lbm.LBM_ESTATE   # no step yet
    assert L.lbm_forces_noalloc(sim.h, None) == lbm.LBM_EINVAL
    sim.step(1)
    assert L.lbm_forces_noalloc(sim.h, ctypes.c_void_p(out.data_ptr())) == lbm.LBM_OK

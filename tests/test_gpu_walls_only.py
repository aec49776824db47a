"""The walls-only step variant (no general path; used for D2Q9 / D3Q27
domains whose lattice faces are all walls) gives bitwise the results of the
full kernel, with solids next to the walls and a moving lid, in both AA
parities and both storage widths."""
import os
import sys

import numpy as np
import pytest

from paper_2311_16080_amd import inputs, lbm

pytestmark = pytest.mark.gpu
W = lbm.WALL


def _run(lattice, shape, faces, storage, solid, walls_only):
    import torch
    old = os.environ.get("LBM_WALLS_ONLY")
    os.environ["LBM_WALLS_ONLY"] = "1" if walls_only else "0"
    try:
        sim = lbm.Sim(lattice, shape, 0.6, faces=faces, storage=storage)
    finally:
        if old is None:
            del os.environ["LBM_WALLS_ONLY"]
        else:
            os.environ["LBM_WALLS_ONLY"] = old
    sim.set_solid(solid)
    D = len(shape)
    rho = torch.tensor(inputs.random_density(shape, 61, amp=0.01), device="cuda")
    u = torch.tensor(np.moveaxis(inputs.random_velocity(shape, D, 62, amp=0.03), -1, 0).copy(), device="cuda")
    sim.init_equilibrium(rho, u)
    out = []
    for n in (10, 11):
        sim.step(n - (out and 10 or 0))
        out.append(sim.moments())
    return out


@pytest.mark.parametrize("lattice,shape", [("D3Q27", (12, 10, 70)), ("D2Q9", (40, 70))])
@pytest.mark.parametrize("storage", ["f32", "f64", "f16"])
def test_walls_only_variant_is_bitwise_the_full_kernel(lattice, shape, storage):
    import torch
    print(f"\n[case] walls-only {lattice} {storage}", flush=True)
    sys.stdout.flush()
    if len(shape) == 3:
        faces = [(W,)] * 5 + [(W, (0.04, 0.01, 0.0))]
        solid = inputs.sphere_obstacles(*shape, seed=9, rmin=1.5, rmax=3, xlo=2, xhi=10, fraction=0.05)
    else:
        faces = [(W,), (W,), (W,), (W, (0.05, 0.0)), (lbm.PERIODIC,), (lbm.PERIODIC,)]
        solid = np.zeros(shape, np.uint8)
        solid[0:4, 30:40] = 1          # touching the -x wall
        solid[20:24, 66:70] = 1        # touching the +y wall
    a = _run(lattice, shape, faces, storage, solid, True)
    b = _run(lattice, shape, faces, storage, solid, False)
    for (ra, ua), (rb, ub) in zip(a, b):
        assert torch.equal(ra, rb) and torch.equal(ua, ub)

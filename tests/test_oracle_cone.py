"""The light-cone oracle (cases.cone_oracle) used by the full-size GPU parity
tests reproduces the oracle's full-grid run at every sampled cell: faces,
corners, periodic wrap, obstacles."""
import numpy as np

import oracle
from cases import _oface, cone_oracle
from paper_2311_16080_amd import inputs, lbm

W, P, ZV, ZP, OUT = lbm.WALL, lbm.PERIODIC, lbm.ZOUHE_VELOCITY, lbm.ZOUHE_PRESSURE, lbm.EQ_OUTFLOW


def _full(q, shape, tau, faces, steps, seed, solid=None):
    of = [_oface(F) for F in faces]
    osh = tuple(shape) + ((1,) if q == 9 else ())
    if q == 9:
        of[4] = of[5] = oracle.Face()
    S = oracle.Sim(q=q, nx=osh[0], ny=osh[1], nz=osh[2], tau=tau, faces=of,
                   solid=None if solid is None else solid.reshape(osh))
    rho, u = inputs.wave_field(tuple(shape), seed)
    f = S.equilibrium_state(rho=rho.reshape(osh), u=u.reshape(osh + (len(shape),)))
    S.run(f, steps)
    return S.moments(f)


def test_cone_matches_full_grid_d3q27_channel():
    shape = (40, 24, 30)
    faces = [(ZV, (0.04, 0, 0)), (OUT, (0, 0, 0), 1.0), (W,), (W, (0.0, 0.0, 0.03)), (P,), (P,)]
    solid = inputs.sphere_obstacles(*shape, seed=3, rmin=2, rmax=4, xlo=5, xhi=35, fraction=0.05)
    R, U = _full(27, shape, 0.6, faces, 5, 9, solid)
    rng = np.random.default_rng(0)
    cells = [(0, 0, 0), (39, 23, 29), (0, 12, 15), (20, 0, 3), (39, 5, 28)]
    cells += [tuple(int(rng.integers(0, n)) for n in shape) for _ in range(8)]
    for c in cells:
        r, v = cone_oracle(27, shape, 0.6, faces, c, 5, 9, solid=solid)
        assert abs(r - R[c]) <= 1e-14 and np.max(np.abs(v - U[c])) <= 1e-15, c


def test_cone_matches_full_grid_d2q9_pressure_channel():
    shape = (50, 30)
    faces = [(ZP, (0, 0, 0), 1.01), (ZP, (0, 0, 0), 0.99), (W, (0.02, 0.0)), (W,), (P,), (P,)]
    R, U = _full(9, shape, 0.7, faces, 6, 4)
    for c in [(0, 0), (49, 29), (0, 15), (25, 0), (25, 14), (3, 28)]:
        r, v = cone_oracle(9, shape, 0.7, faces, c, 6, 4)
        assert abs(r - R[c + (0,)]) <= 1e-14 and np.max(np.abs(v - U[c + (0,)])) <= 1e-15, c

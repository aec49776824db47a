"""Pins of the oracle's momentum-exchange force (orc_forces).

* Momentum balance, exact up to rounding: in a closed domain (walls,
  periodic faces, solid obstacles, moving walls) collision and free
  streaming conserve momentum, so the change of the fluid's momentum over a
  step is minus the force handed to the solids and walls:
  P(t+1) - P(t) = -(F_solid + sum_f F_face(f)).  P comes from orc_sums, a
  separate code path.
* Steady Couette flow: the shear force on the moving wall is
  -rho nu (U / ny) per unit area (nu = (tau - 1/2) / 3), +rho nu U / ny on the
  static wall; the normal force is the pressure rho / 3 per unit area.
"""
import numpy as np
import pytest

from oracle import Face, PERIODIC, Sim, WALL
from paper_2311_16080_amd import inputs


def _closed_cases():
    sph = inputs.sphere_obstacles(10, 9, 12, seed=3, rmin=1.5, rmax=2.5, xlo=3, xhi=7, fraction=0.04)
    cube = np.zeros((8, 8, 8), np.uint8)
    cube[3:5, 3:6, 2:4] = 1
    plate = np.zeros((24, 16, 1), np.uint8)
    plate[10:12, 5:11, 0] = 1
    return {
        "d3q19_walls_spheres": (19, (10, 9, 12), [Face(WALL), Face(WALL, (0, 0.02, 0.01)), Face(WALL), Face(WALL),
                                                  Face(WALL), Face(WALL, (0.05, 0.01, 0))], sph),
        "d3q27_lid_cube": (27, (8, 8, 8), [Face(WALL)] * 5 + [Face(WALL, (0.04, 0, 0))], cube),
        "d2q9_periodic_x_plate": (9, (24, 16, 1), [Face(), Face(), Face(WALL), Face(WALL, (0.03, 0, 0)), Face(),
                                                   Face()], plate),
        "d3q19_periodic_obstacle": (19, (8, 8, 8), [Face()] * 6, cube),
    }


@pytest.mark.parametrize("name", sorted(_closed_cases()))
def test_momentum_balance_is_exact(oracle_mod, name):
    q, shape, faces, solid = _closed_cases()[name]
    S = Sim(q=q, nx=shape[0], ny=shape[1], nz=shape[2], tau=0.7, faces=faces, solid=solid)
    D = 2 if q == 9 else 3
    rho = inputs.random_density(shape, 11, amp=0.01)
    u = inputs.random_velocity(shape, D, 12, amp=0.03)
    f = S.equilibrium_state(rho=rho, u=u)
    for _ in range(5):
        P0 = S.sums(f)[1:4]
        S.run(f, 1)
        P1 = S.sums(f)[1:4]
        Fs, Ff = S.forces(f)
        total = Fs + Ff.sum(0)
        scale = np.abs(Fs).sum() + np.abs(Ff).sum()
        assert scale > 0
        assert np.max(np.abs((P1 - P0) + total)) <= 1e-12 * scale, (P1 - P0, total)


@pytest.mark.parametrize("q", [9, 19, 27])
@pytest.mark.parametrize("tau", [0.6, 1.1])
def test_couette_wall_forces(oracle_mod, q, tau):
    ny, U, nx = 8, 0.01, 2
    nz = 1 if q == 9 else 2
    faces = [Face(), Face(), Face(WALL), Face(WALL, (U, 0, 0)), Face(), Face()]
    S = Sim(q=q, nx=nx, ny=ny, nz=nz, tau=tau, faces=faces)
    f = S.equilibrium_state()
    S.run(f, 40000)
    Fs, Ff = S.forces(f)
    area = nx * nz
    shear = (tau - 0.5) / 3.0 * U / ny * area
    assert np.all(Fs == 0.0)
    assert abs(Ff[3, 0] + shear) <= 1e-10 * shear       # moving wall (+y face)
    assert abs(Ff[2, 0] - shear) <= 1e-10 * shear       # static wall (-y face)
    assert abs(Ff[3, 1] - area / 3.0) <= 1e-10 * area   # pressure rho / 3 outward
    assert abs(Ff[2, 1] + area / 3.0) <= 1e-10 * area

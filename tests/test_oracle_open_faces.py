"""Pins of the oracle's open-face fills that no other test fixes exactly: the
equilibrium outflow (reading O7(3): f_i = feq_i(rho_face, u(x, t)) for the
directions whose source lies across the outflow face) and the perimeter rule
of open faces (reading O7(4): on a cell that also lies on a wall face, the
face-crossing directions that do not cross the wall take feq(rho0, u_in) on a
velocity face and feq(rho_w, u(x, t)) on a pressure face).

Each case starts from a uniform equilibrium that every rule of the step
reproduces exactly when it is computed as read -- the BGK collision leaves an
equilibrium unchanged (eq. LBM-BGK), streaming moves a uniform field onto
itself (eq. streaming), halfway bounce-back of feq(rho0, u_w) off a wall moving
at u_w returns feq(rho0, u_w) (the moving-wall term is the odd part
6 w_i rho0 c_i.u_w), and Zou-He's closure restores the moments it is given
(Sec. 3.5) -- so the state must stay a fixed point to rounding over 200 steps.
A fill that used rho0 in place of rho_face / rho_w, u = 0 in place of the
cell's velocity, or a linear equilibrium breaks the fixed point at the first
step by O(|rho_face - rho0|) or O(|u|^2)."""
import numpy as np
import pytest

from oracle import OUTFLOW, PERIODIC, WALL, ZOUHE_PRES, ZOUHE_VEL, Face, Sim

TOL = 2e-15          # per population, after 200 steps (populations are O(0.01 .. 0.4))
STEPS = 200


def _shape(q):
    return (12, 8, 1) if q == 9 else (10, 6, 5)


def _run_fixed_point(q, faces, rho, u):
    nx, ny, nz = _shape(q)
    if q == 9:
        faces = faces[:4] + [Face(PERIODIC), Face(PERIODIC)]
    S = Sim(q=q, nx=nx, ny=ny, nz=nz, tau=0.7, faces=faces)
    uu = np.zeros((nx, ny, nz, 3))
    uu[...] = np.asarray(u, dtype=np.float64)
    f0 = S.equilibrium_state(rho=np.full((nx, ny, nz), rho), u=uu)
    f = f0.copy()
    S.run(f, STEPS)
    return float(np.max(np.abs(f - f0)))


@pytest.mark.parametrize("q", [9, 19, 27])
def test_outflow_fill_uses_face_density_and_cell_velocity(oracle_mod, q):
    """Velocity inlet (Zou-He) -> equilibrium outflow at rho_face = 1.02 != rho0,
    periodic transverse faces: the plug flow feq(1.02, u0) is a fixed point only
    if the outflow fill is feq(rho_face, u(x, t)) with the full quadratic
    equilibrium (u0 has tangential parts, so the inlet's transverse
    corrections are exercised as well)."""
    u0 = (0.05, 0.01, 0.0) if q == 9 else (0.05, 0.01, -0.02)
    faces = [Face(ZOUHE_VEL, u0), Face(OUTFLOW, (0, 0, 0), 1.02)] + [Face(PERIODIC)] * 4
    err = _run_fixed_point(q, faces, 1.02, u0)
    assert err <= TOL, err


@pytest.mark.parametrize("q", [9, 19, 27])
def test_open_face_perimeters_next_to_moving_walls(oracle_mod, q):
    """Velocity inlet and equilibrium outflow with every transverse face a wall
    moving at the plug velocity u0: feq(rho0, u0) is a fixed point only if the
    perimeter cells of the inlet take feq(rho0, u_in) and those of the outflow
    feq(rho_face, u(x, t)) for the directions that cross the open face alone,
    and bounce back with the wall's term where a wall is crossed too."""
    u0 = (0.05, 0.0, 0.0)
    faces = [Face(ZOUHE_VEL, u0), Face(OUTFLOW, (0, 0, 0), 1.0)] + [Face(WALL, u0)] * 4
    err = _run_fixed_point(q, faces, 1.0, u0)
    assert err <= TOL, err


@pytest.mark.parametrize("q", [9, 19, 27])
@pytest.mark.parametrize("outlet", ["pressure", "outflow"])
def test_pressure_perimeters_use_face_density(oracle_mod, q, outlet):
    """Pressure inlet at rho_w = 1.03 != rho0, a pressure outlet (or an
    equilibrium outflow) at the same density, static walls: the rest state
    feq(1.03, 0) is a fixed point only if the pressure faces' perimeter cells
    take feq(rho_w, u(x, t)) and the outflow's feq(rho_face, u(x, t)), not
    rho0."""
    rw = 1.03
    out = Face(ZOUHE_PRES, (0, 0, 0), rw) if outlet == "pressure" else Face(OUTFLOW, (0, 0, 0), rw)
    faces = [Face(ZOUHE_PRES, (0, 0, 0), rw), out] + [Face(WALL)] * 4
    err = _run_fixed_point(q, faces, rw, (0.0, 0.0, 0.0))
    assert err <= TOL, err


@pytest.mark.parametrize("q", [9, 19, 27])
def test_fixed_points_detect_a_wrong_fill(oracle_mod, q):
    """The same fixed points are broken by a fill with the wrong density: the
    plug flow at 1.02 with an outflow face declared at rho0 drifts by
    O(0.02 w_i) within the run (so the pins above are not vacuous)."""
    u0 = (0.05, 0.01, 0.0) if q == 9 else (0.05, 0.01, -0.02)
    faces = [Face(ZOUHE_VEL, u0), Face(OUTFLOW, (0, 0, 0), 1.0)] + [Face(PERIODIC)] * 4
    err = _run_fixed_point(q, faces, 1.02, u0)
    assert err > 1e-4, err

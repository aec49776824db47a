"""Pins of the oracle's regularized velocity / pressure faces (Latt et al.
2008; listed among the paper's boundary conditions, Sec. 3.5).

* The closed face cell carries exactly the prescribed moments: (rho, rho u_w)
  with rho from the known populations on a velocity face, (rho_w, rho_w u_n n)
  on a pressure face.
* Its non-equilibrium part lies in the span of the second-order Hermite
  tensors w_i (c_i c_i - I/3): least squares leaves no residual, so the
  higher-order (ghost) content is removed; and its momentum flux is
  rho/3 I + rho u u + Pi_neq with Pi_neq of the bounce-back-completed input.
* An equilibrium with the face's own (rho, u) is a fixed point.
* Uniform plug flow: a regularized velocity inlet and pressure outlet in a
  channel periodic across converge from rest to u = u_in, rho = rho_out.
* Pressure-driven Poiseuille between static walls: the mid-channel profile is
  the parabola of the measured pressure gradient.
"""
import numpy as np
import pytest

from oracle import Face, PERIODIC, REG_PRES, REG_VEL, Sim, WALL, equilibrium, tables


def _normal(face):
    n = np.zeros(3)
    n[face // 2] = 1.0 if face % 2 == 0 else -1.0
    return n


@pytest.mark.parametrize("q", [9, 19, 27])
@pytest.mark.parametrize("face", [0, 1, 2, 3, 4, 5])
@pytest.mark.parametrize("kind", [REG_VEL, REG_PRES])
def test_regularized_closure_moments_and_structure(q, face, kind):
    if q == 9 and face >= 4:
        pytest.skip("2-D lattice has no z faces")
    rng = np.random.default_rng(500 + q + 7 * face + kind)
    c, w, _ = tables(q)
    c = c.astype(np.float64)
    n = _normal(face)
    uw = 0.05 * rng.standard_normal(3)
    if q == 9:
        uw[2] = 0.0
    rhow = 1.0 + 0.02 * rng.standard_normal()
    faces = [Face() for _ in range(6)]
    faces[face] = Face(kind, tuple(uw), rhow)
    S = Sim(q=q, nx=3, ny=3, nz=1 if q == 9 else 3, faces=faces)
    f = equilibrium(q, 1.0 + 0.01 * rng.standard_normal(), 0.03 * rng.standard_normal(3) * (
        np.array([1, 1, 0]) if q == 9 else 1)) * (1 + 0.05 * rng.standard_normal(q))
    cn = c @ n
    g = S.zouhe_closure(face, f.copy())
    known = f[cn == 0].sum() + 2 * f[cn == -1].sum()
    if kind == REG_VEL:
        rho = known / (1.0 - uw @ n)
        u = uw
    else:
        rho = rhow
        u = (1.0 - known / rhow) * n
    assert abs(g.sum() - rho) < 1e-14
    assert np.max(np.abs(g @ c - rho * u)) < 1e-14
    feq = equilibrium(q, rho, u)
    # non-equilibrium in the span of w_i Q_i
    basis = []
    for a in range(3):
        for b in range(a, 3):
            basis.append(w * (c[:, a] * c[:, b] - (1.0 / 3.0 if a == b else 0.0)))
    B = np.array(basis).T
    coef, *_ = np.linalg.lstsq(B, g - feq, rcond=None)
    assert np.max(np.abs(B @ coef - (g - feq))) < 1e-14
    # momentum flux: rho/3 I + rho u u + Pi_neq of the completed input
    fneq = f - feq
    opp = [int(np.where(np.all(c == -c[i], axis=1))[0][0]) for i in range(q)]
    for i in range(q):
        if cn[i] == 1:
            fneq[i] = fneq[opp[i]]
    Pi = (c * fneq[:, None]).T @ c
    if q == 9:
        Pi[2, :] = Pi[:, 2] = 0.0
    M2 = (c * g[:, None]).T @ c
    expect = rho / 3.0 * np.diag([1, 1, 0 if q == 9 else 1]) + rho * np.outer(u, u) + Pi
    assert np.max(np.abs(M2 - expect)) < 1e-14


@pytest.mark.parametrize("q", [9, 19])
@pytest.mark.parametrize("kind", [REG_VEL, REG_PRES])
def test_equilibrium_is_a_fixed_point(q, kind):
    rng = np.random.default_rng(600 + q + kind)
    face = 0
    n = _normal(face)
    uw = np.array([0.04, 0.01, 0.0 if q == 9 else -0.02])
    rho = 1.01
    faces = [Face() for _ in range(6)]
    if kind == REG_VEL:
        faces[face] = Face(kind, tuple(uw), 1.0)
        u = uw
    else:
        faces[face] = Face(kind, (0, 0, 0), rho)
        u = 0.03 * n
    S = Sim(q=q, nx=3, ny=3, nz=1 if q == 9 else 3, faces=faces)
    rho_in = rho
    if kind == REG_VEL:
        rho_in = 1.0 + 0.02 * rng.random()
    f = equilibrium(q, rho_in, u)
    g = S.zouhe_closure(face, f.copy())
    assert np.max(np.abs(g - f)) < 1e-15


@pytest.mark.parametrize("q", [9, 19])
def test_plug_flow_converges(q):
    u0, nx = 0.03, 16
    faces = [Face(REG_VEL, (u0, 0, 0)), Face(REG_PRES, (0, 0, 0), 1.0), Face(), Face(), Face(), Face()]
    nz = 1 if q == 9 else 2
    S = Sim(q=q, nx=nx, ny=2, nz=nz, tau=0.8, faces=faces)
    f = S.equilibrium_state()
    S.run(f, 20000)                 # acoustic transients decay slowly through the open faces
    rho, u = S.moments(f)
    assert np.max(np.abs(u[..., 0] - u0)) < 1e-10
    assert np.max(np.abs(u[..., 1:])) < 1e-12
    assert np.max(np.abs(rho - 1.0)) < 1e-10


def test_pressure_driven_poiseuille():
    q, nx, ny, tau = 9, 40, 9, 0.5 + np.sqrt(3) / 4
    d = 5e-4
    faces = [Face(REG_PRES, (0, 0, 0), 1.0 + d), Face(REG_PRES, (0, 0, 0), 1.0 - d), Face(WALL), Face(WALL),
             Face(), Face()]
    S = Sim(q=q, nx=nx, ny=ny, nz=1, tau=tau, faces=faces)
    f = S.equilibrium_state()
    S.run(f, 30000)
    rho, u = S.moments(f)
    nu = (tau - 0.5) / 3
    x0 = nx // 2
    G = -(rho[x0 + 1, :, 0].mean() - rho[x0 - 1, :, 0].mean()) / 2.0 / 3.0     # -dp/dx, p = rho / 3
    y = np.arange(ny) + 0.5
    ex = G / (2 * rho[x0, :, 0].mean() * nu) * y * (ny - y)
    err = np.max(np.abs(u[x0, :, 0, 0] - ex)) / ex.max()
    assert err < 2e-3

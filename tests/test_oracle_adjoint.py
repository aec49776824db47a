"""Pins of the oracle's discrete adjoint (the transpose of one step's Jacobian).

The adjoint is the exact transpose of the derivative of the forward map, so it
is pinned by linear algebra on the forward oracle alone:
* a dense Jacobian built column by column with central differences on a tiny
  grid (walls, a moving wall, a solid cell, Zou-He, outflow, partial
  bounce-back, regularized velocity and pressure faces, the KBC collision)
  equals the transpose the adjoint applies, row by row;
* the dot-product identity <w, J v> = <J^T w, v> on a larger grid;
* finite-difference gradients of a velocity loss through several steps with
  respect to the solid fraction s, tau and the lid velocity.
"""
import numpy as np
import pytest

from oracle import KBC, Face, OUTFLOW, REG_PRES, REG_VEL, Sim, WALL, ZOUHE_PRES, ZOUHE_VEL

KINDS = ["cavity", "channel", "pressure", "regularized", "kbc_cavity", "kbc_channel"]


def _scene(q, kind, rng):
    collision = 0
    if kind.startswith("kbc_"):
        # the KBC collision (its Jacobian is the oracle's complex step)
        collision, kind = KBC, kind[4:]
    if q == 9:
        nx, ny, nz = 6, 5, 1
    else:
        nx, ny, nz = 5, 4, 4
    faces = [Face() for _ in range(6)]
    if kind == "cavity":
        faces = [Face(WALL) for _ in range(6)]
        lid = 3 if q == 9 else 5
        faces[lid] = Face(WALL, (0.07, 0, 0))
    elif kind == "channel":
        faces[0] = Face(ZOUHE_VEL, (0.04, 0.01 if q != 9 else 0.0, 0))
        faces[1] = Face(OUTFLOW, (0, 0, 0), 1.0)
        faces[2] = Face(WALL)
        faces[3] = Face(WALL, (0.03, 0, 0))
    elif kind == "pressure":
        faces[0] = Face(ZOUHE_VEL, (0.03, 0, 0))
        faces[1] = Face(ZOUHE_PRES, (0, 0, 0), 0.995)
        if q != 9:
            faces[4] = Face(WALL)
            faces[5] = Face(WALL)
    elif kind == "regularized":
        # regularized velocity inlet and pressure outlet; walls on y (perimeter
        # cells), periodic z
        faces[0] = Face(REG_VEL, (0.04, 0.01 if q != 9 else 0.0, 0))
        faces[1] = Face(REG_PRES, (0, 0, 0), 0.995)
        faces[2] = Face(WALL)
        faces[3] = Face(WALL, (0.03, 0, 0))
    solid = np.zeros((nx, ny, nz), np.uint8)
    solid[nx // 2, ny // 2, nz // 2] = 1
    s = np.clip(0.3 + 0.2 * rng.standard_normal((nx, ny, nz)), 0, 1)
    S = Sim(q=q, nx=nx, ny=ny, nz=nz, tau=0.67, faces=faces, solid=solid, s=s, collision=collision)
    u = 0.03 * rng.standard_normal((nx, ny, nz, 3))
    if q == 9:
        u[..., 2] = 0
    f = S.equilibrium_state(rho=1 + 0.01 * rng.standard_normal((nx, ny, nz)), u=u)
    f *= 1 + 0.02 * rng.standard_normal(f.shape)
    f[solid.astype(bool)] = 0
    return S, f


def _fd_step(kind):
    # KBC's gamma is a ratio of two entropic products of the small non-shear
    # part, so its third derivatives are large: central differences need a
    # smaller step there (truncation 6e-8 at 1e-6, 9e-10 at 1e-7)
    return 1e-7 if kind.startswith("kbc_") else 1e-6


def _step(S, f):
    g = f.copy()
    S.run(g, 1)
    return g


@pytest.mark.parametrize("kind", KINDS)
def test_dense_jacobian_transpose_d2q9(oracle_mod, kind):
    rng = np.random.default_rng(1 + KINDS.index(kind))
    S, f = _scene(9, kind, rng)
    fluid = ~S.solid.astype(bool)
    idx = [(x, y, z, i) for x, y, z in zip(*np.nonzero(fluid)) for i in range(9)]
    eps = _fd_step(kind)
    J = np.zeros((len(idx), len(idx)))
    for col, k in enumerate(idx):
        fp, fm = f.copy(), f.copy()
        fp[k] += eps
        fm[k] -= eps
        d = (_step(S, fp) - _step(S, fm)) / (2 * eps)
        J[:, col] = [d[r] for r in idx]
    # rows of J^T via the adjoint of unit vectors on the output
    worst = 0.0
    for row, k in enumerate(idx):
        a = np.zeros_like(f)
        a[k] = 1.0
        at, _, _, _ = S.adjoint_step(f, a)
        jt = np.array([at[r] for r in idx])
        worst = max(worst, np.max(np.abs(jt - J[row, :])))
    assert worst < 1e-8


@pytest.mark.parametrize("q", [9, 19, 27])
@pytest.mark.parametrize("kind", KINDS)
def test_dot_product_identity(oracle_mod, q, kind):
    if q == 19 and kind.startswith("kbc_"):
        pytest.skip("KBC runs on D2Q9 and D3Q27")
    rng = np.random.default_rng(7 + q)
    S, f = _scene(q, kind, rng)
    fluid = ~S.solid.astype(bool)
    v = rng.standard_normal(f.shape) * fluid[..., None]
    w = rng.standard_normal(f.shape) * fluid[..., None]
    eps = _fd_step(kind)
    Jv = (_step(S, f + eps * v) - _step(S, f - eps * v)) / (2 * eps)
    JTw, _, _, _ = S.adjoint_step(f, w)
    lhs = np.sum(w * Jv)
    rhs = np.sum(JTw * v)
    assert abs(lhs - rhs) <= 1e-7 * max(abs(lhs), 1.0)


def _loss_and_grad(S, f0, nsteps, target):
    states = S.trajectory(f0, nsteps)
    rho, u = S.moments(states[-1])
    fluid = (~S.solid.astype(bool)) if S.solid is not None else np.ones(S.shape, bool)
    diff = (u - target) * fluid[..., None]
    L = np.sum(diff ** 2)
    seed = S.seed_from_velocity_grad(states[-1], 2 * diff)
    _, dlds, dtau, duw = S.adjoint(states, seed)
    return L, dlds, dtau, duw


def _loss(S, f0, nsteps, target):
    f = f0.copy()
    S.run(f, nsteps)
    _, u = S.moments(f)
    fluid = (~S.solid.astype(bool)) if S.solid is not None else np.ones(S.shape, bool)
    return np.sum(((u - target) * fluid[..., None]) ** 2)


@pytest.mark.parametrize("q,kind", [(9, "channel"), (19, "channel"), (9, "regularized"), (19, "regularized"),
                                    (9, "kbc_channel"), (27, "kbc_channel")])
def test_parameter_gradients_match_finite_differences(oracle_mod, q, kind):
    rng = np.random.default_rng(11 + q)
    S, f0 = _scene(q, kind, rng)
    nsteps = 6
    target = 0.02 * rng.standard_normal(S.shape + (3,))
    L, dlds, dtau, duw = _loss_and_grad(S, f0, nsteps, target)
    h = 1e-6
    base_s = S.s.copy()
    cells = [tuple(c) for c in np.argwhere(~S.solid.astype(bool))[::5]]
    for cell in cells:
        S.s = base_s.copy(); S.s[cell] += h
        Lp = _loss(S, f0, nsteps, target)
        S.s = base_s.copy(); S.s[cell] -= h
        Lm = _loss(S, f0, nsteps, target)
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - dlds[cell]) <= 1e-6 * max(abs(fd), 1e-3 * abs(L)), cell
    S.s = base_s
    tau0 = S.tau
    S.tau = tau0 + h
    Lp = _loss(S, f0, nsteps, target)
    S.tau = tau0 - h
    Lm = _loss(S, f0, nsteps, target)
    S.tau = tau0
    fd = (Lp - Lm) / (2 * h)
    assert abs(fd - dtau) <= 1e-6 * abs(fd)
    # moving +y wall, x component
    u0 = S.faces[3].u
    S.faces[3] = Face(WALL, (u0[0] + h, 0, 0))
    Lp = _loss(S, f0, nsteps, target)
    S.faces[3] = Face(WALL, (u0[0] - h, 0, 0))
    Lm = _loss(S, f0, nsteps, target)
    S.faces[3] = Face(WALL, u0)
    fd = (Lp - Lm) / (2 * h)
    assert abs(fd - duw[3, 0]) <= 1e-6 * abs(fd)


def test_kinetic_energy_seed(oracle_mod):
    """d(1/2 rho |u|^2)/df_i = c_i.u - |u|^2/2 (from rho = sum f, rho u = sum c f),
    checked against central differences of the oracle's own moments."""
    rng = np.random.default_rng(5)
    q = 9
    c, _, _ = oracle_mod.tables(q)
    f = oracle_mod.equilibrium(q, 1.01, [0.03, -0.02, 0]) * (1 + 0.05 * rng.standard_normal(q))
    rho, u = oracle_mod.cell_moments(f)
    an = c @ u - 0.5 * u @ u
    h = 1e-6
    for i in range(q):
        fp, fm = f.copy(), f.copy()
        fp[i] += h
        fm[i] -= h
        rp, up = oracle_mod.cell_moments(fp)
        rm, um = oracle_mod.cell_moments(fm)
        fd = (0.5 * rp * up @ up - 0.5 * rm * um @ um) / (2 * h)
        assert abs(fd - an[i]) < 1e-9

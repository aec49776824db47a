"""Pins of the oracle's body force by the exact-difference method (paper
Sec. 4.4 and 6.1, after Kupershtokh): the relaxed populations gain
feq_i(rho, u + F/rho) - feq_i(rho, u).

* Uniform force on a uniform rest state, periodic box: BGK keeps an
  equilibrium, so after n steps f = feq(rho0, n F / rho0) exactly (rho0 != 1
  catches a missing division by rho).
* One step from rest with a force field F(x): f_i(x, 1) is the equilibrium
  with velocity F(x - c_i) / rho0 at the upstream cell (catches an index or
  axis mix-up of the per-cell force).
* Moments of the change at a single cell (a one-cell periodic box, where a
  step is one collision): zero mass, momentum F, and momentum flux
  rho (u'u' - uu) with u' = u + F/rho -- the textbook moments of the
  second-order equilibrium; the force-free step is subtracted.
* Random state and random force field, periodic box: mass is kept and the
  momentum grows by exactly sum_x F(x) each step.
* Force-driven Poiseuille between static halfway walls: the velocity
  u + F/(2 rho) (the method's physical velocity) is the exact parabola at
  tau = 1/2 + sqrt(3)/4, with the usual wall slip elsewhere.
"""
import numpy as np
import pytest

from oracle import Face, Sim, WALL, equilibrium, tables


def _dims(q):
    return 2 if q == 9 else 3


@pytest.mark.parametrize("q", [9, 19, 27])
def test_uniform_force_keeps_shifted_equilibrium(q):
    rho0, n = 1.3, 9
    F = np.array([1.5e-4, -2.5e-4, 3e-4])
    if q == 9:
        F[2] = 0.0
    shape = (4, 5, 1) if q == 9 else (4, 5, 6)
    S = Sim(q=q, nx=shape[0], ny=shape[1], nz=shape[2], tau=0.7,
            edm=np.broadcast_to(F, shape + (3,)).copy())
    f = S.equilibrium_state(rho=np.full(shape, rho0))
    S.run(f, n)
    expect = equilibrium(q, rho0, n * F / rho0)
    assert np.max(np.abs(f - expect)) < 1e-15
    rho, u = S.moments(f)
    assert np.max(np.abs(rho - rho0)) < 1e-14
    assert np.max(np.abs(u - n * F / rho0)) < 1e-15


@pytest.mark.parametrize("q", [9, 19, 27])
def test_one_step_streams_the_local_forced_equilibrium(q):
    rng = np.random.default_rng(40 + q)
    rho0 = 0.9
    shape = (5, 6, 1) if q == 9 else (5, 4, 6)
    F = 1e-3 * rng.standard_normal(shape + (3,))
    if q == 9:
        F[..., 2] = 0.0
    S = Sim(q=q, nx=shape[0], ny=shape[1], nz=shape[2], tau=0.8, edm=F)
    f = S.equilibrium_state(rho=np.full(shape, rho0))
    S.run(f, 1)
    c, _, _ = tables(q)
    err = 0.0
    for x in np.ndindex(shape):
        for i in range(q):
            up = tuple((x[a] - c[i][a]) % shape[a] for a in range(3))
            e = equilibrium(q, rho0, F[up] / rho0)[i]
            err = max(err, abs(f[x][i] - e))
    assert err < 1e-15


@pytest.mark.parametrize("q", [9, 19, 27])
def test_single_cell_moments_of_the_change(q):
    rng = np.random.default_rng(70 + q)
    c, w, _ = tables(q)
    c = c.astype(np.float64)
    D = _dims(q)
    rho = 1.0 + 0.1 * rng.random()
    u = np.zeros(3)
    u[:D] = 0.05 * rng.standard_normal(D)
    f0 = equilibrium(q, rho, u) * (1 + 0.05 * rng.standard_normal(q))   # off equilibrium
    F = np.zeros(3)
    F[:D] = 2e-3 * rng.standard_normal(D)
    outs = []
    for edm in (None, F):
        S = Sim(q=q, nx=1, ny=1, nz=1, tau=0.75, edm=None if edm is None else edm.reshape(1, 1, 1, 3))
        f = f0.reshape(1, 1, 1, q).copy()
        S.run(f, 1)
        outs.append(f.reshape(q))
    d = outs[1] - outs[0]
    r = f0.sum()
    v = (f0 @ c) / r
    vp = v + F / r
    assert abs(d.sum()) < 1e-15
    assert np.max(np.abs(d @ c - F)) < 1e-15
    flux = (c * d[:, None]).T @ c
    assert np.max(np.abs(flux - r * (np.outer(vp, vp) - np.outer(v, v)))) < 1e-15


@pytest.mark.parametrize("q", [9, 19, 27])
def test_periodic_momentum_grows_by_the_total_force(q):
    rng = np.random.default_rng(90 + q)
    shape = (6, 7, 1) if q == 9 else (5, 6, 7)
    D = _dims(q)
    F = np.zeros(shape + (3,))
    F[..., :D] = 1e-3 * rng.standard_normal(shape + (D,))
    S = Sim(q=q, nx=shape[0], ny=shape[1], nz=shape[2], tau=0.6, edm=F)
    rho = 1.0 + 0.05 * rng.random(shape)
    u = np.zeros(shape + (3,))
    u[..., :D] = 0.04 * rng.standard_normal(shape + (D,))
    f = S.equilibrium_state(rho=rho, u=u)
    f *= 1 + 0.02 * rng.standard_normal(f.shape)
    c, _, _ = tables(q)
    for _ in range(3):
        m0 = f.sum()
        P0 = (f.reshape(-1, q) @ c.astype(np.float64)).sum(0)
        S.run(f, 1)
        P1 = (f.reshape(-1, q) @ c.astype(np.float64)).sum(0)
        assert abs(f.sum() - m0) < 1e-12 * m0
        assert np.max(np.abs(P1 - P0 - F.reshape(-1, 3).sum(0))) < 1e-13


@pytest.mark.parametrize("q", [9, 19])
def test_poiseuille_edm_magic_tau_exact(q):
    ny, Fx = 8, 1e-6
    nz = 1 if q == 9 else 2
    shape = (2, ny, nz)
    faces = [Face(), Face(), Face(WALL), Face(WALL), Face(), Face()]
    y = np.arange(ny) + 0.5
    field = np.zeros(shape + (3,))
    field[..., 0] = Fx
    errs = {}
    for tau in (0.5 + np.sqrt(3) / 4, 0.8):
        nu = (tau - 0.5) / 3
        S = Sim(q=q, nx=2, ny=ny, nz=nz, tau=tau, faces=faces, edm=field)
        f = S.equilibrium_state()
        S.run(f, 100000)
        rho, u = S.moments(f)
        ex = Fx / (2 * nu) * y * (ny - y)
        errs[tau] = np.max(np.abs(u[0, :, 0, 0] + Fx / (2 * rho[0, :, 0]) - ex)) / ex.max()
    assert errs[0.5 + np.sqrt(3) / 4] < 1e-10
    assert 1e-3 < errs[0.8] < 3e-2


# ---- adjoint of the body force ------------------------------------------------
# Pinned by linear algebra on the forward oracle alone: the dot-product identity
# <w, J v> = <J^T w, v> of one step with the force on, and central differences
# of a velocity loss through several steps with respect to force-field entries,
# the uniform force, s and tau.
from test_oracle_adjoint import _scene, _step   # noqa: E402


def _with_force(S, rng, amp=3e-3):
    F = np.zeros(S.shape + (3,))
    D = 2 if S.q == 9 else 3
    F[..., :D] = amp * rng.standard_normal(S.shape + (D,))
    S.edm = F
    return F


@pytest.mark.parametrize("q", [9, 19, 27])
@pytest.mark.parametrize("kind", ["cavity", "channel", "pressure"])
def test_edm_dot_product_identity(q, kind):
    rng = np.random.default_rng(300 + q)
    S, f = _scene(q, kind, rng)
    _with_force(S, rng)
    fluid = ~S.solid.astype(bool)
    v = rng.standard_normal(f.shape) * fluid[..., None]
    w = rng.standard_normal(f.shape) * fluid[..., None]
    eps = 1e-6
    Jv = (_step(S, f + eps * v) - _step(S, f - eps * v)) / (2 * eps)
    JTw, _, _, _ = S.adjoint_step(f, w)
    lhs = np.sum(w * Jv)
    rhs = np.sum(JTw * v)
    assert abs(lhs - rhs) <= 1e-7 * max(abs(lhs), 1.0)
    # and the force term is really in the transpose: without it the identity fails
    S.edm = None
    JTw0, _, _, _ = S.adjoint_step(f, w)
    assert abs(np.sum(JTw0 * v) - lhs) > 1e-6 * max(abs(lhs), 1.0)


def _edm_loss(S, f0, nsteps, target):
    f = f0.copy()
    S.run(f, nsteps)
    _, u = S.moments(f)
    fluid = ~S.solid.astype(bool)
    return np.sum(((u - target) * fluid[..., None]) ** 2)


@pytest.mark.parametrize("q", [9, 19])
def test_edm_gradients_match_finite_differences(q):
    rng = np.random.default_rng(320 + q)
    S, f0 = _scene(q, "channel", rng)
    F = _with_force(S, rng)
    nsteps = 6
    target = 0.02 * rng.standard_normal(S.shape + (3,))
    states = S.trajectory(f0, nsteps)
    _, u = S.moments(states[-1])
    fluid = ~S.solid.astype(bool)
    diff = (u - target) * fluid[..., None]
    L = np.sum(diff ** 2)
    seed = S.seed_from_velocity_grad(states[-1], 2 * diff)
    _, dlds, dtau, _, dldf = S.adjoint(states, seed, with_force=True)
    h = 1e-6
    D = 2 if q == 9 else 3
    cells = [tuple(c) for c in np.argwhere(fluid)[::4]]
    for cell in cells:
        for a in range(D):
            Fp, Fm = F.copy(), F.copy()
            Fp[cell + (a,)] += h
            Fm[cell + (a,)] -= h
            S.edm = Fp
            Lp = _edm_loss(S, f0, nsteps, target)
            S.edm = Fm
            Lm = _edm_loss(S, f0, nsteps, target)
            fd = (Lp - Lm) / (2 * h)
            assert abs(fd - dldf[cell + (a,)]) <= 1e-6 * max(abs(fd), 1e-3 * abs(L)), (cell, a)
    # uniform part: the sum of the per-cell gradients over fluid cells
    for a in range(D):
        S.edm = F + h * np.eye(3)[a]
        Lp = _edm_loss(S, f0, nsteps, target)
        S.edm = F - h * np.eye(3)[a]
        Lm = _edm_loss(S, f0, nsteps, target)
        fd = (Lp - Lm) / (2 * h)
        g = dldf[..., a][fluid].sum()
        assert abs(fd - g) <= 1e-6 * max(abs(fd), 1e-3 * abs(L))
    S.edm = F
    # s and tau with the force on (the force enters before the mix)
    base_s = S.s.copy()
    for cell in cells[:6]:
        S.s = base_s.copy(); S.s[cell] += h
        Lp = _edm_loss(S, f0, nsteps, target)
        S.s = base_s.copy(); S.s[cell] -= h
        Lm = _edm_loss(S, f0, nsteps, target)
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - dlds[cell]) <= 1e-6 * max(abs(fd), 1e-3 * abs(L)), cell
    S.s = base_s
    tau0 = S.tau
    S.tau = tau0 + h
    Lp = _edm_loss(S, f0, nsteps, target)
    S.tau = tau0 - h
    Lm = _edm_loss(S, f0, nsteps, target)
    S.tau = tau0
    fd = (Lp - Lm) / (2 * h)
    assert abs(fd - dtau) <= 1e-6 * abs(fd)

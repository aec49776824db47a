"""Pins of the oracle's local operators and of periodic streaming.

Equilibrium (eq. feq) moments are the exact closed forms rho, rho u and
rho (delta/3 + u u); BGK (eq. LBM-BGK) conserves rho and rho u per cell and
returns feq at tau = 1; periodic streaming (eq. streaming, Sec. 3.4) moves a
perturbation by exactly c_i, keeps uniform equilibrium a fixed point, and
conserves mass and momentum.
"""
import numpy as np
import pytest

from oracle import Face, Sim, WALL


def _rand_state(rng, q):
    rho = 1.0 + 0.05 * rng.standard_normal()
    u = 0.05 * rng.standard_normal(3)
    if q == 9:
        u[2] = 0.0
    return rho, u


@pytest.mark.parametrize("q", [9, 19, 27])
def test_equilibrium_moments(oracle_mod, q):
    rng = np.random.default_rng(10 + q)
    c, _, _ = oracle_mod.tables(q)
    c = c.astype(np.float64)
    for _ in range(20):
        rho, u = _rand_state(rng, q)
        feq = oracle_mod.equilibrium(q, rho, u)
        assert abs(feq.sum() - rho) < 1e-15
        assert np.allclose(c.T @ feq, rho * u, atol=1e-15, rtol=0)
        P = np.einsum("i,ia,ib->ab", feq, c, c)
        D = 2 if q == 9 else 3
        ref = rho * (np.eye(3) / 3.0 + np.outer(u, u))
        assert np.allclose(P[:D, :D], ref[:D, :D], atol=1e-15, rtol=0)


@pytest.mark.parametrize("q", [9, 19, 27])
def test_collision_conserves_mass_momentum(oracle_mod, q):
    rng = np.random.default_rng(20 + q)
    c, _, _ = oracle_mod.tables(q)
    c = c.astype(np.float64)
    S = Sim(q=q, nx=1, ny=1, nz=1, tau=0.63)
    for _ in range(20):
        rho, u = _rand_state(rng, q)
        f = oracle_mod.equilibrium(q, rho, u) * (1 + 0.1 * rng.standard_normal(q))
        fs = S.collide_cell(f)
        assert abs(fs.sum() - f.sum()) < 1e-15
        assert np.allclose(c.T @ fs, c.T @ f, atol=1e-15, rtol=0)


@pytest.mark.parametrize("q", [9, 19, 27])
def test_tau_one_gives_equilibrium(oracle_mod, q):
    rng = np.random.default_rng(30 + q)
    S = Sim(q=q, nx=1, ny=1, nz=1, tau=1.0)
    rho, u = _rand_state(rng, q)
    f = oracle_mod.equilibrium(q, rho, u) * (1 + 0.1 * rng.standard_normal(q))
    r, v = oracle_mod.cell_moments(f)
    assert np.allclose(S.collide_cell(f), oracle_mod.equilibrium(q, r, v), atol=1e-16, rtol=0)


@pytest.mark.parametrize("q", [9, 19, 27])
def test_uniform_equilibrium_is_fixed_point(oracle_mod, q):
    nz = 1 if q == 9 else 4
    S = Sim(q=q, nx=5, ny=4, nz=nz, tau=0.7)
    u = np.zeros((5, 4, nz, 3))
    u[..., 0] = 0.03
    u[..., 1] = -0.02
    f = S.equilibrium_state(rho=1.02, u=u)
    f0 = f.copy()
    S.run(f, 7)
    # every cell computes the same thing: the state stays bitwise uniform,
    # and equal to the start up to the rounding of the moments
    assert np.array_equal(f, np.broadcast_to(f[:1, :1, :1], f.shape))
    assert np.max(np.abs(f - f0)) < 1e-15


@pytest.mark.parametrize("q", [9, 19, 27])
def test_delta_streams_by_c(oracle_mod, q):
    """With tau so large that collision is the identity, a perturbation of
    population i at x0 arrives at x0 + c_i (periodic wrap) and nowhere else."""
    c, _, _ = oracle_mod.tables(q)
    nz = 1 if q == 9 else 3
    S = Sim(q=q, nx=4, ny=3, nz=nz, tau=1e30)
    base = S.equilibrium_state()
    x0 = (0, 2, nz - 1)
    for i in range(q):
        f = base.copy()
        f[x0 + (i,)] += 0.125
        S.run(f, 1)
        dst = tuple((np.array(x0) + c[i]) % np.array([4, 3, nz]))
        expect = base.copy()
        expect[dst + (i,)] += 0.125
        assert np.array_equal(f, expect), i


@pytest.mark.parametrize("q", [9, 19, 27])
def test_periodic_conservation(oracle_mod, q):
    rng = np.random.default_rng(40 + q)
    nz = 1 if q == 9 else 6
    S = Sim(q=q, nx=8, ny=7, nz=nz, tau=0.56)
    u = 0.05 * rng.standard_normal((8, 7, nz, 3))
    if q == 9:
        u[..., 2] = 0
    f = S.equilibrium_state(rho=1 + 0.01 * rng.standard_normal((8, 7, nz)), u=u)
    f *= 1 + 0.01 * rng.standard_normal(f.shape)
    s0 = S.sums(f)
    S.run(f, 50)
    s1 = S.sums(f)
    assert abs(s1[0] - s0[0]) / s0[0] < 1e-13
    assert np.all(np.abs(s1[1:4] - s0[1:4]) / s0[0] < 1e-13)


@pytest.mark.parametrize("q", [9, 19])
def test_rest_state_with_walls_is_fixed(oracle_mod, q):
    nz = 1 if q == 9 else 5
    faces = [Face(WALL) for _ in range(6)]
    S = Sim(q=q, nx=5, ny=6, nz=nz, tau=0.55, faces=faces)
    f = S.equilibrium_state()
    f0 = f.copy()
    S.run(f, 20)
    # bounce-back of a uniform rest state is the same value: all cells stay
    # bitwise equal; the weights sum to 1 only up to one rounding
    assert np.array_equal(f, np.broadcast_to(f[:1, :1, :1], f.shape))
    assert np.max(np.abs(f - f0)) <= 4.5e-16


def test_partial_bounce_back_zero_is_bgk(oracle_mod):
    rng = np.random.default_rng(50)
    u = 0.04 * rng.standard_normal((9, 7, 1, 3))
    u[..., 2] = 0
    A = Sim(q=9, nx=9, ny=7, tau=0.6)
    B = Sim(q=9, nx=9, ny=7, tau=0.6, s=np.zeros((9, 7, 1)))
    fa = A.equilibrium_state(u=u)
    fb = fa.copy()
    A.run(fa, 10)
    B.run(fb, 10)
    assert np.array_equal(fa, fb)


def test_partial_bounce_back_one_reverses_momentum(oracle_mod):
    """s = 1 everywhere reflects every population in place, so the total
    momentum flips sign each step and mass is kept: no net flow."""
    rng = np.random.default_rng(51)
    u = 0.04 * rng.standard_normal((6, 5, 1, 3))
    u[..., 2] = 0
    S = Sim(q=9, nx=6, ny=5, tau=0.7, s=np.ones((6, 5, 1)))
    f = S.equilibrium_state(u=u)
    p0 = S.sums(f)
    for k in range(1, 5):
        S.run(f, 1)
        p = S.sums(f)
        assert abs(p[0] - p0[0]) < 1e-13
        assert np.allclose(p[1:3], ((-1) ** k) * p0[1:3], atol=1e-15)

"""Pins of the oracle's KBC collision (D2Q9, D3Q27).

* Mass and momentum are conserved by the collision (a one-cell periodic box,
  where a step is one collision).
* At tau = 1 (beta = 1/2) the entropic gamma is 2 for every state: KBC is BGK.
* gamma minimizes the quadratic entropy <f* - feq|f* - feq> (weights 1/feq):
  the KBC result is orthogonal, in that product, to its difference from BGK.
* The deviatoric momentum flux relaxes exactly as in BGK, by (1 - 1/tau), so
  the shear viscosity is BGK's; a Taylor-Green vortex decays at BGK's rate.
* Stability: a 64^2 lid-driven cavity at tau = 0.502 (Re ~ 4800) stays bounded
  with KBC where BGK diverges.
"""
import numpy as np
import pytest

from oracle import BGK, KBC, Face, Sim, WALL, equilibrium, tables


def _collide(q, f0, tau, collision):
    S = Sim(q=q, nx=1, ny=1, nz=1, tau=tau, collision=collision)
    f = f0.reshape(1, 1, 1, q).copy()
    S.run(f, 1)
    return f.reshape(q)


def _state(q, rng):
    u = 0.05 * rng.standard_normal(3)
    if q == 9:
        u[2] = 0.0
    rho = 1.0 + 0.05 * rng.random()
    feq = equilibrium(q, rho, u)
    return feq * (1 + 0.08 * rng.standard_normal(q)), rho, u


@pytest.mark.parametrize("q", [9, 27])
def test_kbc_conserves_mass_and_momentum(q):
    rng = np.random.default_rng(700 + q)
    c, _, _ = tables(q)
    c = c.astype(np.float64)
    for tau in (0.51, 0.6, 0.9, 1.7):
        f, _, _ = _state(q, rng)
        g = _collide(q, f, tau, KBC)
        assert abs(g.sum() - f.sum()) < 1e-15
        assert np.max(np.abs(g @ c - f @ c)) < 1e-15


@pytest.mark.parametrize("q", [9, 27])
def test_kbc_is_bgk_at_tau_one(q):
    rng = np.random.default_rng(710 + q)
    for _ in range(5):
        f, _, _ = _state(q, rng)
        assert np.max(np.abs(_collide(q, f, 1.0, KBC) - _collide(q, f, 1.0, BGK))) < 1e-15


@pytest.mark.parametrize("q", [9, 27])
def test_kbc_gamma_minimizes_the_quadratic_entropy(q):
    rng = np.random.default_rng(720 + q)
    c, _, _ = tables(q)
    c = c.astype(np.float64)
    for tau in (0.52, 0.7, 1.3):
        f, _, _ = _state(q, rng)
        rho = f.sum()
        feq = equilibrium(q, rho, (f @ c) / rho)
        k = _collide(q, f, tau, KBC)
        b = _collide(q, f, tau, BGK)
        d = k - b
        assert np.linalg.norm(d) > 1e-6            # the entropic step is not BGK here
        assert abs(np.sum((k - feq) * d / feq)) < 1e-14 * np.sum(d * d / feq) ** 0.5 * 1e2


@pytest.mark.parametrize("q", [9, 27])
def test_kbc_relaxes_the_deviatoric_stress_like_bgk(q):
    rng = np.random.default_rng(730 + q)
    c, _, _ = tables(q)
    c = c.astype(np.float64)
    D = 2 if q == 9 else 3

    def dev(P):
        P = P[:D, :D]
        return P - np.trace(P) / D * np.eye(D)

    for tau in (0.55, 0.8):
        f, _, _ = _state(q, rng)
        rho = f.sum()
        feq = equilibrium(q, rho, (f @ c) / rho)
        g = _collide(q, f, tau, KBC)
        Pn = (c * (f - feq)[:, None]).T @ c
        Pg = (c * (g - feq)[:, None]).T @ c
        assert np.max(np.abs(dev(Pg) - (1 - 1 / tau) * dev(Pn))) < 1e-15


def _tgv_ke(collision, steps):
    n = 64
    k = 2 * np.pi / n
    x = np.arange(n)[:, None]
    y = np.arange(n)[None, :]
    u = np.zeros((n, n, 1, 3))
    u[..., 0] = (0.01 * np.sin(k * x) * np.cos(k * y))[..., None]
    u[..., 1] = (-0.01 * np.cos(k * x) * np.sin(k * y))[..., None]
    S = Sim(q=9, nx=n, ny=n, nz=1, tau=0.6, collision=collision)
    f = S.equilibrium_state(u=u)
    S.run(f, steps)
    rho, v = S.moments(f)
    return float(np.sum(rho * (v ** 2).sum(-1)))


def test_kbc_taylor_green_decays_at_the_bgk_rate():
    k0 = _tgv_ke(KBC, 0)
    kk = _tgv_ke(KBC, 400)
    kb = _tgv_ke(BGK, 400)
    rate_k = -np.log(kk / k0) / 400
    rate_b = -np.log(kb / k0) / 400
    assert abs(rate_k - rate_b) < 1e-3 * rate_b


def test_kbc_stays_bounded_where_bgk_diverges():
    faces = [Face(WALL)] * 3 + [Face(WALL, (0.05, 0, 0))] + [Face(), Face()]
    out = {}
    for col in (BGK, KBC):
        S = Sim(q=9, nx=64, ny=64, nz=1, tau=0.502, faces=faces, collision=col)
        f = S.equilibrium_state()
        S.run(f, 3000)
        _, u = S.moments(f)
        out[col] = float(np.max(np.abs(u))) if np.all(np.isfinite(u)) else np.inf
    assert out[BGK] > 1.0 or not np.isfinite(out[BGK])
    assert out[KBC] < 0.06

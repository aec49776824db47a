"""GPU body force by the exact-difference method (lbm_set_force) against the
FP64 oracle (pinned in test_oracle_edm.py): uniform and per-cell forces with
walls, solids, Zou-He / outflow faces, the partial bounce-back field and both
step patterns; the exact momentum growth on the GPU itself; a field updated
between steps; graphs; errors."""
import sys

import numpy as np
import pytest

from cases import Case, _oface, compare, fluid_mask, gpu_sim
from paper_2311_16080_amd import inputs, lbm

pytestmark = pytest.mark.gpu
W, P, ZV, ZP, OUT = lbm.WALL, lbm.PERIODIC, lbm.ZOUHE_VELOCITY, lbm.ZOUHE_PRESSURE, lbm.EQ_OUTFLOW
TOL = {"f64": (1e-12, 1e-13), "f32": (1e-5, 1e-6), "f16": (1e-3, 1e-4), "bf16": (3e-2, 3e-3)}


def _announce(name):
    print(f"\n[case] {name}", flush=True)
    sys.stdout.flush()


def _cube(shape, lo, hi):
    s = np.zeros(shape, np.uint8)
    s[tuple(slice(a, b) for a, b in zip(lo, hi))] = 1
    return s


def _field(case, seed, amp=2e-4):
    """Seeded force field (*shape, D) and a uniform part (D,)."""
    fld = inputs.random_velocity(case.shape, case.D, seed, amp=amp)
    uni = amp * np.array([0.5, -0.3, 0.2])[: case.D]
    return fld, uni


CASES = {
    "d2q9_channel_walls": (Case(9, (48, 40), 0.7, [(P,), (P,), (W,), (W, (0.02, 0.0)), (P,), (P,)], init_seed=201), 1.0),
    "d3q19_walls_spheres": (Case(19, (12, 10, 70), 0.65, [(W,), (W,), (W,), (W, (0.03, 0, 0.01)), (P,), (P,)],
                                 init_seed=202, solid=inputs.sphere_obstacles(12, 10, 70, seed=5, rmin=1.5, rmax=3,
                                                                              xlo=3, xhi=9, fraction=0.05)), 1.0),
    "d3q27_zouhe_outflow_cube": (Case(27, (20, 9, 66), 0.6, [(ZV, (0.03, 0, 0)), (OUT, (0, 0, 0), 1.0), (W,), (W,),
                                                             (P,), (P,)], init_seed=203,
                                      solid=_cube((20, 9, 66), (8, 3, 20), (11, 6, 40))), 0.5),
    "d3q19_pressure_faces": (Case(19, (18, 8, 64), 0.8, [(ZP, (0, 0, 0), 1.01), (ZP, (0, 0, 0), 0.99), (W,), (W,),
                                                         (P,), (P,)], init_seed=204), 2.0),
}


def _oracle(case, fld, uni, eps, steps):
    import oracle
    e = np.zeros(case.oshape + (3,))
    e[..., : case.D] = eps * (fld.reshape(case.oshape + (case.D,)) + uni)
    faces = [_oface(F) for F in case.faces]
    if case.q == 9:
        faces[4] = faces[5] = oracle.Face()
    sol = None if case.solid is None else case.solid.reshape(case.oshape).astype(np.uint8)
    sv = None if case.s is None else case.s.reshape(case.oshape).astype(np.float32).astype(np.float64)
    S = oracle.Sim(q=case.q, nx=case.oshape[0], ny=case.oshape[1], nz=case.oshape[2], tau=case.tau, faces=faces,
                   solid=sol, s=sv, edm=e)
    rho, u = case.init_fields()
    f = S.equilibrium_state(rho=rho.reshape(case.oshape), u=u.reshape(case.oshape + (case.D,)))
    S.run(f, steps)
    r, v = S.moments(f)
    return r, v, S, f


def _gpu(case, fld, uni, eps, steps):
    import torch
    sim = gpu_sim(case)
    ft = torch.tensor(np.moveaxis(fld, -1, 0).copy(), dtype=torch.float64, device="cuda")
    sim.set_force(uni, ft, eps)
    sim.step(steps)
    return sim, _moments(sim, case)


def _moments(sim, case):
    import torch
    rho, u = sim.moments(dtype=torch.float64)
    torch.cuda.synchronize()
    r = rho.cpu().numpy().reshape(case.oshape)
    v = np.zeros(case.oshape + (3,))
    uu = u.cpu().numpy()
    for a in range(case.D):
        v[..., a] = uu[a].reshape(case.oshape)
    return r, v


def _field_as_stored(fld, storage):
    # the library converts the field to the compute type: give the oracle the same values
    return fld if storage == "f64" else fld.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("storage", ["f64", "f32", "f16", "bf16"])
def test_force_matches_oracle(name, storage):
    base, eps = CASES[name]
    utol, rtol = TOL[storage]
    for steps in (20, 21):
        case = Case(base.q, base.shape, base.tau, base.faces, steps=steps, storage=storage,
                    init_seed=base.init_seed, solid=base.solid)
        fld, uni = _field(case, 300 + steps)
        _announce(f"edm {name} {storage} steps={steps}")
        sim, g = _gpu(case, fld, uni, eps, steps)
        o = _oracle(case, _field_as_stored(fld, storage), uni, eps, steps)
        eu, er = compare(case, g, o)
        print(f"[case] {name} {storage} steps={steps}: u rel-L2 {eu:.3e}, max|drho| {er:.3e}", flush=True)
        assert eu < utol and er < rtol


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_force_with_solid_fraction_and_double_buffer(storage):
    """Partial bounce-back field (the force goes in before the mix) and the
    double-buffer patterns (push and pull: their own step kernels)."""
    rng = np.random.default_rng(7)
    shape = (10, 12, 66)
    s = (rng.random(shape) * (rng.random(shape) < 0.3)).astype(np.float64)
    utol, rtol = TOL[storage]
    for pattern in ("inplace", "double", "pull"):
        case = Case(19, shape, 0.7, [(W,), (W, (0, 0.02, 0)), (P,), (P,), (P,), (P,)], steps=15, storage=storage,
                    pattern=pattern, init_seed=210, s=s)
        fld, uni = _field(case, 310)
        _announce(f"edm pbb {pattern} {storage}")
        sim, g = _gpu(case, fld, uni, 1.0, case.steps)
        o = _oracle(case, _field_as_stored(fld, storage), uni, 1.0, case.steps)
        eu, er = compare(case, g, o)
        print(f"[case] pbb {pattern} {storage}: u rel-L2 {eu:.3e}, max|drho| {er:.3e}", flush=True)
        assert eu < utol and er < rtol


def test_uniform_force_momentum_growth_on_gpu():
    """Periodic box, FP64: each step adds exactly N F of momentum."""
    _announce("edm momentum growth")
    case = Case(19, (16, 12, 64), 0.6, [(P,)] * 6, storage="f64", init_seed=220)
    sim = gpu_sim(case)
    F = np.array([3e-5, -1e-5, 2e-5])
    sim.set_force(F)
    N = np.prod(case.shape)
    for _ in range(4):
        s0 = sim.sums()
        sim.step(1)
        s1 = sim.sums()
        assert abs(s1[0] - s0[0]) < 1e-13 * s0[0]
        assert np.max(np.abs((s1[1:4] - s0[1:4]) - N * F)) < 1e-12 * N * np.abs(F).max()


def test_field_update_between_steps():
    """The library reads the field at every step: an in-place update between
    steps is seen by the next step (oracle: two segments with two fields)."""
    import oracle
    import torch
    _announce("edm field update")
    case = Case(9, (40, 36), 0.75, [(P,), (P,), (W,), (W,), (P,), (P,)], storage="f64", init_seed=230)
    f1, _ = _field(case, 331)
    f2, _ = _field(case, 332)
    sim = gpu_sim(case)
    ft = torch.tensor(np.moveaxis(f1, -1, 0).copy(), dtype=torch.float64, device="cuda")
    sim.set_force(None, ft)
    sim.step(5)
    sim._force_field.copy_(torch.tensor(np.moveaxis(f2, -1, 0).copy(), dtype=torch.float64, device="cuda"))
    sim.step(6)
    g = _moments(sim, case)
    _, _, S1, f = _oracle(case, f1, np.zeros(2), 1.0, 5)
    e2 = np.zeros(case.oshape + (3,))
    e2[..., :2] = f2.reshape(case.oshape + (2,))
    faces = [_oface(F) for F in case.faces]
    faces[4] = faces[5] = oracle.Face()
    S2 = oracle.Sim(q=9, nx=case.oshape[0], ny=case.oshape[1], nz=1, tau=case.tau, faces=faces, edm=e2)
    S2.run(f, 6)
    r, v = S2.moments(f)
    eu, er = compare(case, g, (r, v))
    assert eu < 1e-12 and er < 1e-13


def test_force_off_and_graph():
    """set_force() switches the force off (bitwise the force-free run); a
    graph captured with the force replays the eager steps bitwise; setting
    the force drops a captured graph."""
    import torch
    _announce("edm off / graph")
    case = Case(19, (8, 10, 64), 0.7, [(W,), (W, (0, 0.02, 0)), (P,), (P,), (P,), (P,)], storage="f32",
                init_seed=240)
    a = gpu_sim(case)
    b = gpu_sim(case)
    b.set_force([1e-4, 0, 0])
    b.set_force()
    a.step(7)
    b.step(7)
    ra, ua = a.moments()
    rb, ub = b.moments()
    assert torch.equal(ra, rb) and torch.equal(ua, ub)

    fld, uni = _field(case, 341)
    ft = torch.tensor(np.moveaxis(fld, -1, 0).copy(), dtype=torch.float32, device="cuda")
    e = gpu_sim(case)
    gsim = gpu_sim(case)
    for s in (e, gsim):
        s.set_force(uni, ft)
    e.step(6)
    gsim.capture_graph(2)
    for _ in range(3):
        gsim.graph_launch()
    torch.cuda.synchronize()
    re, ue = e.moments()
    rg, ug = gsim.moments()
    assert torch.equal(re, rg) and torch.equal(ue, ug)
    gsim.set_force()
    with pytest.raises(lbm.LbmError):
        gsim.graph_launch()


def test_force_errors():
    import torch
    _announce("edm errors")
    sim = gpu_sim(Case(19, (6, 7, 64), 0.6, [(W,)] * 6, storage="f32"))
    with pytest.raises(lbm.LbmError):
        sim.set_force([float("nan"), 0, 0])
    with pytest.raises(lbm.LbmError):
        sim.set_force([1e-4, 0, 0], eps=float("inf"))
    bs = lbm.BatchSim("D2Q9", [(8, 8)], [0.7], [[(W,), (W,), (W,), (W, (0.05, 0.0)), (P,), (P,)]])
    f = (lbm.ctypes.c_double * 3)(1e-4, 0, 0)
    assert lbm.lib().lbm_set_force(bs.h, f, None, 1.0) == lbm.LBM_EUNSUPPORTED
    bs.init_equilibrium()
    bs.tape_begin(2, 4)
    bs.step(2)
    bs.tape_end()
    out = (lbm.ctypes.c_double * 3)()
    assert lbm.lib().lbm_backward_force(bs.h, None, None, lbm.F32, None, None, None, None, out) == \
        lbm.LBM_EUNSUPPORTED


# ---- adjoint of the body force ---------------------------------------------------------
def _adj_case(name, storage):
    if name == "d2q9_channel_pbb":
        c = Case(9, (40, 24), 0.6, [(ZV, (0.04, 0.0)), (OUT, (0, 0, 0), 1.0), (W,), (W, (0.03, 0.0)), (P,), (P,)],
                 steps=16, storage=storage, init_seed=250,
                 s=inputs.smooth_solid_fraction(40, 24, seed=4, sigma=3, edge=4))
        return c, 5, 0.5
    c = Case(19, (10, 12, 64), 0.7, [(W,), (W, (0.0, 0.02, 0.01)), (W,), (W,), (P,), (P,)], steps=12,
             storage=storage, init_seed=251,
             solid=inputs.sphere_obstacles(10, 12, 64, seed=8, rmin=1.5, rmax=3, xlo=3, xhi=7, fraction=0.04))
    return c, 4, 1.0


def _oracle_force_grads(case, fld, uni, eps, target):
    import oracle
    e = np.zeros(case.oshape + (3,))
    e[..., : case.D] = eps * (fld.reshape(case.oshape + (case.D,)) + uni)
    faces = [_oface(F) for F in case.faces]
    if case.q == 9:
        faces[4] = faces[5] = oracle.Face()
    sol = None if case.solid is None else case.solid.reshape(case.oshape).astype(np.uint8)
    sv = None if case.s is None else case.s.reshape(case.oshape).astype(np.float32).astype(np.float64)
    S = oracle.Sim(q=case.q, nx=case.oshape[0], ny=case.oshape[1], nz=case.oshape[2], tau=case.tau, faces=faces,
                   solid=sol, s=sv, edm=e)
    rho, u = case.init_fields()
    f = S.equilibrium_state(rho=rho.reshape(case.oshape), u=u.reshape(case.oshape + (case.D,)))
    states = S.trajectory(f, case.steps)
    _, uf = S.moments(states[-1])
    m = fluid_mask(case)[..., None]
    seed = S.seed_from_velocity_grad(states[-1], 2.0 * (uf[..., : case.D] - target) * m)
    _, dlds, dtau, duw, dldf = S.adjoint(states, seed, with_force=True)
    dfield = eps * dldf[..., : case.D]
    dforce = dfield[fluid_mask(case)].sum(0)
    return dlds, dtau, duw, dfield, dforce


@pytest.mark.parametrize("name", ["d2q9_channel_pbb", "d3q19_zperiodic_spheres"])
@pytest.mark.parametrize("storage,tol", [("f64", 1e-10), ("f32", 1e-4)])
def test_force_adjoint_matches_oracle(name, storage, tol):
    import torch
    case, K, eps = _adj_case(name, storage)
    _announce(f"edm adjoint {name} {storage}")
    fld, uni = _field(case, 350, amp=1e-3)
    fld_s = _field_as_stored(fld, storage)
    target = inputs.random_velocity(case.oshape, case.D, 71, amp=0.02)
    sim = gpu_sim(case)
    ft = torch.tensor(np.moveaxis(fld, -1, 0).copy(), dtype=torch.float64, device="cuda")
    sim.set_force(uni, ft, eps)
    sim.tape_begin(K, case.steps)
    sim.step(case.steps)
    sim.tape_end()
    dt = torch.float64 if storage == "f64" else torch.float32
    rho, u = sim.moments(dtype=dt)
    m = torch.tensor(fluid_mask(case).reshape(case.shape), device="cuda")
    tgt = torch.tensor(np.moveaxis(target[..., : case.D].reshape(case.shape + (case.D,)), -1, 0).copy(),
                       dtype=dt, device="cuda")
    ds, dtau, duw, dfield, dforce = sim.backward_force(None, 2.0 * (u - tgt) * m, want_s=case.s is not None)
    o_ds, o_dtau, o_duw, o_dfield, o_dforce = _oracle_force_grads(case, fld_s, uni, eps, target[..., : case.D])
    g = np.moveaxis(dfield.double().cpu().numpy(), 0, -1).reshape(case.oshape + (case.D,))
    fm = fluid_mask(case)
    e_field = np.linalg.norm((g - o_dfield)[fm]) / np.linalg.norm(o_dfield[fm])
    e_force = np.max(np.abs(dforce - o_dforce)) / np.max(np.abs(o_dforce))
    print(f"[case] {name} {storage}: dL/dfield rel-L2 {e_field:.3e}, dL/dforce rel {e_force:.3e}, "
          f"dtau {dtau[0]:.6e} vs {o_dtau:.6e}", flush=True)
    assert e_field <= tol and e_force <= tol
    assert abs(dtau[0] - o_dtau) <= tol * abs(o_dtau)
    nz = np.abs(o_duw) > 0
    if np.any(nz):
        assert np.linalg.norm(duw[0][nz] - o_duw[nz]) <= tol * np.linalg.norm(o_duw[nz])
    if case.s is not None:
        d = ds.double().cpu().numpy().reshape(case.oshape)
        assert np.linalg.norm((d - o_ds)[fm]) <= max(tol, 1e-7) * np.linalg.norm(o_ds[fm])
    # lbm_backward with the force on gives the same tau gradient
    _, dtau2, _ = sim.backward(None, 2.0 * (u - tgt) * m)
    assert abs(dtau2[0] - dtau[0]) <= 1e-12 * abs(dtau[0])


def test_force_autograd_matches_finite_differences():
    """torch.autograd through lbm.rollout with a force field: field.grad against
    central differences of the GPU forward itself (FP64)."""
    import torch
    _announce("edm autograd FD")
    shape = (24, 20)
    faces = [(P,), (P,), (W,), (W, (0.03, 0.0)), (P,), (P,)]
    sim = lbm.Sim("D2Q9", shape, 0.7, faces=faces, storage="f64")
    rho0 = torch.tensor(inputs.random_density(shape, 80, amp=0.01), device="cuda")
    u0 = torch.tensor(np.moveaxis(inputs.random_velocity(shape, 2, 81, amp=0.03), -1, 0).copy(), device="cuda")
    target = torch.tensor(np.moveaxis(inputs.random_velocity(shape, 2, 82, amp=0.02), -1, 0).copy(), device="cuda")
    field = torch.tensor(np.moveaxis(inputs.random_velocity(shape, 2, 83, amp=1e-3), -1, 0).copy(), device="cuda",
                         requires_grad=True)

    def loss_of(fl):
        _, u = lbm.rollout(sim, 10, 4, rho0=rho0, u0=u0, field=fl, eps=0.5)
        return torch.sum((u - target) ** 2)

    L = loss_of(field)
    L.backward()
    g = field.grad.detach().cpu().numpy()
    h = 1e-6
    for idx in [(0, 3, 4), (1, 10, 0), (0, 23, 19), (1, 12, 9)]:
        fp = field.detach().clone()
        fp[idx] += h
        fm = field.detach().clone()
        fm[idx] -= h
        with torch.no_grad():
            fd = (float(loss_of(fp)) - float(loss_of(fm))) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-6 * max(abs(fd), 1e-6 * float(L)), idx

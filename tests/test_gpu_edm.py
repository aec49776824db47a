"""GPU body force by the exact-difference method (lbm_set_force) against the
FP64 oracle (pinned in test_oracle_edm.py): uniform and per-cell forces with
walls, solids, Zou-He / outflow faces, the partial bounce-back field and both
step patterns; the exact momentum growth on the GPU itself; a field updated
between steps; graphs; errors."""
import sys

import numpy as np
import pytest

from cases import Case, _oface, compare, gpu_sim
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
    double-buffer pattern (its own step kernel)."""
    rng = np.random.default_rng(7)
    shape = (10, 12, 66)
    s = (rng.random(shape) * (rng.random(shape) < 0.3)).astype(np.float64)
    utol, rtol = TOL[storage]
    for pattern in ("inplace", "double"):
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
    sim.set_force([1e-4, 0, 0])
    sim.tape_begin(2, 4)
    sim.step(2)
    sim.tape_end()
    rho_bar = torch.zeros((6, 7, 64), dtype=torch.float32, device="cuda")
    with pytest.raises(lbm.LbmError) as ei:
        sim.backward(rho_bar, None)
    assert ei.value.code == lbm.LBM_EUNSUPPORTED
    bs = lbm.BatchSim("D2Q9", [(8, 8)], [0.7], [[(W,), (W,), (W,), (W, (0.05, 0.0)), (P,), (P,)]])
    f = (lbm.ctypes.c_double * 3)(1e-4, 0, 0)
    assert lbm.lib().lbm_set_force(bs.h, f, None, 1.0) == lbm.LBM_EUNSUPPORTED

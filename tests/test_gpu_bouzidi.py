"""GPU interpolated bounce-back on curved walls (lbm_set_curved_links) against
the FP64 oracle, element by element on the same seeded inputs: a cylinder in
a D2Q9 channel (the paper's flow past a cylinder, Sec. 4.3) and random
spheres in D3Q19 / D3Q27 channels, both interpolation orders, every storage,
both streaming patterns, odd and even step counts; the momentum-exchange
force of Mei et al. over the curved links against the oracle's step force;
the halfway fraction bit for bit against plain bounce-back; graph replay;
argument checks.

Tolerances as in test_gpu_parity.py (rel-L2 of u; max |rho - rho_oracle|):
FP64 1e-12 / 1e-13, FP32 1e-5 / 1e-6, FP16 1e-3 / 1e-4.  Forces: FP64 1e-11,
FP32 1e-4 relative to the largest force component."""
import sys

import numpy as np
import pytest

from cases import Case, compare, gpu_run, gpu_sim, oracle_run
from paper_2311_16080_amd import inputs, lbm

pytestmark = pytest.mark.gpu

W, P, ZV, OUT = lbm.WALL, lbm.PERIODIC, lbm.ZOUHE_VELOCITY, lbm.EQ_OUTFLOW
TOL = {"f64": (1e-12, 1e-13), "f32": (1e-5, 1e-6), "f16": (1e-3, 1e-4)}


def _announce(name):
    print(f"\n[case] {name}", flush=True)
    sys.stdout.flush()


def cylinder_case(storage="f64", order=1, steps=25, pattern="inplace", shape=(70, 36)):
    nx, ny = shape
    cx, cy, r = 20.3, 17.6, 5.7
    solid = inputs.cylinder_obstacle(nx, ny, cx, cy, r)
    c, _ = lbm.lattice_info("D2Q9")
    links = inputs.ball_wall_fractions(solid, np.array([[cx, cy, r]]), c[:, :2])
    faces = [(ZV, (0.04, 0.0)), (OUT, (0, 0, 0), 1.0), (W,), (W,), (P,), (P,)]
    return Case(9, shape, 0.6, faces, steps=steps, storage=storage, pattern=pattern, solid=solid, init_seed=31,
                links=links, bz_order=order)


def spheres_case(q, storage="f64", order=1, steps=20, pattern="inplace", shape=(30, 14, 70)):
    solid, balls = inputs.sphere_obstacles(*shape, seed=8, rmin=2.2, rmax=4.6, xlo=6, xhi=shape[0] - 6,
                                           fraction=0.06, return_spheres=True)
    c, _ = lbm.lattice_info("D3Q19" if q == 19 else "D3Q27")
    links = inputs.ball_wall_fractions(solid, balls, c)
    faces = [(ZV, (0.03, 0.0, 0.0)), (OUT, (0, 0, 0), 1.0), (W,), (W,), (P,), (P,)]
    return Case(q, shape, 0.6, faces, steps=steps, storage=storage, pattern=pattern, solid=solid, init_seed=32,
                links=links, bz_order=order)


CASES = {}
for _order in (1, 2):
    for _st in ("f64", "f32", "f16"):
        CASES[f"cylinder_d2q9_{_st}_o{_order}"] = ("cyl", dict(storage=_st, order=_order))
    CASES[f"cylinder_d2q9_f64_o{_order}_even"] = ("cyl", dict(order=_order, steps=26))
    CASES[f"cylinder_d2q9_f64_o{_order}_double"] = ("cyl", dict(order=_order, pattern="double"))
    for _q in (19, 27):
        CASES[f"spheres_d3q{_q}_f64_o{_order}"] = ("sph", dict(q=_q, order=_order))
        CASES[f"spheres_d3q{_q}_f32_o{_order}"] = ("sph", dict(q=_q, storage="f32", order=_order, steps=21))
CASES["spheres_d3q19_f64_o2_double"] = ("sph", dict(q=19, order=2, pattern="double", steps=17))
CASES["spheres_d3q19_f64_o2_pull"] = ("sph", dict(q=19, order=2, pattern="pull", steps=17))
CASES["cylinder_d2q9_f64_o1_pull"] = ("cyl", dict(order=1, pattern="pull"))
CASES["spheres_d3q27_f16_o1_pull"] = ("sph", dict(q=27, storage="f16", order=1, pattern="pull"))
CASES["spheres_d3q27_f16_o1"] = ("sph", dict(q=27, storage="f16", order=1))


def _make(name):
    kind, kw = CASES[name]
    return cylinder_case(**kw) if kind == "cyl" else spheres_case(**kw)


@pytest.mark.parametrize("name", sorted(CASES))
def test_curved_walls_match_oracle(name):
    case = _make(name)
    _announce(f"{name}: {case.links[0].size} links")
    g = gpu_run(case)
    o = oracle_run(case)
    du, drho = compare(case, g, o)
    tol_u, tol_rho = TOL[case.storage]
    print(f"[case] {name}: u rel-L2 {du:.3e} (tol {tol_u:g}), max|drho| {drho:.3e}", flush=True)
    assert np.all(np.isfinite(g[1]))
    assert du <= tol_u and drho <= tol_rho


@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("kind", ["cyl", "sph"])
def test_half_fraction_is_plain_bounce_back_bitwise(kind, order):
    _announce(f"q = 1/2 links == halfway bounce-back ({kind}, order {order})")
    case = cylinder_case(order=order, storage="f32") if kind == "cyl" else spheres_case(19, "f32", order)
    cells, dirs, _ = case.links
    half = Case(**{**case.__dict__, "links": (cells, dirs, np.full(cells.size, 0.5))})
    plain = Case(**{**case.__dict__, "links": None})
    for steps in (6, 7):
        a = gpu_run(half, steps)
        b = gpu_run(plain, steps)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), steps
        del a, b


@pytest.mark.parametrize("storage,tol", [("f64", 1e-11), ("f32", 1e-4)])
@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("kind", ["cyl", "sph27"])
@pytest.mark.parametrize("steps", [12, 13])
def test_link_forces_match_oracle(kind, order, storage, tol, steps):
    """lbm_forces after `steps` steps vs the oracle's momentum exchange of the
    same (last) step, from its post-collision and new populations."""
    _announce(f"curved-link forces {kind} order {order} {storage} after {steps} steps")
    case = cylinder_case(storage, order) if kind == "cyl" else spheres_case(27, storage, order)
    sim = gpu_sim(case)
    sim.step(steps)
    Fs, Ff = sim.forces()
    _, _, _, S, f = oracle_run(case, steps - 1)
    Os, Of = S.step_forces(f)
    D = case.D
    scale = max(np.max(np.abs(Os[:D])), np.max(np.abs(Of[:, :D])))
    print(f"[case] solids {Fs[:D]} vs {Os[:D]}", flush=True)
    assert np.max(np.abs(Fs[:D] - Os[:D])) <= tol * scale
    assert np.max(np.abs(Ff[:, :D] - Of[:, :D])) <= tol * scale


def test_graph_replay_with_curved_links_is_bitwise():
    import torch
    _announce("graph replay with curved links")
    case = cylinder_case("f32", 2)
    a = gpu_sim(case)
    b = gpu_sim(case)
    a.step(4)
    b.step(4)
    b.capture_graph(10)
    for _ in range(3):
        a.step(10)
        b.graph_launch()
        torch.cuda.synchronize()
        ra, ua = a.moments(dtype=torch.float64)
        rb, ub = b.moments(dtype=torch.float64)
        assert torch.equal(ra, rb) and torch.equal(ua, ub)


def test_link_argument_checks():
    _announce("curved link argument checks")
    case = cylinder_case("f32", 1)
    sim = gpu_sim(case)
    cells, dirs, q = case.links
    L = lbm.lib()

    def call(c, d, qq, order=1, n=None):
        c = np.ascontiguousarray(np.asarray(c, np.int64))
        d = np.ascontiguousarray(np.asarray(d, np.int32))
        qq = np.ascontiguousarray(np.asarray(qq, np.float64))
        import ctypes
        P = ctypes.POINTER
        return L.lbm_set_curved_links(sim.h, c.size if n is None else n, c.ctypes.data_as(P(ctypes.c_int64)),
                                      d.ctypes.data_as(P(ctypes.c_int32)), qq.ctypes.data_as(P(ctypes.c_double)),
                                      order)

    solid_cell = int(np.flatnonzero(case.solid.reshape(-1))[0])
    assert call([solid_cell], [1], [0.3]) == lbm.LBM_EINVAL
    assert call([0], [1], [0.3]) == lbm.LBM_EINVAL                     # neighbour is fluid
    assert call(cells[:1], dirs[:1], [0.0]) == lbm.LBM_EINVAL
    assert call(cells[:1], dirs[:1], [1.5]) == lbm.LBM_EINVAL
    assert call(cells[:1], dirs[:1], q[:1], order=3) == lbm.LBM_EINVAL
    assert call(np.r_[cells[:1], cells[:1]], np.r_[dirs[:1], dirs[:1]], np.r_[q[:1], q[:1]]) == lbm.LBM_EINVAL
    assert call(cells[:1], [12], q[:1]) == lbm.LBM_EINVAL                # no such direction
    assert call(cells, dirs, q) == lbm.LBM_OK
    # the adjoint refuses curved links
    import torch
    sim.init_equilibrium()
    sim.tape_begin(2, 4)
    sim.step(4)
    sim.tape_end()
    with pytest.raises(lbm.LbmError) as err:
        sim.backward(None, torch.zeros((2,) + case.shape, device="cuda"))
    assert err.value.code == lbm.LBM_EUNSUPPORTED
    # no solid cells: refused
    free = lbm.Sim("D2Q9", case.shape, 0.6, faces=case.faces, storage="f32")
    free.init_equilibrium()
    with pytest.raises(lbm.LbmError):
        free.set_curved_links(cells[:1], dirs[:1], q[:1])

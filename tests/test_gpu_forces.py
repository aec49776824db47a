"""GPU momentum-exchange forces (lbm_forces) against the FP64 oracle's
orc_forces after the same steps, for both AA parities, closed and open
domains; plus the exact momentum balance on the GPU itself.  The oracle's
forces are pinned in test_oracle_forces.py (momentum balance, Couette)."""
import sys

import numpy as np
import pytest

from cases import Case, _oface, gpu_sim
from paper_2311_16080_amd import inputs, lbm

pytestmark = pytest.mark.gpu
W, P, ZV, ZP, OUT = lbm.WALL, lbm.PERIODIC, lbm.ZOUHE_VELOCITY, lbm.ZOUHE_PRESSURE, lbm.EQ_OUTFLOW


def _announce(name):
    print(f"\n[case] {name}", flush=True)
    sys.stdout.flush()


def _cube(shape, lo, hi):
    s = np.zeros(shape, np.uint8)
    s[tuple(slice(a, b) for a, b in zip(lo, hi))] = 1
    return s


CASES = {
    "d3q19_walls_spheres": Case(19, (10, 9, 70), 0.7, [(W,), (W, (0, 0.02, 0.01)), (W,), (W,), (W,),
                                                       (W, (0.05, 0.01, 0))], init_seed=101,
                                solid=inputs.sphere_obstacles(10, 9, 70, seed=3, rmin=1.5, rmax=3, xlo=3, xhi=7,
                                                              fraction=0.05)),
    "d3q27_lid_cube": Case(27, (8, 8, 66), 0.6, [(W,)] * 5 + [(W, (0.04, 0, 0))], init_seed=102,
                           solid=_cube((8, 8, 66), (3, 3, 20), (5, 6, 30))),
    "d2q9_periodic_x_plate": Case(9, (24, 80), 0.8, [(P,), (P,), (W,), (W, (0.03, 0.0)), (P,), (P,)], init_seed=103,
                                  solid=_cube((24, 80), (10, 30), (12, 50))),
    "d3q19_channel_open_faces": Case(19, (20, 8, 66), 0.65, [(ZV, (0.03, 0, 0)), (OUT, (0, 0, 0), 1.0), (W,), (W,),
                                                             (W,), (W,)], init_seed=104,
                                     solid=_cube((20, 8, 66), (8, 2, 20), (11, 5, 40))),
}


def _oracle_forces(case, steps):
    import oracle
    faces = [_oface(F) for F in case.faces]
    if case.q == 9:
        faces[4] = faces[5] = oracle.Face()
    S = oracle.Sim(q=case.q, nx=case.oshape[0], ny=case.oshape[1], nz=case.oshape[2], tau=case.tau, faces=faces,
                   solid=None if case.solid is None else case.solid.reshape(case.oshape))
    rho, u = case.init_fields()
    f = S.equilibrium_state(rho=rho.reshape(case.oshape), u=u.reshape(case.oshape + (case.D,)))
    S.run(f, steps)
    return S.forces(f)


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("storage,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_forces_match_oracle(name, storage, tol):
    base = CASES[name]
    _announce(f"forces {name} {storage}")
    for steps in (6, 7):    # after an odd and an even AA step
        case = Case(base.q, base.shape, base.tau, base.faces, steps=steps, storage=storage,
                    init_seed=base.init_seed, solid=base.solid)
        sim = gpu_sim(case)
        sim.step(steps)
        Fs, Ff = sim.forces()
        Os, Of = _oracle_forces(case, steps)
        if case.q == 9:
            Of = Of[:, :2]
            Of = np.vstack([Of[:4], np.zeros((2, 2))])
            Os = Os[:2]
            Fs, Ff = Fs[:2], Ff[:, :2]
        scale = np.abs(Os).sum() + np.abs(Of).sum()
        err = max(np.max(np.abs(Fs - Os)), np.max(np.abs(Ff - Of)))
        print(f"[case] {name} {storage} steps={steps}: max |dF| {err:.3e} (scale {scale:.3e})", flush=True)
        assert err <= tol * scale


def test_momentum_balance_on_gpu():
    """Closed domain, FP64: the fluid momentum (lbm_moments sums) changes over
    each step by exactly minus the total force."""
    _announce("momentum balance")
    case = CASES["d3q19_walls_spheres"]
    sim = gpu_sim(Case(case.q, case.shape, case.tau, case.faces, storage="f64", init_seed=case.init_seed,
                       solid=case.solid))
    for _ in range(4):
        P0 = sim.sums()[1:4]
        sim.step(1)
        P1 = sim.sums()[1:4]
        Fs, Ff = sim.forces()
        total = Fs + Ff.sum(0)
        scale = np.abs(Fs).sum() + np.abs(Ff).sum()
        assert np.max(np.abs((P1 - P0) + total)) <= 1e-12 * scale


def test_forces_errors():
    _announce("forces errors")
    sim = gpu_sim(Case(19, (6, 7, 66), 0.6, [(W,)] * 6, storage="f32"))
    with pytest.raises(lbm.LbmError):
        sim.forces()            # no step since init
    sim.step(1)
    Fs, Ff = sim.forces()
    assert np.all(np.isfinite(Ff))
    bs = lbm.BatchSim("D2Q9", [(8, 8)], [0.7], [[(W,), (W,), (W,), (W, (0.05, 0.0)), (P,), (P,)]])
    bs.init_equilibrium()
    bs.step(1)
    out = (lbm.ctypes.c_double * 21)()
    assert lbm.lib().lbm_forces(bs.h, out) == lbm.LBM_EUNSUPPORTED

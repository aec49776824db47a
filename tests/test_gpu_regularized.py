"""GPU regularized velocity / pressure faces against the FP64 oracle (pinned
in test_oracle_regularized.py): inlet / outlet combinations on every lattice,
open faces across the contiguous axis, mixed with Zou-He and outflow faces,
solids, all storages, both AA parities; batch domains equal single-domain
runs bitwise; the adjoint (compared with the oracle's in test_gpu_adjoint.py)
refuses them on batches and with body forces."""
import sys

import numpy as np
import pytest

from cases import Case, compare, gpu_run, gpu_sim, oracle_run
from paper_2311_16080_amd import lbm

pytestmark = pytest.mark.gpu
W, P, ZV, ZP, OUT = lbm.WALL, lbm.PERIODIC, lbm.ZOUHE_VELOCITY, lbm.ZOUHE_PRESSURE, lbm.EQ_OUTFLOW
RV, RP = lbm.REG_VELOCITY, lbm.REG_PRESSURE
TOL = {"f64": (1e-12, 1e-13), "f32": (1e-5, 1e-6), "f16": (1e-3, 1e-4), "bf16": (3e-2, 3e-3)}


def _announce(name):
    print(f"\n[case] {name}", flush=True)
    sys.stdout.flush()


def _cube(shape, lo, hi):
    s = np.zeros(shape, np.uint8)
    s[tuple(slice(a, b) for a, b in zip(lo, hi))] = 1
    return s


CASES = {
    "d2q9_vel_pres": Case(9, (48, 40), 0.7, [(RV, (0.04, 0.0)), (RP, (0, 0, 0), 1.0), (W,), (W, (0.02, 0.0)), (P,),
                                             (P,)], init_seed=401),
    "d3q19_vel_outflow_cube": Case(19, (24, 10, 66), 0.65, [(RV, (0.03, 0.005, 0)), (OUT, (0, 0, 0), 1.0), (W,), (W,),
                                                            (P,), (P,)], init_seed=402,
                                   solid=_cube((24, 10, 66), (8, 3, 20), (12, 6, 40))),
    "d3q27_pres_pres": Case(27, (20, 9, 66), 0.6, [(RP, (0, 0, 0), 1.01), (RP, (0, 0, 0), 0.99), (W,), (W,), (P,),
                                                   (P,)], init_seed=403),
    "d3q19_z_open_faces": Case(19, (8, 10, 70), 0.7, [(W,), (W,), (W,), (W, (0.02, 0, 0)), (RV, (0.0, 0.01, 0.03)),
                                                      (RP, (0, 0, 0), 1.0)], init_seed=404),
    "d2q9_reg_vel_zouhe_pres": Case(9, (40, 24), 0.8, [(RV, (0.03, 0.0)), (ZP, (0, 0, 0), 1.0), (W,), (W,), (P,),
                                                       (P,)], init_seed=405),
}


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_regularized_matches_oracle(name, storage):
    base = CASES[name]
    utol, rtol = TOL[storage]
    for steps in (20, 21):
        case = Case(base.q, base.shape, base.tau, base.faces, steps=steps, storage=storage,
                    init_seed=base.init_seed, solid=base.solid)
        _announce(f"regularized {name} {storage} steps={steps}")
        g = gpu_run(case)
        o = oracle_run(case)
        eu, er = compare(case, g, o)
        print(f"[case] {name} {storage} steps={steps}: u rel-L2 {eu:.3e}, max|drho| {er:.3e}", flush=True)
        assert eu < utol and er < rtol


def test_regularized_double_buffer_equals_in_place():
    import torch
    base = CASES["d3q27_pres_pres"]
    out = []
    for pattern in ("inplace", "double", "pull"):
        case = Case(base.q, base.shape, base.tau, base.faces, steps=13, storage="f32", pattern=pattern,
                    init_seed=base.init_seed)
        sim = gpu_sim(case)
        sim.step(13)
        out.append(sim.moments())
    for o in out[1:]:
        assert torch.equal(out[0][0], o[0]) and torch.equal(out[0][1], o[1])


def test_batch_with_regularized_faces_equals_single_domains():
    import torch
    _announce("regularized batch")
    shapes = [(40, 24), (33, 20)]
    taus = [0.7, 0.9]
    faces = [[(RV, (0.04, 0.0)), (RP, (0, 0, 0), 1.0), (W,), (W,), (P,), (P,)],
             [(RP, (0, 0, 0), 1.01), (RV, (-0.02, 0.0)), (W, (0.03, 0.0)), (W,), (P,), (P,)]]
    bs = lbm.BatchSim("D2Q9", shapes, taus, faces, storage="f32")
    bs.init_equilibrium()
    bs.step(17)
    rho_b, u_b = bs.moments()
    off = bs.offsets
    for d in range(2):
        sim = lbm.Sim("D2Q9", shapes[d], taus[d], faces=faces[d], storage="f32")
        sim.init_equilibrium()
        sim.step(17)
        rho, u = sim.moments()
        n = int(np.prod(shapes[d]))
        assert torch.equal(rho_b[off[d]:off[d] + n].reshape(shapes[d]), rho)
        assert torch.equal(u_b[:, off[d]:off[d] + n].reshape((2,) + shapes[d]), u)


def test_adjoint_of_regularized_faces_refusals():
    """The regularized closure's transpose runs on single domains without a
    body force: a force (set, or asked for by backward_force) is refused."""
    import torch
    _announce("regularized adjoint refusals")
    case = Case(9, (24, 16), 0.7, [(RV, (0.03, 0.0)), (OUT, (0, 0, 0), 1.0), (W,), (W,), (P,), (P,)], storage="f32")
    sim = gpu_sim(case)
    sim.tape_begin(2, 4)
    sim.step(4)
    sim.tape_end()
    with pytest.raises(lbm.LbmError) as ei:
        sim.backward_force(None, torch.zeros((2, 24, 16), device="cuda"))
    assert ei.value.code == lbm.LBM_EUNSUPPORTED
    ds, dtau, _ = sim.backward(None, torch.zeros((2, 24, 16), device="cuda"))
    assert dtau[0] == 0.0
    sim.set_force([1e-5, 0.0])
    sim.tape_begin(2, 4)
    sim.step(4)
    sim.tape_end()
    with pytest.raises(lbm.LbmError) as ei:
        sim.backward(None, torch.zeros((2, 24, 16), device="cuda"))
    assert ei.value.code == lbm.LBM_EUNSUPPORTED

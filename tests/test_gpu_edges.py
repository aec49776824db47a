"""Edge and degenerate cases of the GPU path against the FP64 oracle (or exact
expectations): grids thinner than a wavefront or a single cell thick, rows of
64k + 1 cells, tau at the stability edge and tau = 1, zero-step calls, all-solid
domains, a tape with no steps, batches of tiny domains."""
import sys

import numpy as np
import pytest

from cases import Case, compare, gpu_run, gpu_sim, oracle_run
from paper_2311_16080_amd import inputs, lbm

pytestmark = pytest.mark.gpu
W, P, ZV, ZP, OUT = lbm.WALL, lbm.PERIODIC, lbm.ZOUHE_VELOCITY, lbm.ZOUHE_PRESSURE, lbm.EQ_OUTFLOW


def _announce(name):
    print(f"\n[case] {name}", flush=True)
    sys.stdout.flush()


EDGE = {
    "d3q19_1x1x130_periodic": Case(19, (1, 1, 130), 0.7, steps=17, init_seed=80),
    "d3q19_5x6x1_periodic_z": Case(19, (5, 6, 1), 0.8, [(W,), (W, (0, 0.02, 0.01)), (W,), (W,), (P,), (P,)],
                                   steps=15, init_seed=81),
    "d2q9_1x70_periodic_x": Case(9, (1, 70), 0.9, [(P,), (P,), (W,), (W, (0.03, 0)), (P,), (P,)], steps=21,
                                 init_seed=82),
    "d3q27_3x3x5_walls": Case(27, (3, 3, 5), 0.6, [(W,)] * 5 + [(W, (0.05, 0.0, 0.0))], steps=19, init_seed=83),
    "d3q19_2x2x65_walls": Case(19, (2, 2, 65), 0.55, [(W,)] * 5 + [(W, (0.04, 0.01, 0.0))], steps=23,
                               init_seed=84),
    "d3q19_2x3x257_zouhe_z": Case(19, (2, 3, 257), 0.65, [(W,), (W,), (P,), (P,), (ZV, (0.0, 0.01, 0.03)),
                                                          (ZP, (0, 0, 0), 0.998)], steps=13, init_seed=85),
    "d2q9_tau_edge": Case(9, (33, 65), 0.5 + 1e-6, [(P,), (P,), (W,), (W, (0.01, 0)), (P,), (P,)], steps=9,
                          init_seed=86, amp=0.005),
    "d3q19_tau_one": Case(19, (6, 7, 70), 1.0, [(W,)] * 5 + [(W, (0.05, 0, 0))], steps=12, init_seed=87),
    "d3q27_single_fluid_cell_in_solid": Case(27, (3, 3, 3), 0.7, [(P,)] * 6, steps=5, init_seed=88,
                                             solid=(np.arange(27).reshape(3, 3, 3) != 13).astype(np.uint8)),
}


@pytest.mark.parametrize("name", sorted(EDGE))
def test_edge_case_matches_oracle(name):
    case = EDGE[name]
    _announce(name)
    g = gpu_run(case)
    o = oracle_run(case)
    du, drho = compare(case, g, o)
    print(f"[case] {name}: u rel-L2 {du:.3e}, max |drho| {drho:.3e}", flush=True)
    assert du <= 1e-12 and drho <= 1e-13
    _assert_sums(g[2], o[2])


def _assert_sums(sg, so):
    """FP64 block sums (mass, momentum, kinetic energy) against the oracle's
    Kahan sums over the fluid cells (eqs. density, velocity)."""
    assert abs(sg[0] - so[0]) <= 1e-12 * abs(so[0]), (sg[0], so[0])
    for a in (1, 2, 3):
        assert abs(sg[a] - so[a]) <= 1e-12 * abs(so[0]), (a, sg[a], so[a])
    assert abs(sg[4] - so[4]) <= 1e-10 * abs(so[4]) + 1e-300, (sg[4], so[4])


@pytest.mark.parametrize("block", [64, 128, 192, 256])
def test_moment_sums_at_every_block_size(block, monkeypatch):
    """Rows of 300 cells launched with blocks of 64 / 128 / 192 / 256 lanes
    (LBM_BLOCK): the moment sums cover every cell of every block, whatever the
    block size."""
    monkeypatch.setenv("LBM_BLOCK", str(block))
    case = Case(19, (3, 4, 300), 0.7, [(W,)] * 5 + [(W, (0.04, 0.0, 0.0))], steps=9, init_seed=93)
    _announce(f"moment sums, block {block}")
    g = gpu_run(case)
    o = oracle_run(case)
    du, drho = compare(case, g, o)
    assert du <= 1e-12 and drho <= 1e-13
    _assert_sums(g[2], o[2])


def test_zero_steps_change_nothing():
    import torch
    _announce("step(0)")
    sim = gpu_sim(Case(19, (6, 7, 70), 0.6, [(W,)] * 5 + [(W, (0.05, 0, 0))], storage="f32", init_seed=89))
    sim.step(3)
    r0, u0 = sim.moments(dtype=torch.float64)
    blob = sim.save()
    sim.step(0)
    assert sim.t == 3
    r1, u1 = sim.moments(dtype=torch.float64)
    assert torch.equal(r0, r1) and torch.equal(u0, u1)
    assert sim.save() == blob


def test_all_solid_domain():
    """Every cell solid: moments report rho0 and 0, sums are zero, steps are no-ops."""
    import torch
    _announce("all solid")
    c = Case(19, (4, 5, 66), 0.7, [(W,)] * 6, storage="f32", solid=np.ones((4, 5, 66), np.uint8))
    sim = gpu_sim(c)
    sim.step(4)
    rho, u, s = sim.moments(dtype=torch.float64, sums=True)
    assert torch.all(rho == 1.0) and torch.all(u == 0.0)
    assert np.all(s == 0.0)


def test_tape_without_steps():
    """A tape of zero steps: the backward is the seed's own transpose; the
    parameter gradients are exactly zero."""
    import torch
    _announce("empty tape")
    sim = gpu_sim(Case(19, (6, 7, 70), 0.6, [(W,)] * 5 + [(W, (0.05, 0, 0))], storage="f64", init_seed=90))
    sim.step(2)
    sim.tape_begin(4, 8)
    sim.tape_end()
    rho, u = sim.moments(dtype=torch.float64)
    _, dtau, duw = sim.backward(None, u.clone())
    assert dtau[0] == 0.0 and np.all(duw == 0.0)


def test_batch_of_tiny_domains_matches_oracle():
    """Domains smaller than a tile and a wavefront, some a single cell thick."""
    import torch
    _announce("batch of tiny domains")
    shapes = [(2, 2), (1, 5), (3, 64), (65, 1), (7, 7)]
    taus = [0.6, 0.7, 0.8, 0.9, 0.55]
    faces = [[(W,), (W,), (W,), (W, (0.05, 0.0)), (P,), (P,)],
             [(P,), (P,), (W,), (W, (0.02, 0.0)), (P,), (P,)],
             [(W,), (W,), (P,), (P,), (P,), (P,)],
             [(W,), (W, (0.0, 0.03)), (P,), (P,), (P,), (P,)],
             [(W,), (W,), (W,), (W, (0.08, 0.0)), (P,), (P,)]]
    bs = lbm.BatchSim("D2Q9", shapes, taus, faces, storage="f64")
    bs.tuning(64, 0)
    rho0 = torch.tensor(inputs.random_density((bs.N,), 91, amp=0.01), device="cuda")
    u0 = torch.tensor(inputs.random_velocity((bs.N,), 2, 92, amp=0.03).T.copy(), device="cuda")
    bs.init_equilibrium(rho0, u0)
    bs.step(11)
    r, u = bs.moments(dtype=torch.float64)
    for d in range(len(shapes)):
        a, b = int(bs.offsets[d]), int(bs.offsets[d + 1])
        c = Case(9, shapes[d], taus[d], faces[d], steps=11,
                 init_u=u0[:, a:b].T.cpu().numpy().reshape(shapes[d] + (2,)))
        rho_d = rho0[a:b].cpu().numpy().reshape(shapes[d])
        import oracle
        from cases import _oface
        of = [_oface(F) for F in c.faces]
        of[4] = of[5] = oracle.Face()
        S = oracle.Sim(q=9, nx=shapes[d][0], ny=shapes[d][1], nz=1, tau=taus[d], faces=of)
        f = S.equilibrium_state(rho=rho_d.reshape(c.oshape), u=c.init_u.reshape(c.oshape + (2,)))
        S.run(f, 11)
        ro, uo = S.moments(f)
        rg = bs.domain(r, d).cpu().numpy()
        ug = np.stack([bs.domain(u, d)[k].cpu().numpy() for k in range(2)], -1)
        assert np.max(np.abs(rg - ro[..., 0])) <= 1e-13, d
        assert np.max(np.abs(ug - uo[..., 0, :2])) <= 1e-13, d


@pytest.mark.parametrize("q,shape,faces", [
    (19, (7, 6, 300), [(ZV, (0.03, 0, 0)), (OUT, (0, 0, 0), 1.0), (W,), (W, (0.02, 0, 0)), (W,), (W,)]),
    (9, (33, 65), [(W,), (W,), (P,), (P,), (P,), (P,)]),
    (27, (5, 6, 70), [(W,)] * 5 + [(W, (0.05, 0.0, 0.0))]),
    (19, (4, 3, 1), [(W,), (W, (0, 0.02, 0.0)), (W,), (W,), (P,), (P,)]),
])
@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_flat_and_row_lane_mappings_agree_bitwise(q, shape, faces, storage, monkeypatch):
    """Rows whose length is not a multiple of 64 cells run with blocks of
    consecutive cells of the whole grid (LBM_FLAT=1, the default there); the
    row-chunk mapping (LBM_FLAT=0) runs the same per-cell arithmetic, so the
    moments agree bit for bit after even and odd step counts."""
    _announce(f"flat vs row lanes q={q} {shape} {storage}")
    out = {}
    for flat in ("0", "1"):
        monkeypatch.setenv("LBM_FLAT", flat)
        for steps in (8, 9):
            g = gpu_run(Case(q, shape, 0.6, faces, steps=steps, storage=storage, init_seed=95))
            out[(flat, steps)] = (g[0], g[1])
    for steps in (8, 9):
        a, b = out[("0", steps)], out[("1", steps)]
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), steps

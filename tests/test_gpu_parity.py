"""GPU (liblbm.so, HIP) vs FP64 CPU oracle, element by element on the same
seeded inputs.  Sizes span several Z tiles with a ragged tail; every boundary
type, all three lattices, both streaming patterns and every storage format.

Tolerances (rel-L2 of u over fluid cells; max |rho - rho_oracle|):
  FP64 storage/compute: 1e-12 / 1e-13   (same recurrence, rounding order only)
  FP32 storage (deviation form), FP32 compute: 1e-5 / 1e-6
  FP16 storage (h_i / w_i), FP32 compute: 1e-3 / 1e-4
  BF16 storage: reported, gated only at 3e-2 (8-bit mantissa)
"""
import sys

import numpy as np
import pytest

from cases import Case, compare, gpu_run, gpu_sim, oracle_run
from paper_2311_16080_amd import inputs, lbm

pytestmark = pytest.mark.gpu

W, P, ZV, ZP, OUT = lbm.WALL, lbm.PERIODIC, lbm.ZOUHE_VELOCITY, lbm.ZOUHE_PRESSURE, lbm.EQ_OUTFLOW
TOL = {"f64": (1e-12, 1e-13), "f32": (1e-5, 1e-6), "f16": (1e-3, 1e-4), "bf16": (3e-2, 3e-3)}


def _announce(name):
    print(f"\n[case] {name}", flush=True)
    sys.stdout.flush()


def cavity_faces3(U=0.05):
    return [(W,), (W,), (W,), (W,), (W,), (W, (U, 0, 0))]


def cavity_faces2(U=0.08):
    return [(W,), (W,), (W,), (W, (U, 0, 0)), (P,), (P,)]


def channel_faces3(uin=0.04):
    return [(ZV, (uin, 0, 0)), (OUT, (0, 0, 0), 1.0), (W,), (W,), (W,), (W,)]


def spheres(shape, seed=3):
    nx, ny, nz = shape
    return inputs.sphere_obstacles(nx, ny, nz, seed=seed, rmin=2, rmax=5, xlo=4, xhi=nx - 4, fraction=0.05)


CASES = {
    # Taylor-Green vortex, the paper's Sec. 4.1 problem (config: 128^2, FP64, tau 0.8)
    "tgv_d2q9_f64": Case(9, (128, 128), 0.8, steps=201,
                         init_u=inputs.taylor_green_velocity(128, 128, 0.01)),
    "periodic_d2q9_f64_ragged": Case(9, (37, 300), 0.7, steps=33, init_seed=1),
    "periodic_d3q19_f64_ragged": Case(19, (6, 5, 300), 0.6, steps=21, init_seed=2),
    # rows of 576 cells run as three 192-lane blocks (the block size that
    # launches the fewest lanes); the FP64 sums cover all of them
    "periodic_d2q9_f64_rows576": Case(9, (21, 576), 0.7, steps=15, init_seed=12),
    "cavity_d3q19_f64_rows130": Case(19, (5, 6, 130), 0.6, cavity_faces3(), steps=19, init_seed=13),
    "periodic_d3q27_f64": Case(27, (7, 6, 70), 0.9, steps=12, init_seed=3),
    "cavity_d3q19_f64": Case(19, (10, 9, 300), 0.55, cavity_faces3(), steps=61),
    "cavity_d3q19_f64_double": Case(19, (10, 9, 300), 0.55, cavity_faces3(), steps=61, pattern="double"),
    "cavity_d3q27_f64": Case(27, (9, 8, 70), 0.6, cavity_faces3(), steps=40, init_seed=4),
    "cavity_d2q9_f64": Case(9, (40, 330), 0.52, cavity_faces2(), steps=80),
    "cavity_d3q19_f32": Case(19, (10, 9, 300), 0.55, cavity_faces3(), steps=61, storage="f32"),
    "cavity_d3q19_f16": Case(19, (10, 9, 300), 0.55, cavity_faces3(), steps=61, storage="f16"),
    "cavity_d3q19_bf16": Case(19, (10, 9, 300), 0.55, cavity_faces3(), steps=61, storage="bf16"),
    "moving_walls_d3q19_f64": Case(19, (8, 9, 66), 0.7, [(W,), (W, (0, 0.02, 0.01)), (W,), (W, (0.03, 0, -0.02)),
                                                         (W,), (W, (0.05, 0.01, 0))], steps=25, init_seed=5),
    "channel_spheres_d3q27_f64": Case(27, (24, 12, 70), 0.6, channel_faces3(), steps=30, init_seed=6,
                                      solid=spheres((24, 12, 70))),
    "channel_spheres_d3q27_f32": Case(27, (24, 12, 70), 0.6, channel_faces3(), steps=30, init_seed=6,
                                      solid=spheres((24, 12, 70)), storage="f32"),
    "channel_spheres_d3q19_f64_double": Case(19, (24, 12, 70), 0.6, channel_faces3(), steps=31, init_seed=7,
                                             solid=spheres((24, 12, 70), seed=8), pattern="double"),
    "zouhe_vel_pres_d3q19_f64_periodic_z": Case(19, (20, 9, 70), 0.7,
                                                [(ZV, (0.03, 0.005, 0.002)), (ZP, (0, 0, 0), 0.99), (W,), (W,),
                                                 (P,), (P,)], steps=27, init_seed=9),
    "zouhe_pres_in_d3q27_f64_y_axis": Case(27, (7, 20, 66), 0.65,
                                           [(W,), (W, (0.0, 0, 0.02)), (ZP, (0, 0, 0), 1.01), (OUT, (0, 0, 0), 1.0),
                                            (P,), (P,)], steps=24, init_seed=10),
    "zouhe_z_axis_d3q19_f64": Case(19, (7, 8, 90), 0.6, [(W,), (W,), (P,), (P,), (ZV, (0.01, 0, 0.04)),
                                                         (OUT, (0, 0, 0), 1.0)], steps=22, init_seed=11),
    "channel_pbb_d2q9_f64": Case(9, (96, 40), 0.6, [(ZV, (0.04, 0)), (OUT, (0, 0, 0), 1.0), (W,), (W,), (P,), (P,)],
                                 steps=50, s=inputs.smooth_solid_fraction(96, 40, seed=4, sigma=3, edge=8)),
    "channel_pbb_d2q9_f32": Case(9, (96, 40), 0.6, [(ZV, (0.04, 0)), (OUT, (0, 0, 0), 1.0), (W,), (W,), (P,), (P,)],
                                 steps=50, s=inputs.smooth_solid_fraction(96, 40, seed=4, sigma=3, edge=8),
                                 storage="f32"),
    "zouhe_pres_pres_d2q9_f64_y_axis": Case(9, (33, 70), 0.8, [(W,), (W,), (ZP, (0, 0, 0), 1.005),
                                                               (ZP, (0, 0, 0), 0.995), (P,), (P,)], steps=45),
    # the pull pattern (two buffers, every step gathers): walls, solids and open
    # faces, periodic Z faces, partial bounce-back
    "cavity_d3q19_f64_pull": Case(19, (10, 9, 300), 0.55, cavity_faces3(), steps=61, pattern="pull"),
    "channel_spheres_d3q27_f32_pull": Case(27, (24, 12, 70), 0.6, channel_faces3(), steps=30, init_seed=6,
                                           solid=spheres((24, 12, 70)), storage="f32", pattern="pull"),
    "zouhe_vel_pres_d3q19_f64_periodic_z_pull": Case(19, (20, 9, 70), 0.7,
                                                     [(ZV, (0.03, 0.005, 0.002)), (ZP, (0, 0, 0), 0.99), (W,), (W,),
                                                      (P,), (P,)], steps=27, init_seed=9, pattern="pull"),
    "channel_pbb_d2q9_f64_pull": Case(9, (96, 40), 0.6, [(ZV, (0.04, 0)), (OUT, (0, 0, 0), 1.0), (W,), (W,), (P,), (P,)],
                                      steps=50, s=inputs.smooth_solid_fraction(96, 40, seed=4, sigma=3, edge=8),
                                      pattern="pull"),
    "periodic_d3q27_f16_pull": Case(27, (7, 6, 128), 0.9, steps=12, init_seed=3, storage="f16", pattern="pull"),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_parity_vs_oracle(name):
    case = CASES[name]
    _announce(name)
    g = gpu_run(case)
    o = oracle_run(case)
    du, drho = compare(case, g, o)
    tol_u, tol_rho = TOL[case.storage]
    print(f"[case] {name}: u rel-L2 {du:.3e} (tol {tol_u:g}), max|drho| {drho:.3e} (tol {tol_rho:g})", flush=True)
    assert np.all(np.isfinite(g[1]))
    assert du <= tol_u
    assert drho <= tol_rho
    if case.storage == "f64":
        # FP64 block sums (mass, momentum, KE) against the oracle's Kahan sums
        so = o[2]
        sg = g[2]
        assert abs(sg[0] - so[0]) <= 1e-12 * abs(so[0])
        for a in (1, 2, 3):
            assert abs(sg[a] - so[a]) <= 1e-12 * abs(so[0])
        assert abs(sg[4] - so[4]) <= 1e-10 * abs(so[4]) + 1e-300


@pytest.mark.parametrize("q,shape", [(9, (40, 130)), (19, (6, 7, 130)), (27, (5, 6, 66))])
@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_inplace_equals_double_buffer_bitwise(q, shape, storage):
    """The in-place AA pattern, the double-buffer push pattern and the pull
    pattern run the same arithmetic; their moments agree bitwise after even and
    odd step counts (and after the pull pattern's first, local step)."""
    import torch
    _announce(f"inplace-vs-double-vs-pull q={q} {storage}")
    faces = [(ZV, (0.03, 0, 0)), (OUT, (0, 0, 0), 1.0), (W,), (W, (0.02, 0, 0)), (W,), (W,)]
    for steps in (1, 6, 7):
        res = [gpu_run(Case(q, shape, 0.6, faces, steps=steps, storage=storage, init_seed=20, pattern=pat))
               for pat in ("inplace", "double", "pull")]
        for k, g in enumerate(res[1:], 1):
            assert np.array_equal(res[0][0], g[0]) and np.array_equal(res[0][1], g[1]), (steps, k)
        del res
        torch.cuda.synchronize()


def test_pull_pattern_graph_replay_equals_steps():
    """A graph of pull steps replays what lbm_step does, replay after replay;
    a graph captured before the first (local) step is refused afterwards."""
    import torch
    _announce("pull graph replay")
    case = Case(19, (8, 9, 130), 0.6, cavity_faces3(), steps=0, storage="f32", init_seed=21, pattern="pull")
    a, b = gpu_sim(case), gpu_sim(case)
    c = gpu_sim(case)
    c.capture_graph(2)
    c.graph_launch()           # from t = 0: the local step, then a pull step
    a.step(1)
    b.step(1)
    b.capture_graph(2)
    for k in range(3):
        a.step(2)
        b.graph_launch()
        torch.cuda.synchronize()
        ra, ua = a.moments()
        rb, ub = b.moments()
        assert torch.equal(ra, rb) and torch.equal(ua, ub), k
    with pytest.raises(lbm.LbmError):
        c.graph_launch()       # t > 0 now: the captured local step no longer applies


def test_uniform_rest_with_walls_fixed_point():
    _announce("rest fixed point")
    c = Case(19, (8, 9, 70), 0.55, [(W,)] * 6, steps=40, storage="f32")
    g = gpu_run(c)
    assert np.max(np.abs(g[1])) == 0.0
    assert np.max(np.abs(g[0] - 1.0)) < 1e-6


def test_pbb_zero_is_plain_bgk_bitwise():
    _announce("pbb zero")
    base = dict(q=9, shape=(64, 40), tau=0.6, faces=[(ZV, (0.04, 0)), (OUT, (0, 0, 0), 1.0), (W,), (W,), (P,), (P,)],
                steps=31, storage="f32", init_seed=30)
    a = gpu_run(Case(**base))
    b = gpu_run(Case(**base, s=np.zeros((64, 40))))
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_save_load_resume_bitwise():
    import torch
    _announce("save/load")
    c = Case(19, (8, 9, 70), 0.6, cavity_faces3(), steps=0, storage="f32", init_seed=40)
    from cases import gpu_sim
    ref = gpu_sim(c)
    ref.step(13)
    r_ref, u_ref = ref.moments(dtype=torch.float64)
    sim = gpu_sim(c)
    sim.step(5)
    blob = sim.save()
    sim2 = gpu_sim(c)
    sim2.step(2)
    sim2.load(blob)
    assert sim2.t == 5
    sim2.step(8)
    r2, u2 = sim2.moments(dtype=torch.float64)
    assert torch.equal(r_ref, r2) and torch.equal(u_ref, u2)


def test_graph_replay_matches_eager():
    import torch
    _announce("graph replay")
    c = Case(19, (8, 9, 70), 0.6, cavity_faces3(), steps=0, storage="f32", init_seed=41)
    from cases import gpu_sim
    eager = gpu_sim(c)
    eager.step(30)
    r_e, u_e = eager.moments(dtype=torch.float64)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        g = gpu_sim(c)
        g.use_current_stream()
        g.step(2)                        # zh-independent, parity 0
        g.capture_graph(4)
        for k in range(7):
            g.graph_launch()
            torch.cuda.synchronize()     # eager work between replays
        r_g, u_g = g.moments(dtype=torch.float64)
    torch.cuda.synchronize()
    assert g.t == 30
    assert torch.equal(r_e, r_g) and torch.equal(u_e, u_g)



@pytest.mark.parametrize("storage", ["f64", "f32", "f16", "bf16"])
def test_memory_hints_do_not_change_results(storage, monkeypatch):
    """Plain, non-temporal and non-temporal-store variants of the step kernel
    differ only in cache hints: bitwise equal moments."""
    _announce(f"memory hints {storage}")
    faces = [(W,), (W,), (P,), (P,), (ZV, (0.01, 0, 0.03)), (OUT, (0, 0, 0), 1.0)]
    ref = None
    for nt in ("0", "1", "2"):
        monkeypatch.setenv("LBM_NT", nt)
        g = gpu_run(Case(19, (6, 5, 264), 0.62, faces, steps=7, storage=storage, init_seed=50))
        if ref is None:
            ref = g
        else:
            assert np.array_equal(ref[0], g[0]) and np.array_equal(ref[1], g[1]), nt


PAIR_CASES = {
    "cavity_d3q19": (19, (8, 9, 256), [(W,)] * 5 + [(W, (0.05, 0.01, 0))]),
    "moving_walls_d3q19": (19, (6, 7, 384), [(W,), (W, (0, 0.02, 0.01)), (W,), (W, (0.03, 0, -0.02)),
                                             (W, (0.02, 0.01, 0)), (W, (0.05, 0.01, 0))]),
    "periodic_z_d3q19": (19, (6, 5, 128), [(W,), (W, (0, 0.01, 0.02)), (W,), (W,), (P,), (P,)]),
    "periodic_xy_d3q27": (27, (4, 5, 256), [(P,), (P,), (P,), (P,), (W,), (W, (0.04, 0, 0))]),
    "channel_zouhe_d3q19": (19, (20, 6, 128), [(ZV, (0.03, 0, 0)), (OUT, (0, 0, 0), 1.0), (W,), (W,), (W,), (W,)]),
    "cavity_d2q9": (9, (40, 256), [(W,), (W,), (W,), (W, (0.08, 0.0)), (P,), (P,)]),
    "spheres_d3q27": (27, (24, 12, 128), [(ZV, (0.03, 0, 0)), (OUT, (0, 0, 0), 1.0), (W,), (W,), (W,), (W,)]),
    # rows of several blocks (768 cells: two blocks of 192 lanes; 1024: two of 256)
    "cavity_d3q19_rows768": (19, (4, 5, 768), [(W,), (W, (0, 0.02, 0.01)), (W,), (W,), (W,), (W, (0.05, 0.01, 0))]),
    "cavity_d3q27_rows1024": (27, (3, 4, 1024), [(W,)] * 5 + [(W, (0.04, 0.02, 0.0))]),
    "pbb_d2q9": (9, (24, 256), [(W,), (W,), (W,), (W, (0.06, 0.0)), (P,), (P,)]),
    # one wavefront per row (both Z walls in every wavefront), moving walls on Y and Z faces
    "cavity_d3q19_rows128": (19, (5, 6, 128), [(W,), (W,), (W,), (W, (0.02, 0, 0.01)), (W, (0.01, 0.02, 0)),
                                               (W, (0.05, 0.01, 0))]),
}


@pytest.mark.parametrize("name", sorted(PAIR_CASES))
@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_pair_kernel_matches_one_cell_per_lane_bitwise(name, storage, monkeypatch):
    """2-byte storage runs two cells per lane where rows allow it; the result
    is bitwise that of the one-cell-per-lane kernel (same per-cell arithmetic)."""
    _announce(f"pair kernel {name} {storage}")
    q, shape, faces = PAIR_CASES[name]
    solid = spheres(shape) if name.startswith("spheres") else None
    sfrac = inputs.smooth_solid_fraction(*shape, seed=4, sigma=3, edge=4) if name.startswith("pbb") else None
    res = {}
    # never / even steps / even and odd steps; the pull pattern (pull steps)
    for pair in ("0", "1", "2"):
        monkeypatch.setenv("LBM_PAIR", pair)
        for steps in (7, 8):
            res[(pair, steps)] = gpu_run(Case(q, shape, 0.6, faces, steps=steps, storage=storage, init_seed=55,
                                              solid=solid, s=sfrac))
            if pair != "2":
                res[(pair, steps, "pull")] = gpu_run(Case(q, shape, 0.6, faces, steps=steps, storage=storage,
                                                          init_seed=55, solid=solid, s=sfrac, pattern="pull"))
    for key in [("1", 7), ("1", 8), ("2", 7), ("2", 8), ("0", 7, "pull"), ("0", 8, "pull"), ("1", 7, "pull"),
                ("1", 8, "pull")]:
        a, b = res[("0", key[1])], res[key]
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), key

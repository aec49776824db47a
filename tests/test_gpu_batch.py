"""Batched domains (one tile list, per-step or persistent launches, HIP graph)
against single-domain runs of the same domains: bitwise equal moments, for
every tile size and both launch modes; plus the FP64 batch against the oracle."""
import sys

import numpy as np
import pytest

from cases import Case, compare, gpu_run, oracle_run
from paper_2311_16080_amd import inputs, lbm

pytestmark = pytest.mark.gpu
W, P, ZV, OUT = lbm.WALL, lbm.PERIODIC, lbm.ZOUHE_VELOCITY, lbm.EQ_OUTFLOW


def _announce(name):
    print(f"\n[case] {name}", flush=True)
    sys.stdout.flush()


def cavities2d(n=10, seed=5):
    L, tau, U = inputs.batch_cavities(n, seed=seed, lmin=17, lmax=90)
    shapes = [(int(l), int(l) + 3 * (d % 3)) for d, l in enumerate(L)]
    faces = [[(W,), (W,), (W,), (W, (float(U[d]), 0.0)), (P,), (P,)] for d in range(n)]
    return shapes, tau, faces


def domains3d():
    shapes = [(6, 7, 33), (5, 9, 64), (8, 4, 20)]
    taus = [0.6, 0.75, 0.9]
    faces = [[(W,)] * 5 + [(W, (0.05, 0, 0))],
             [(ZV, (0.03, 0, 0)), (OUT, (0, 0, 0), 1.0), (W,), (W,), (P,), (P,)],
             [(P,), (P,), (W,), (W, (0.0, 0, 0.04)), (P,), (P,)]]
    return shapes, taus, faces


def _batch_moments(bs, steps, graph=False):
    import torch
    if graph:
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            bs.use_current_stream()
            bs.step(2)
            bs.capture_graph(4)
            for _ in range((steps - 2) // 4):
                bs.graph_launch()
                torch.cuda.synchronize()
            bs.step((steps - 2) % 4)
            r, u, s = bs.moments(dtype=torch.float64, sums=True)
        torch.cuda.synchronize()
    else:
        bs.step(steps)
        r, u, s = bs.moments(dtype=torch.float64, sums=True)
    return r.cpu().numpy(), u.cpu().numpy(), s


@pytest.mark.parametrize("tile", [64, 128, 256])
@pytest.mark.parametrize("persistent", [0, 1])
@pytest.mark.parametrize("kind", ["2d", "3d"])
def test_batch_equals_single_domain_runs(tile, persistent, kind):
    _announce(f"batch vs single {kind} tile={tile} persistent={persistent}")
    shapes, taus, faces = cavities2d() if kind == "2d" else domains3d()
    q = 9 if kind == "2d" else 19
    steps = 23
    bs = lbm.BatchSim("D2Q9" if q == 9 else "D3Q19", shapes, taus, faces, storage="f32")
    bs.tuning(tile, persistent)
    bs.init_equilibrium()
    r, u, s = _batch_moments(bs, steps)
    assert bs.config() [0] == tile
    for d in range(len(shapes)):
        g = gpu_run(Case(q, shapes[d], taus[d], faces[d], steps=steps, storage="f32"))
        rd = bs.domain(r, d)
        ud = bs.domain(u, d)
        assert np.array_equal(rd, g[0].reshape(shapes[d])), d
        for a in range(bs.D):
            assert np.array_equal(ud[a], g[1][..., a].reshape(shapes[d])), (d, a)
        assert np.allclose(s[d], g[2], rtol=1e-12, atol=1e-15)


def test_batch_graph_replay_matches_eager():
    _announce("batch graph")
    shapes, taus, faces = cavities2d(6, seed=7)
    a = lbm.BatchSim("D2Q9", shapes, taus, faces)
    a.tuning(128, 1)
    a.init_equilibrium()
    ra, ua, _ = _batch_moments(a, 30)
    for persistent in (0, 1):
        b = lbm.BatchSim("D2Q9", shapes, taus, faces)
        b.tuning(128, persistent)
        b.init_equilibrium()
        rb, ub, _ = _batch_moments(b, 30, graph=True)
        assert b.t == 30
        assert np.array_equal(ra, rb) and np.array_equal(ua, ub), persistent


def test_batch_f64_matches_oracle():
    _announce("batch f64 vs oracle")
    shapes, taus, faces = cavities2d(4, seed=9)
    bs = lbm.BatchSim("D2Q9", shapes, taus, faces, storage="f64")
    bs.init_equilibrium()
    r, u, s = _batch_moments(bs, 40)
    for d in range(4):
        c = Case(9, shapes[d], taus[d], faces[d], steps=40)
        o = oracle_run(c)
        g = (bs.domain(r, d).reshape(c.oshape), np.stack([bs.domain(u, d)[a] for a in range(2)] +
                                                          [np.zeros(shapes[d])], -1).reshape(c.oshape + (3,)))
        du, drho = compare(c, g, o)
        assert du <= 1e-12 and drho <= 1e-13, (d, du, drho)


def test_autotuner_picks_a_configuration(tmp_path, monkeypatch):
    _announce("autotuner")
    monkeypatch.setenv("LBM_AUTOTUNE_CACHE", str(tmp_path / "tune.txt"))
    shapes, taus, faces = cavities2d(8, seed=11)
    ref = lbm.BatchSim("D2Q9", shapes, taus, faces)
    ref.tuning(64, 0)
    ref.init_equilibrium()
    r0, u0, _ = _batch_moments(ref, 9)
    bs = lbm.BatchSim("D2Q9", shapes, taus, faces)
    bs.init_equilibrium()
    r1, u1, _ = _batch_moments(bs, 9)     # tunes on a copy of the state first
    tile, pers = bs.config()
    assert tile in (64, 128, 256) and pers in (0, 1)
    assert np.array_equal(r0, r1) and np.array_equal(u0, u1)
    assert (tmp_path / "tune.txt").read_text().strip()

"""C-ABI checks that need no GPU: the library loads, exports every symbol that
include/lbm.h declares, and rejects bad arguments before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2311_16080_amd import lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "lbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(lbm_[a-z_0-9]+)\s*\(", src)
    return sorted(set(names))


def test_every_declared_symbol_is_exported():
    L = lbm.lib()
    names = _declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(lbm.SIGNATURES), set(names) ^ set(lbm.SIGNATURES)


def test_version():
    assert "gfx950" in lbm.lib().lbm_version().decode()


@pytest.mark.parametrize("args,msg", [
    ((7, 8, 8, 8, 0.8), "unknown lattice"),
    ((lbm.D3Q19, 0, 8, 8, 0.8), "nx, ny"),
    ((lbm.D3Q19, 8, 8, 0, 0.8), "nz >= 1"),
    ((lbm.D2Q9, 8, 8, 5, 0.8), "nz = 0 or 1"),
    ((lbm.D3Q19, 8, 8, 8, 0.5), "tau"),
    ((lbm.D3Q19, 8, 8, 8, float("nan")), "tau"),
    ((lbm.D3Q27, 2048, 1024, 1024, 0.8), "2^31"),
])
def test_create_rejects(args, msg):
    h = lbm.lib().lbm_create(*args, None)
    assert not h
    assert msg in lbm.last_error()


def _bc(faces):
    return ctypes.byref(lbm.make_bc(faces))


@pytest.mark.parametrize("faces,msg", [
    ([lbm.WALL, lbm.PERIODIC, 0, 0, 0, 0], "periodic must be set on both"),
    ([(lbm.WALL, (0.1, 0, 0)), lbm.WALL, 0, 0, 0, 0], "tangential"),
    ([(lbm.ZOUHE_VELOCITY, (0.1, 0, 0)), lbm.EQ_OUTFLOW, (lbm.ZOUHE_PRESSURE, (0, 0, 0), 1.0), lbm.WALL, 0, 0],
     "one axis"),
    ([(lbm.ZOUHE_PRESSURE, (0, 0, 0), 0.0), lbm.WALL, 0, 0, 0, 0], "density"),
    ([(9,), lbm.WALL, 0, 0, 0, 0], "unknown boundary type"),
    ([(lbm.ZOUHE_VELOCITY, (1.5, 0, 0)), lbm.WALL, 0, 0, 0, 0], "below 1"),
])
def test_create_rejects_faces(faces, msg):
    h = lbm.lib().lbm_create(lbm.D3Q19, 8, 8, 8, 0.8, _bc(faces))
    assert not h
    assert msg in lbm.last_error()


def test_open_axis_needs_two_cells():
    faces = [(lbm.ZOUHE_VELOCITY, (0.01, 0, 0)), lbm.EQ_OUTFLOW, lbm.WALL, lbm.WALL, 0, 0]
    assert not lbm.lib().lbm_create(lbm.D3Q19, 1, 8, 8, 0.8, _bc(faces))
    assert ">= 2 cells" in lbm.last_error()


def test_2d_rejects_z_velocity():
    faces = [0, 0, lbm.WALL, (lbm.WALL, (0.05, 0, 0.01)), 0, 0]
    assert not lbm.lib().lbm_create(lbm.D2Q9, 8, 8, 0, 0.8, _bc(faces))
    assert "z velocity" in lbm.last_error()


def test_create_and_options_without_device():
    """lbm_create does no device work, so it succeeds on a host without a GPU;
    option checks also run before any device call."""
    L = lbm.lib()
    faces = [lbm.WALL] * 5 + [(lbm.WALL, (0.05, 0, 0))]
    h = L.lbm_create(lbm.D3Q19, 16, 16, 16, 0.55, _bc(faces))
    assert h
    h = ctypes.c_void_p(h)
    bad = lbm.lbm_options(9, lbm.F32, lbm.INPLACE, 0, 1.0)
    assert L.lbm_set_options(h, ctypes.byref(bad)) == lbm.LBM_EINVAL
    bad = lbm.lbm_options(lbm.F16, lbm.F64, lbm.INPLACE, 0, 1.0)
    assert L.lbm_set_options(h, ctypes.byref(bad)) == lbm.LBM_EUNSUPPORTED
    bad = lbm.lbm_options(lbm.F32, lbm.F32, 5, 0, 1.0)
    assert L.lbm_set_options(h, ctypes.byref(bad)) == lbm.LBM_EINVAL
    bad = lbm.lbm_options(lbm.F32, lbm.F32, lbm.INPLACE, 0, -1.0)
    assert L.lbm_set_options(h, ctypes.byref(bad)) == lbm.LBM_EINVAL
    ok = lbm.lbm_options(lbm.F32, lbm.F32, lbm.PULL, 0, 1.0)
    assert L.lbm_set_options(h, ctypes.byref(ok)) == lbm.LBM_OK
    ok = lbm.lbm_options(lbm.BF16, lbm.F32, lbm.DOUBLE, 0, 1.0)
    assert L.lbm_set_options(h, ctypes.byref(ok)) == lbm.LBM_OK
    # state-dependent calls before init
    assert L.lbm_step(h, 1) == lbm.LBM_ESTATE
    assert L.lbm_step(h, -1) == lbm.LBM_EINVAL
    assert L.lbm_moments(h, None, None, lbm.F32, None) == lbm.LBM_ESTATE
    assert L.lbm_backward(h, None, None, lbm.F32, None, None, None) == lbm.LBM_ESTATE
    assert L.lbm_capture_graph(h, 0) == lbm.LBM_EINVAL
    assert L.lbm_graph_launch(h) == lbm.LBM_ESTATE
    assert L.lbm_time(h) == 0
    assert L.lbm_state_bytes(h) > 19 * 16 ** 3 * 2
    L.lbm_destroy(h)


def test_null_context_everywhere():
    L = lbm.lib()
    assert L.lbm_step(None, 1) == lbm.LBM_EINVAL
    assert L.lbm_set_stream(None, None) == lbm.LBM_EINVAL
    assert L.lbm_moments(None, None, None, lbm.F32, None) == lbm.LBM_EINVAL
    assert L.lbm_sync(None) == lbm.LBM_EINVAL
    assert L.lbm_tape_end(None) == lbm.LBM_EINVAL
    assert L.lbm_time(None) == -1
    L.lbm_destroy(None)


def test_copy_probe_rejects_misaligned():
    L = lbm.lib()
    assert L.lbm_copy_probe(ctypes.c_void_p(16), ctypes.c_void_p(32), 17, None) == lbm.LBM_EINVAL
    assert L.lbm_copy_probe(None, ctypes.c_void_p(32), 16, None) == lbm.LBM_EINVAL


def test_binding_raises_on_bad_create():
    with pytest.raises(lbm.LbmError):
        lbm.Sim("D3Q19", (8, 8, 8), tau=0.4)


def test_force_collision_and_face_checks_without_device():
    """lbm_set_force / lbm_set_collision validate and record on the host; a set
    field pins the compute type; regularized face types are accepted."""
    L = lbm.lib()
    h = ctypes.c_void_p(L.lbm_create(lbm.D3Q19, 8, 8, 8, 0.7, None))
    assert h
    nan3 = (ctypes.c_double * 3)(float("nan"), 0.0, 0.0)
    assert L.lbm_set_force(h, nan3, None, 1.0) == lbm.LBM_EINVAL
    ok3 = (ctypes.c_double * 3)(1e-5, 0.0, 0.0)
    assert L.lbm_set_force(h, ok3, None, float("inf")) == lbm.LBM_EINVAL
    # a (never dereferenced) field pointer: the compute type is now fixed
    assert L.lbm_set_force(h, ok3, ctypes.c_void_p(4096), 1.0) == lbm.LBM_OK
    f64 = lbm.lbm_options(lbm.F64, lbm.F64, lbm.INPLACE, 0, 1.0)
    assert L.lbm_set_options(h, ctypes.byref(f64)) == lbm.LBM_ESTATE
    f16 = lbm.lbm_options(lbm.F16, lbm.F32, lbm.INPLACE, 0, 1.0)
    assert L.lbm_set_options(h, ctypes.byref(f16)) == lbm.LBM_OK
    assert L.lbm_set_force(h, None, None, 1.0) == lbm.LBM_OK          # off
    assert L.lbm_set_options(h, ctypes.byref(f64)) == lbm.LBM_OK
    assert L.lbm_set_collision(h, lbm.KBC) == lbm.LBM_EUNSUPPORTED      # D3Q19
    assert L.lbm_set_collision(h, 3) == lbm.LBM_EINVAL
    assert L.lbm_set_collision(h, lbm.BGK) == lbm.LBM_OK
    L.lbm_destroy(h)
    h = ctypes.c_void_p(L.lbm_create(lbm.D3Q27, 8, 8, 8, 0.7, None))
    assert L.lbm_set_collision(h, lbm.KBC) == lbm.LBM_OK
    L.lbm_destroy(h)
    faces = [(lbm.REG_VELOCITY, (0.02, 0, 0)), (lbm.REG_PRESSURE, (0, 0, 0), 1.0), lbm.WALL, lbm.WALL, 0, 0]
    h = L.lbm_create(lbm.D3Q19, 8, 8, 8, 0.7, _bc(faces))
    assert h
    L.lbm_destroy(ctypes.c_void_p(h))
    bad = [(lbm.REG_PRESSURE, (0, 0, 0), 0.0), lbm.WALL, 0, 0, 0, 0]
    assert not L.lbm_create(lbm.D3Q19, 8, 8, 8, 0.7, _bc(bad))
    assert "density" in lbm.last_error()
    assert not L.lbm_create(lbm.D3Q19, 8, 8, 8, 0.7, _bc([(7,), lbm.WALL, 0, 0, 0, 0]))
    assert "unknown boundary type" in lbm.last_error()


def test_tape_id_without_device():
    """lbm_tape_id: -1 for NULL, 0 while no tape is held (no device work)."""
    L = lbm.lib()
    assert L.lbm_tape_id(None) == -1
    h = L.lbm_create(lbm.D2Q9, 8, 8, 0, 0.8, None)
    assert h
    try:
        assert L.lbm_tape_id(h) == 0
    finally:
        L.lbm_destroy(h)


@pytest.mark.parametrize("lat,q", [(lbm.D2Q9, 9), (lbm.D3Q19, 19), (lbm.D3Q27, 27)])
def test_lattice_info_matches_the_figure(lat, q):
    """lbm_lattice_info (no device work) reports the paper's vector order
    (tests/golden/lattice_vectors.txt) and weights that sum to one with
    sum_i w_i c_ia c_ib = delta_ab / 3 in exact rationals."""
    from fractions import Fraction
    c, w = lbm.lattice_info(lat)
    assert c.shape == (q, 3)
    rows = []
    with open(os.path.join(ROOT, "tests", "golden", "lattice_vectors.txt")) as fh:
        for line in fh:
            v = line.split()
            if v and not v[0].startswith("#") and int(v[0]) == q:
                rows.append([int(x) for x in v[1:4]])
    ref = np.array(rows)
    assert ref.shape == (q, 3)
    assert np.array_equal(c, ref)
    W = [Fraction(x).limit_denominator(1000) for x in w]
    assert sum(W) == 1
    for a in range(3 if q != 9 else 2):
        for b in range(3 if q != 9 else 2):
            assert sum(W[i] * int(c[i, a]) * int(c[i, b]) for i in range(q)) == (Fraction(1, 3) if a == b else 0)
    assert lbm.lib().lbm_lattice_info(7, None, None) == lbm.LBM_EINVAL

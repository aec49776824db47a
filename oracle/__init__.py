"""FP64 CPU oracle of the lattice Boltzmann step -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  The GPU library never uses it and shares no code with
it.  The arithmetic lives in ``lbm_oracle.c`` (plain C, FP64, double-buffered,
array-of-structures ``f[x, y, z, i]`` as in the paper's array representation,
Sec. 3.3); this module only marshals numpy arrays to it and adds the loss seeds
used by the adjoint checks.

Every function that carries arithmetic cites the paper passage it follows in the
C source.  Functions without an independent pin are marked "parity unpinned"
there and in the design notes (none at present).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB = os.path.join(_HERE, "liblbm_oracle.so")

PERIODIC, WALL, ZOUHE_VEL, ZOUHE_PRES, OUTFLOW, REG_VEL, REG_PRES = 0, 1, 2, 3, 4, 5, 6
BGK, KBC = 0, 1
FACE_NAMES = ("-x", "+x", "-y", "+y", "-z", "+z")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP contraction off, OpenMP on)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
               "-shared", "-std=c11", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Face(ctypes.Structure):
    _fields_ = [("type", ctypes.c_int), ("u", ctypes.c_double * 3), ("rho", ctypes.c_double)]


class _Sim(ctypes.Structure):
    _fields_ = [("q", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("tau", ctypes.c_double), ("rho0", ctypes.c_double), ("face", _Face * 6),
                ("solid", ctypes.c_void_p), ("s", ctypes.c_void_p), ("force", ctypes.c_double * 3),
                ("edm", ctypes.c_void_p), ("collision", ctypes.c_int), ("qlink", ctypes.c_void_p),
                ("bouzidi_order", ctypes.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        dp = P(ctypes.c_double)
        L.orc_tables.argtypes = [ctypes.c_int, P(ctypes.c_int), dp, P(ctypes.c_int)]
        L.orc_equilibrium.argtypes = [ctypes.c_int, ctypes.c_double, dp, dp]
        L.orc_cell_moments.argtypes = [ctypes.c_int, dp, dp, dp]
        L.orc_collide_cell.argtypes = [P(_Sim), dp, dp]
        L.orc_zouhe_closure.argtypes = [P(_Sim), ctypes.c_int, dp]
        L.orc_run.argtypes = [P(_Sim), dp, ctypes.c_int]
        L.orc_run.restype = ctypes.c_int
        L.orc_init_equilibrium.argtypes = [P(_Sim), ctypes.c_void_p, ctypes.c_void_p, dp]
        L.orc_moments.argtypes = [P(_Sim), dp, dp, dp]
        L.orc_sums.argtypes = [P(_Sim), dp, dp]
        L.orc_forces.argtypes = [P(_Sim), dp, dp]
        L.orc_step_forces.argtypes = [P(_Sim), dp, dp]
        L.orc_step_forces.restype = ctypes.c_int
        L.orc_adjoint_step.argtypes = [P(_Sim), dp, dp, dp, ctypes.c_void_p, dp, dp, ctypes.c_void_p]
        L.orc_adjoint_step.restype = ctypes.c_int
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_set_num_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def tables(q: int):
    """(c[q,3] int, w[q] float64, opp[q] int) of the oracle's lattice."""
    c = (ctypes.c_int * (3 * q))()
    w = np.zeros(q)
    o = (ctypes.c_int * q)()
    if lib().orc_tables(q, c, _dp(w), o) != 0:
        raise ValueError(f"unknown lattice q={q}")
    return np.array(list(c), dtype=np.int64).reshape(q, 3), w, np.array(list(o), dtype=np.int64)


def equilibrium(q: int, rho: float, u: Sequence[float]) -> np.ndarray:
    feq = np.zeros(q)
    uu = np.ascontiguousarray(np.array(list(u) + [0.0] * (3 - len(u)), dtype=np.float64))
    lib().orc_equilibrium(q, float(rho), _dp(uu), _dp(feq))
    return feq


def cell_moments(f: np.ndarray):
    f = np.ascontiguousarray(f, dtype=np.float64)
    r = np.zeros(1)
    u = np.zeros(3)
    lib().orc_cell_moments(f.shape[0], _dp(f), _dp(r), _dp(u))
    return float(r[0]), u


@dataclass
class Face:
    type: int = PERIODIC
    u: tuple = (0.0, 0.0, 0.0)
    rho: float = 1.0


def periodic_faces():
    return [Face() for _ in range(6)]


@dataclass
class Sim:
    """An oracle problem: lattice q, grid, tau, faces (-x,+x,-y,+y,-z,+z)."""
    q: int
    nx: int
    ny: int
    nz: int = 1
    tau: float = 0.8
    faces: list = field(default_factory=periodic_faces)
    rho0: float = 1.0
    solid: Optional[np.ndarray] = None     # (nx,ny,nz) uint8
    s: Optional[np.ndarray] = None         # (nx,ny,nz) float64 solid fraction
    force: tuple = (0.0, 0.0, 0.0)
    edm: Optional[np.ndarray] = None       # (nx,ny,nz,3) body force, exact-difference method
    collision: int = 0                     # 0 BGK, 1 KBC (D2Q9 / D3Q27)
    qlink: Optional[np.ndarray] = None     # (nx,ny,nz,q) curved-wall fractions of links into solids (0 = halfway)
    bouzidi_order: int = 1                 # 1 linear, 2 quadratic interpolated bounce-back

    @property
    def shape(self):
        return (self.nx, self.ny, self.nz)

    @property
    def N(self):
        return self.nx * self.ny * self.nz

    def _struct(self):
        st = _Sim()
        st.q, st.nx, st.ny, st.nz = self.q, self.nx, self.ny, self.nz
        st.tau, st.rho0 = float(self.tau), float(self.rho0)
        for k, F in enumerate(self.faces):
            st.face[k].type = int(F.type)
            uu = list(F.u) + [0.0] * (3 - len(F.u))
            for a in range(3):
                st.face[k].u[a] = float(uu[a])
            st.face[k].rho = float(F.rho)
        self._keep = []
        if self.solid is not None:
            sol = np.ascontiguousarray(self.solid, dtype=np.uint8).reshape(-1)
            self._keep.append(sol)
            st.solid = sol.ctypes.data
        else:
            st.solid = None
        if self.s is not None:
            sv = np.ascontiguousarray(self.s, dtype=np.float64).reshape(-1)
            self._keep.append(sv)
            st.s = sv.ctypes.data
        else:
            st.s = None
        ff = list(self.force) + [0.0] * (3 - len(self.force))
        for a in range(3):
            st.force[a] = float(ff[a])
        if self.edm is not None:
            e = np.zeros(self.shape + (3,))
            ev = np.asarray(self.edm, dtype=np.float64).reshape(self.shape + (-1,))
            e[..., : ev.shape[-1]] = ev
            e = np.ascontiguousarray(e).reshape(-1)
            self._keep.append(e)
            st.edm = e.ctypes.data
        else:
            st.edm = None
        st.collision = int(self.collision)
        if self.qlink is not None:
            ql = np.ascontiguousarray(self.qlink, dtype=np.float64).reshape(-1)
            assert ql.size == self.N * self.q
            self._keep.append(ql)
            st.qlink = ql.ctypes.data
        else:
            st.qlink = None
        st.bouzidi_order = int(self.bouzidi_order)
        return st

    # --- state ---------------------------------------------------------------
    def equilibrium_state(self, rho=None, u=None) -> np.ndarray:
        """f = feq(rho, u): rho (nx,ny,nz) or None (rho0), u (nx,ny,nz,D<=3) or None (0)."""
        f = np.zeros(self.shape + (self.q,))
        st = self._struct()
        rp = None
        up = None
        if rho is not None:
            rr = np.ascontiguousarray(np.broadcast_to(rho, self.shape), dtype=np.float64)
            rp = rr.ctypes.data
        if u is not None:
            u = np.asarray(u, dtype=np.float64)
            uu = np.zeros(self.shape + (3,))
            uu[..., : u.shape[-1]] = u
            uu = np.ascontiguousarray(uu)
            up = uu.ctypes.data
        lib().orc_init_equilibrium(ctypes.byref(st), rp, up, _dp(f))
        return f

    def run(self, f: np.ndarray, nsteps: int) -> np.ndarray:
        """Advance f (in place) by nsteps; returns f."""
        assert f.shape == self.shape + (self.q,) and f.dtype == np.float64 and f.flags["C_CONTIGUOUS"]
        st = self._struct()
        if lib().orc_run(ctypes.byref(st), _dp(f), int(nsteps)) != 0:
            raise MemoryError("oracle allocation failed")
        return f

    def moments(self, f: np.ndarray):
        """(rho (nx,ny,nz), u (nx,ny,nz,3)); solid cells report rho0 and 0."""
        st = self._struct()
        rho = np.zeros(self.shape)
        u = np.zeros(self.shape + (3,))
        lib().orc_moments(ctypes.byref(st), _dp(np.ascontiguousarray(f)), _dp(rho), _dp(u))
        return rho, u

    def sums(self, f: np.ndarray) -> np.ndarray:
        """[mass, Px, Py, Pz, KE] over fluid cells (Kahan-summed)."""
        st = self._struct()
        out = np.zeros(5)
        lib().orc_sums(ctypes.byref(st), _dp(np.ascontiguousarray(f)), _dp(out))
        return out

    def forces(self, f: np.ndarray):
        """Momentum-exchange force of the step that produced f: (force on the
        solid cells [3], force on each wall face [6, 3])."""
        st = self._struct()
        out = np.zeros(21)
        lib().orc_forces(ctypes.byref(st), _dp(np.ascontiguousarray(f)), _dp(out))
        return out[:3].copy(), out[3:].reshape(6, 3).copy()

    def step_forces(self, f: np.ndarray):
        """Advance f (in place) by one step; return the momentum-exchange force of
        that step from the post-collision and new populations (Mei et al.):
        (force on the solid cells [3], force on each wall face [6, 3])."""
        assert f.shape == self.shape + (self.q,) and f.dtype == np.float64 and f.flags["C_CONTIGUOUS"]
        st = self._struct()
        out = np.zeros(21)
        if lib().orc_step_forces(ctypes.byref(st), _dp(f), _dp(out)) != 0:
            raise MemoryError("oracle allocation failed")
        return out[:3].copy(), out[3:].reshape(6, 3).copy()

    def links_to_qlink(self, cells, dirs, q):
        """Dense (nx,ny,nz,q) wall-fraction array from a link list (flat cell
        index, direction, fraction)."""
        ql = np.zeros(self.N * self.q)
        ql[np.asarray(cells, dtype=np.int64) * self.q + np.asarray(dirs, dtype=np.int64)] = np.asarray(q)
        return ql.reshape(self.shape + (self.q,))

    def collide_cell(self, f_cell: np.ndarray) -> np.ndarray:
        st = self._struct()
        out = np.zeros(self.q)
        lib().orc_collide_cell(ctypes.byref(st), _dp(np.ascontiguousarray(f_cell, dtype=np.float64)), _dp(out))
        return out

    def zouhe_closure(self, face: int, f_cell: np.ndarray) -> np.ndarray:
        st = self._struct()
        out = np.ascontiguousarray(np.array(f_cell, dtype=np.float64))
        lib().orc_zouhe_closure(ctypes.byref(st), int(face), _dp(out))
        return out

    def adjoint_step(self, f_t: np.ndarray, a_next: np.ndarray, with_force: bool = False):
        """Adjoint of one step at state f_t: returns (a_t, dL/ds, dL/dtau, dL/du_w[6,3])
        (+ dL/dF [*shape, 3] of the body force field if with_force)."""
        st = self._struct()
        a_out = np.zeros_like(a_next)
        dlds = np.zeros(self.N)
        dtau = np.zeros(1)
        duw = np.zeros(18)
        dldf = np.zeros(self.N * 3)
        rc = lib().orc_adjoint_step(ctypes.byref(st), _dp(np.ascontiguousarray(f_t)),
                                    _dp(np.ascontiguousarray(a_next)), _dp(a_out),
                                    dlds.ctypes.data if self.s is not None else None,
                                    _dp(dtau), _dp(duw), dldf.ctypes.data)
        if rc != 0:
            raise MemoryError("oracle allocation failed")
        out = (a_out, dlds.reshape(self.shape), float(dtau[0]), duw.reshape(6, 3))
        if with_force:
            out = out + (dldf.reshape(self.shape + (3,)),)
        return out

    # --- loss seeds (adjoint inputs) -------------------------------------------
    def seed_from_velocity_grad(self, f: np.ndarray, g_u: np.ndarray, g_rho=None) -> np.ndarray:
        """dL/df_i = g_rho + sum_a g_u[a] (c_ia - u_a)/rho, from u = sum c f / rho (eq. velocity)."""
        c, _, _ = tables(self.q)
        rho, u = self.moments(f)
        g = np.zeros(self.shape + (3,))
        g[..., : g_u.shape[-1]] = g_u
        a = np.einsum("xyza,ia->xyzi", g, c.astype(np.float64)) - np.sum(g * u, axis=-1)[..., None]
        a = a / rho[..., None]
        if g_rho is not None:
            a = a + np.asarray(g_rho)[..., None]
        if self.solid is not None:
            a[self.solid.astype(bool)] = 0.0
        return np.ascontiguousarray(a)

    def trajectory(self, f0: np.ndarray, nsteps: int):
        """States f(0..nsteps) (list of arrays)."""
        states = [f0.copy()]
        f = f0.copy()
        for _ in range(nsteps):
            self.run(f, 1)
            states.append(f.copy())
        return states

    def adjoint(self, states, a_final, with_force: bool = False):
        """Run the adjoint back through the trajectory: (a(0), dL/ds, dL/dtau, dL/du_w)
        (+ dL/dF [*shape, 3] of the body force field if with_force)."""
        a = a_final
        dlds = np.zeros(self.shape)
        dtau = 0.0
        duw = np.zeros((6, 3))
        dldf = np.zeros(self.shape + (3,))
        for t in range(len(states) - 2, -1, -1):
            a, ds, dt, du, df = self.adjoint_step(states[t], a, with_force=True)
            dlds += ds
            dtau += dt
            duw += du
            dldf += df
        if with_force:
            return a, dlds, dtau, duw, dldf
        return a, dlds, dtau, duw


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the following oracle calls (timing only; results do not depend on it)."""
    lib().orc_set_num_threads(int(n))

"""Python binding of liblbm.so (the C-ABI in include/lbm.h).

Argument marshalling only: every step of the lattice Boltzmann path runs in the
HIP kernels of liblbm.so.  PyTorch provides device memory (caller buffers are
torch tensors) and the HIP stream (the current torch stream).  There is no
fallback: if the library is missing or the call fails, an exception is raised.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")

# ---- constants (include/lbm.h) ------------------------------------------------
LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_ESTATE, LBM_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
D2Q9, D3Q19, D3Q27 = 0, 1, 2
PERIODIC, WALL, ZOUHE_VELOCITY, ZOUHE_PRESSURE, EQ_OUTFLOW, REG_VELOCITY, REG_PRESSURE = 0, 1, 2, 3, 4, 5, 6
BGK, KBC = 0, 1
F64, F32, F16, BF16 = 0, 1, 2, 3
INPLACE, DOUBLE, PULL = 0, 1, 2

LATTICES = {"D2Q9": D2Q9, "D3Q19": D3Q19, "D3Q27": D3Q27}
STORAGE = {"f64": F64, "f32": F32, "f16": F16, "bf16": BF16}
PATTERNS = {"inplace": INPLACE, "double": DOUBLE, "pull": PULL}
Q_OF = {D2Q9: 9, D3Q19: 19, D3Q27: 27}
D_OF = {D2Q9: 2, D3Q19: 3, D3Q27: 3}


class lbm_face(ctypes.Structure):
    _fields_ = [("type", ctypes.c_int32), ("reserved", ctypes.c_int32), ("u", ctypes.c_double * 3),
                ("rho", ctypes.c_double)]


class lbm_bc(ctypes.Structure):
    _fields_ = [("face", lbm_face * 6)]


class lbm_options(ctypes.Structure):
    _fields_ = [("storage", ctypes.c_int32), ("compute", ctypes.c_int32), ("pattern", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("rho0", ctypes.c_double)]


# every symbol the header declares: name -> (restype, argtypes)
_vp, _i, _d, _sz, _i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t, ctypes.c_int64
_ip, _dp = ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)
SIGNATURES = {
    "lbm_last_error": (ctypes.c_char_p, []),
    "lbm_version": (ctypes.c_char_p, []),
    "lbm_lattice_info": (_i, [_i, ctypes.POINTER(ctypes.c_int32), _dp]),
    "lbm_set_curved_links": (_i, [_vp, _i64, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32), _dp, _i]),
    "lbm_create": (_vp, [_i, _i, _i, _i, _d, ctypes.POINTER(lbm_bc)]),
    "lbm_create_batch": (_vp, [_i, _i, _ip, _ip, _ip, _dp, ctypes.POINTER(lbm_bc)]),
    "lbm_batch_offsets": (_i, [_vp, ctypes.POINTER(ctypes.c_int64)]),
    "lbm_batch_tuning": (_i, [_vp, _i, _i]),
    "lbm_batch_config": (_i, [_vp, _ip, _ip]),
    "lbm_destroy": (None, [_vp]),
    "lbm_set_options": (_i, [_vp, ctypes.POINTER(lbm_options)]),
    "lbm_set_params": (_i, [_vp, _d, ctypes.POINTER(lbm_bc)]),
    "lbm_set_stream": (_i, [_vp, _vp]),
    "lbm_set_solid": (_i, [_vp, _vp, _i]),
    "lbm_set_solid_fraction": (_i, [_vp, _vp, _i]),
    "lbm_init_equilibrium": (_i, [_vp, _vp, _vp, _i]),
    "lbm_step": (_i, [_vp, _i]),
    "lbm_time": (_i64, [_vp]),
    "lbm_moments": (_i, [_vp, _vp, _vp, _i, _dp]),
    "lbm_forces": (_i, [_vp, _dp]),
    "lbm_forces_noalloc": (_i, [_vp, _vp]),
    "lbm_set_force": (_i, [_vp, _dp, _vp, ctypes.c_double]),
    "lbm_set_collision": (_i, [_vp, _i]),
    "lbm_tape_begin": (_i, [_vp, _i, _i]),
    "lbm_tape_end": (_i, [_vp]),
    "lbm_tape_free": (_i, [_vp]),
    "lbm_tape_id": (_i64, [_vp]),
    "lbm_backward": (_i, [_vp, _vp, _vp, _i, _vp, _dp, _dp]),
    "lbm_backward_force": (_i, [_vp, _vp, _vp, _i, _vp, _dp, _dp, _vp, _dp]),
    "lbm_capture_graph": (_i, [_vp, _i]),
    "lbm_graph_launch": (_i, [_vp]),
    "lbm_state_bytes": (_sz, [_vp]),
    "lbm_save": (_i, [_vp, _vp, _sz]),
    "lbm_load": (_i, [_vp, _vp, _sz]),
    "lbm_sync": (_i, [_vp]),
    "lbm_copy_probe": (_i, [_vp, _vp, _sz, _vp]),
}

_lib = None


class LbmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


def lib() -> ctypes.CDLL:
    """Load liblbm.so (built in-tree); raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python paper_2311_16080_amd/build.py`")
        # PyTorch-ROCm carries its own HIP runtime.  Loading torch first makes
        # liblbm.so bind to that same runtime (same soname), so the library and
        # torch share one HIP/HSA instance, devices and streams; loading
        # liblbm.so first would bring a second runtime into the process.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def last_error() -> str:
    return lib().lbm_last_error().decode()


def check(rc: int) -> None:
    if rc != LBM_OK:
        raise LbmError(rc, last_error())


def lattice_info(lattice):
    """(c [Q, 3] int, w [Q] float64) of the library's velocity set, caller axes."""
    lat = LATTICES[lattice] if isinstance(lattice, str) else int(lattice)
    Q = Q_OF[lat]
    c = (ctypes.c_int32 * (3 * Q))()
    w = (ctypes.c_double * Q)()
    n = lib().lbm_lattice_info(lat, c, w)
    if n != Q:
        raise LbmError(n, last_error())
    return np.array(list(c), dtype=np.int64).reshape(Q, 3), np.array(list(w))


def make_bc(faces) -> lbm_bc:
    """faces: 6 entries (-x,+x,-y,+y,-z,+z), each an int type or a tuple
    (type, u=(ux,uy,uz), rho=1.0)."""
    bc = lbm_bc()
    for k in range(6):
        F = faces[k] if k < len(faces) else PERIODIC
        if isinstance(F, int):
            F = (F,)
        t = int(F[0])
        u = tuple(F[1]) if len(F) > 1 else (0.0, 0.0, 0.0)
        u = tuple(u) + (0.0,) * (3 - len(u))
        rho = float(F[2]) if len(F) > 2 else 1.0
        bc.face[k].type = t
        for a in range(3):
            bc.face[k].u[a] = float(u[a])
        bc.face[k].rho = rho
    return bc


def _torch():
    import torch
    return torch


def _ptr(t) -> Optional[int]:
    return None if t is None else int(t.data_ptr())


class Sim:
    """One lattice Boltzmann domain on the current GPU (wraps an lbm_ctx)."""

    def __init__(self, lattice, shape: Sequence[int], tau: float, faces=None, storage: str = "f32",
                 pattern: str = "inplace", rho0: float = 1.0):
        self.lattice = LATTICES[lattice] if isinstance(lattice, str) else int(lattice)
        self.Q = Q_OF[self.lattice]
        self.D = D_OF[self.lattice]
        shape = tuple(int(s) for s in shape)
        if self.D == 2:
            shape = shape[:2]
            nz = 0
        else:
            nz = shape[2]
        self.shape = shape
        self.N = int(np.prod(shape))
        self.tau = float(tau)
        self.storage = storage
        bc = make_bc(faces) if faces is not None else None
        self._bc = bc
        h = lib().lbm_create(self.lattice, shape[0], shape[1], nz, self.tau,
                             ctypes.byref(bc) if bc is not None else None)
        if not h:
            raise LbmError(LBM_EINVAL, last_error())
        self.h = ctypes.c_void_p(h)
        opt = lbm_options(STORAGE[storage], F64 if storage == "f64" else F32, PATTERNS[pattern], 0, float(rho0))
        check(lib().lbm_set_options(self.h, ctypes.byref(opt)))
        self._keep = []

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            try:
                lib().lbm_destroy(h)
            except Exception:
                pass
            self.h = None

    # ---- setup ---------------------------------------------------------------
    def set_params(self, tau: Optional[float] = None, faces=None):
        """Change tau and/or the faces' velocities and densities (same types)."""
        tau = self.tau if tau is None else float(tau)
        bc = make_bc(faces) if faces is not None else None
        check(lib().lbm_set_params(self.h, tau, ctypes.byref(bc) if bc is not None else None))
        self.tau = tau
        if bc is not None:
            self._bc = bc

    def use_current_stream(self):
        torch = _torch()
        check(lib().lbm_set_stream(self.h, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))

    def set_solid(self, mask):
        """mask: array/tensor of shape `shape`, nonzero = solid (host or device)."""
        torch = _torch()
        if mask is None:
            check(lib().lbm_set_solid(self.h, None, 0))
            return
        if isinstance(mask, torch.Tensor) and mask.is_cuda:
            m = mask.to(torch.uint8).contiguous()
            self._keep.append(m)
            check(lib().lbm_set_solid(self.h, ctypes.c_void_p(m.data_ptr()), 1))
        else:
            m = np.ascontiguousarray(np.asarray(mask).reshape(self.shape), dtype=np.uint8)
            check(lib().lbm_set_solid(self.h, m.ctypes.data_as(ctypes.c_void_p), 0))

    def set_curved_links(self, cells, dirs, q, order: int = 1):
        """Interpolated bounce-back on links (cells[k], dirs[k]) into solid cells
        cut by the wall at fraction q[k] (host arrays; flat caller-order cells,
        lattice_info direction order); order 1 linear, 2 quadratic.  Empty
        arrays clear the links."""
        cells = np.ascontiguousarray(np.asarray(cells, dtype=np.int64).reshape(-1))
        dirs = np.ascontiguousarray(np.asarray(dirs, dtype=np.int32).reshape(-1))
        q = np.ascontiguousarray(np.asarray(q, dtype=np.float64).reshape(-1))
        if not (cells.size == dirs.size == q.size):
            raise ValueError("cells, dirs and q must have the same length")
        P = ctypes.POINTER
        check(lib().lbm_set_curved_links(self.h, int(cells.size), cells.ctypes.data_as(P(ctypes.c_int64)),
                                         dirs.ctypes.data_as(P(ctypes.c_int32)),
                                         q.ctypes.data_as(P(ctypes.c_double)), int(order)))

    def set_solid_fraction(self, s):
        torch = _torch()
        if s is None:
            check(lib().lbm_set_solid_fraction(self.h, None, 0))
            return
        if isinstance(s, torch.Tensor) and s.is_cuda:
            t = s.to(torch.float32).contiguous()
            self._keep.append(t)
            check(lib().lbm_set_solid_fraction(self.h, ctypes.c_void_p(t.data_ptr()), 1))
        else:
            a = np.ascontiguousarray(np.asarray(s).reshape(self.shape), dtype=np.float32)
            check(lib().lbm_set_solid_fraction(self.h, a.ctypes.data_as(ctypes.c_void_p), 0))

    def init_equilibrium(self, rho=None, u=None):
        """rho: tensor `shape`; u: tensor (D, *shape) -- device, float32/float64."""
        torch = _torch()
        dt = F64
        if rho is not None:
            rho = rho.contiguous()
            dt = F64 if rho.dtype == torch.float64 else F32
        if u is not None:
            u = u.contiguous()
            dt = F64 if u.dtype == torch.float64 else F32
            if rho is not None and rho.dtype != u.dtype:
                rho = rho.to(u.dtype)
        self._keep = [x for x in (rho, u) if x is not None] + self._keep[-2:]
        check(lib().lbm_init_equilibrium(self.h, _ptr(rho), _ptr(u), dt))

    # ---- run -------------------------------------------------------------------
    def step(self, n: int = 1):
        check(lib().lbm_step(self.h, int(n)))

    @property
    def t(self) -> int:
        return int(lib().lbm_time(self.h))

    def moments(self, dtype=None, sums: bool = False):
        """(rho [shape], u [D, *shape]) device tensors (+ host sums [5] if sums)."""
        torch = _torch()
        dtype = dtype or (torch.float64 if self.storage == "f64" else torch.float32)
        rho = torch.empty(self.shape, dtype=dtype, device="cuda")
        u = torch.empty((self.D,) + self.shape, dtype=dtype, device="cuda")
        out = (ctypes.c_double * 5)()
        check(lib().lbm_moments(self.h, _ptr(rho), _ptr(u), F64 if dtype == torch.float64 else F32,
                                out if sums else None))
        if sums:
            return rho, u, np.array(list(out))
        return rho, u

    def sums(self) -> np.ndarray:
        out = (ctypes.c_double * 5)()
        check(lib().lbm_moments(self.h, None, None, F64, out))
        return np.array(list(out))

    def set_collision(self, model):
        """"BGK" / "KBC" (or LBM_BGK / LBM_KBC) for the following steps."""
        m = {"BGK": BGK, "KBC": KBC}.get(model, model) if isinstance(model, str) else int(model)
        check(lib().lbm_set_collision(self.h, m))

    def set_force(self, force=None, field=None, eps: float = 1.0):
        """Body force by the exact-difference method for the following steps:
        force = uniform part (D values, caller axes) or None; field = device
        tensor (D, *shape) or None (kept alive here, converted to the compute
        type); eps scales both.  set_force() switches it off."""
        torch = _torch()
        fu = None
        if force is not None:
            v = [float(x) for x in force] + [0.0] * 3
            fu = (ctypes.c_double * 3)(*v[:3])
        fp = None
        self._force_field = None
        if field is not None:
            if not (isinstance(field, torch.Tensor) and field.is_cuda):
                raise TypeError("field must be a device tensor of shape (D, *shape)")
            if tuple(field.shape) != (self.D,) + self.shape:
                raise ValueError(f"field must have shape {(self.D,) + self.shape}")
            t = field.to(torch.float64 if self.storage == "f64" else torch.float32).contiguous()
            self._force_field = t
            fp = ctypes.c_void_p(t.data_ptr())
        check(lib().lbm_set_force(self.h, fu, fp, float(eps)))

    def forces(self):
        """Momentum-exchange force of the last step: (on solid cells [3], on each
        face [6, 3]) in caller axes, FP64."""
        out = (ctypes.c_double * 21)()
        check(lib().lbm_forces(self.h, out))
        a = np.array(list(out))
        return a[:3], a[3:].reshape(6, 3)

    def sync(self):
        check(lib().lbm_sync(self.h))

    def capture_graph(self, n: int):
        check(lib().lbm_capture_graph(self.h, int(n)))

    def graph_launch(self):
        check(lib().lbm_graph_launch(self.h))

    # ---- checkpoint ------------------------------------------------------------
    def save(self) -> bytes:
        n = lib().lbm_state_bytes(self.h)
        buf = ctypes.create_string_buffer(n)
        check(lib().lbm_save(self.h, buf, n))
        return buf.raw

    def load(self, blob: bytes):
        buf = ctypes.create_string_buffer(blob, len(blob))
        check(lib().lbm_load(self.h, buf, len(blob)))

    # ---- adjoint ---------------------------------------------------------------
    def tape_begin(self, K: int, max_steps: int):
        check(lib().lbm_tape_begin(self.h, int(K), int(max_steps)))

    def tape_end(self):
        check(lib().lbm_tape_end(self.h))

    def tape_free(self):
        check(lib().lbm_tape_free(self.h))

    def tape_id(self) -> int:
        """Identity of the current tape (grows with every tape_begin; 0 = none)."""
        return int(lib().lbm_tape_id(self.h))

    def backward(self, dL_drho=None, dL_du=None, want_s: bool = False, n_domains: int = 1):
        """Adjoint of the taped steps seeded by dL/drho, dL/du (device tensors).
        Returns (dL_ds tensor or None, dL_dtau [n_domains], dL_duw [n_domains, 6, 3])."""
        torch = _torch()
        dt = F64
        ref = dL_du if dL_du is not None else dL_drho
        if ref is not None and ref.dtype == torch.float32:
            dt = F32
        if dL_drho is not None:
            dL_drho = dL_drho.to(torch.float64 if dt == F64 else torch.float32).contiguous()
        if dL_du is not None:
            dL_du = dL_du.to(torch.float64 if dt == F64 else torch.float32).contiguous()
        ds = torch.zeros(self.shape, dtype=torch.float32, device="cuda") if want_s else None
        dtau = (ctypes.c_double * n_domains)()
        duw = (ctypes.c_double * (n_domains * 18))()
        check(lib().lbm_backward(self.h, _ptr(dL_drho), _ptr(dL_du), dt, _ptr(ds), dtau, duw))
        return ds, np.array(list(dtau)), np.array(list(duw)).reshape(n_domains, 6, 3)

    def backward_force(self, dL_drho=None, dL_du=None, want_s: bool = False):
        """backward() plus the body-force gradients: returns (dL_ds or None,
        dL_dtau [1], dL_duw [1, 6, 3], dL_dfield tensor (D, *shape), dL_dforce [D])."""
        torch = _torch()
        dt = F64 if self.storage == "f64" else F32
        tdt = torch.float64 if dt == F64 else torch.float32
        if dL_drho is not None:
            dL_drho = dL_drho.to(tdt).contiguous()
        if dL_du is not None:
            dL_du = dL_du.to(tdt).contiguous()
        ds = torch.zeros(self.shape, dtype=torch.float32, device="cuda") if want_s else None
        dfield = torch.empty((self.D,) + self.shape, dtype=tdt, device="cuda")
        dtau = (ctypes.c_double * 1)()
        duw = (ctypes.c_double * 18)()
        dforce = (ctypes.c_double * 3)()
        check(lib().lbm_backward_force(self.h, _ptr(dL_drho), _ptr(dL_du), dt, _ptr(ds), dtau, duw,
                                       _ptr(dfield), dforce))
        return (ds, np.array(list(dtau)), np.array(list(duw)).reshape(1, 6, 3), dfield,
                np.array(list(dforce))[: self.D])


def copy_probe(dst, src, nbytes: int):
    torch = _torch()
    check(lib().lbm_copy_probe(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()), int(nbytes),
                               ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))


class _Rollout:
    """torch.autograd.Function factory (built lazily so importing this module
    does not import torch)."""
    fn = None

    @classmethod
    def get(cls):
        if cls.fn is None:
            torch = _torch()

            class LbmRollout(torch.autograd.Function):
                @staticmethod
                def forward(ctx, s, tau, sim, nsteps, K, rho0, u0, field=None, eps=1.0):
                    sim.set_params(tau=float(tau))
                    if s is not None:
                        sim.set_solid_fraction(s.detach())
                    if field is not None:
                        sim.set_force(None, field.detach(), eps)
                    ctx.has_field = field is not None
                    sim.init_equilibrium(rho0, u0)
                    sim.tape_begin(K, max(int(nsteps), 1))
                    sim.step(int(nsteps))
                    sim.tape_end()
                    rho, u = sim.moments(dtype=torch.float64 if sim.storage == "f64" else torch.float32)
                    ctx.sim = sim
                    ctx.tape_id = sim.tape_id()
                    ctx.has_s = s is not None
                    ctx.tau_dtype = tau.dtype
                    return rho, u

                @staticmethod
                def backward(ctx, g_rho, g_u):
                    sim = ctx.sim
                    if sim.tape_id() != ctx.tape_id:
                        raise LbmError(LBM_ESTATE, "another rollout on this Sim replaced the tape of this one "
                                                   "before its backward pass; use one Sim per rollout in a graph")
                    g_field = None
                    if ctx.has_field:
                        ds, dtau, _, g_field, _ = sim.backward_force(g_rho, g_u, want_s=ctx.has_s)
                    else:
                        ds, dtau, _ = sim.backward(g_rho, g_u, want_s=ctx.has_s)
                    g_tau = torch.tensor(dtau[0], dtype=ctx.tau_dtype)
                    return ds, g_tau, None, None, None, None, None, g_field, None

            cls.fn = LbmRollout
        return cls.fn


def rollout(sim: "Sim", nsteps: int, K: int, s=None, tau=None, rho0=None, u0=None, field=None, eps: float = 1.0):
    """Differentiable run: init at equilibrium(rho0, u0), `nsteps` steps with a
    checkpoint every K steps, returns (rho, u) of the final state.  Gradients
    flow to the solid fraction `s` (device tensor), `tau` (0-d tensor) and a
    body-force field `field` (device tensor (D, *shape), applied with scale eps
    by the exact-difference method) through the library's adjoint.  A given
    field stays set on `sim` afterwards (the backward pass needs it)."""
    torch = _torch()
    if tau is None:
        tau = torch.tensor(sim.tau, dtype=torch.float64)
    return _Rollout.get().apply(s, tau, sim, nsteps, K, rho0, u0, field, float(eps))


class BatchSim:
    """Many independent domains of one lattice advanced together (wraps a
    batch lbm_ctx).  Fields are packed domain after domain: rho [Ntot],
    u [D, Ntot]; `offsets[d]` is the first packed cell of domain d."""

    def __init__(self, lattice, shapes, taus, faces_list=None, storage: str = "f32", rho0: float = 1.0):
        self.lattice = LATTICES[lattice] if isinstance(lattice, str) else int(lattice)
        self.Q = Q_OF[self.lattice]
        self.D = D_OF[self.lattice]
        n = len(shapes)
        self.n = n
        self.shapes = [tuple(int(v) for v in sh)[: self.D] for sh in shapes]
        nx = (ctypes.c_int * n)(*[sh[0] for sh in self.shapes])
        ny = (ctypes.c_int * n)(*[sh[1] for sh in self.shapes])
        nz = (ctypes.c_int * n)(*[(sh[2] if self.D == 3 else 0) for sh in self.shapes])
        self.taus = [float(t) for t in taus]
        tau = (ctypes.c_double * n)(*self.taus)
        bcs = None
        if faces_list is not None:
            bcs = (lbm_bc * n)(*[make_bc(f) for f in faces_list])
        self.storage = storage
        h = lib().lbm_create_batch(self.lattice, n, nx, ny, nz, tau, bcs)
        if not h:
            raise LbmError(LBM_EINVAL, last_error())
        self.h = ctypes.c_void_p(h)
        opt = lbm_options(STORAGE[storage], F64 if storage == "f64" else F32, INPLACE, 0, float(rho0))
        check(lib().lbm_set_options(self.h, ctypes.byref(opt)))
        off = (ctypes.c_int64 * (n + 1))()
        check(lib().lbm_batch_offsets(self.h, off))
        self.offsets = np.array(list(off), dtype=np.int64)
        self.N = int(self.offsets[-1])

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            try:
                lib().lbm_destroy(h)
            except Exception:
                pass
            self.h = None

    def use_current_stream(self):
        torch = _torch()
        check(lib().lbm_set_stream(self.h, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))

    def tuning(self, tile: int = 0, persistent: int = -1):
        check(lib().lbm_batch_tuning(self.h, int(tile), int(persistent)))

    def config(self):
        t, p = ctypes.c_int(), ctypes.c_int()
        check(lib().lbm_batch_config(self.h, ctypes.byref(t), ctypes.byref(p)))
        return t.value, p.value

    def init_equilibrium(self, rho=None, u=None):
        torch = _torch()
        dt = F64
        if u is not None:
            u = u.contiguous()
            dt = F64 if u.dtype == torch.float64 else F32
        if rho is not None:
            rho = rho.contiguous().to(u.dtype if u is not None else rho.dtype)
            dt = F64 if rho.dtype == torch.float64 else F32
        self._keep = [x for x in (rho, u) if x is not None]
        check(lib().lbm_init_equilibrium(self.h, _ptr(rho), _ptr(u), dt))

    def step(self, n: int = 1):
        check(lib().lbm_step(self.h, int(n)))

    @property
    def t(self) -> int:
        return int(lib().lbm_time(self.h))

    def moments(self, dtype=None, sums: bool = False):
        """packed rho [Ntot], u [D, Ntot] (+ per-domain sums [n, 5] if sums)."""
        torch = _torch()
        dtype = dtype or (torch.float64 if self.storage == "f64" else torch.float32)
        rho = torch.empty((self.N,), dtype=dtype, device="cuda")
        u = torch.empty((self.D, self.N), dtype=dtype, device="cuda")
        out = (ctypes.c_double * (5 * self.n))()
        check(lib().lbm_moments(self.h, _ptr(rho), _ptr(u), F64 if dtype == torch.float64 else F32,
                                out if sums else None))
        if sums:
            return rho, u, np.array(list(out)).reshape(self.n, 5)
        return rho, u

    def sums(self) -> np.ndarray:
        out = (ctypes.c_double * (5 * self.n))()
        check(lib().lbm_moments(self.h, None, None, F64, out))
        return np.array(list(out)).reshape(self.n, 5)

    def domain(self, field, d: int):
        """View of domain d in a packed field ([..., Ntot] -> [..., *shape_d])."""
        a, b = int(self.offsets[d]), int(self.offsets[d + 1])
        return field[..., a:b].reshape(field.shape[:-1] + self.shapes[d])

    def capture_graph(self, n: int):
        check(lib().lbm_capture_graph(self.h, int(n)))

    def graph_launch(self):
        check(lib().lbm_graph_launch(self.h))

    def sync(self):
        check(lib().lbm_sync(self.h))

    def tape_begin(self, K: int, max_steps: int):
        check(lib().lbm_tape_begin(self.h, int(K), int(max_steps)))

    def tape_end(self):
        check(lib().lbm_tape_end(self.h))

    def tape_free(self):
        check(lib().lbm_tape_free(self.h))

    def backward(self, dL_drho=None, dL_du=None):
        """Adjoint of the taped steps: (dL_dtau [n], dL_duw [n, 6, 3]); dL_drho
        [Ntot] and dL_du [D, Ntot] are packed like the moments."""
        torch = _torch()
        ref = dL_du if dL_du is not None else dL_drho
        dt = F32 if (ref is not None and ref.dtype == torch.float32) else F64
        tt = torch.float32 if dt == F32 else torch.float64
        if dL_drho is not None:
            dL_drho = dL_drho.to(tt).contiguous()
        if dL_du is not None:
            dL_du = dL_du.to(tt).contiguous()
        dtau = (ctypes.c_double * self.n)()
        duw = (ctypes.c_double * (self.n * 18))()
        check(lib().lbm_backward(self.h, _ptr(dL_drho), _ptr(dL_du), dt, None, dtau, duw))
        return np.array(list(dtau)), np.array(list(duw)).reshape(self.n, 6, 3)

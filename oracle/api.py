"""ctypes wrapper of the C oracle (test infrastructure only)."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)
_lp = C.POINTER(C.c_long)


def load():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            path = _build.build()
        lib = C.CDLL(path)
        lib.orc_new.restype = C.c_void_p
        lib.orc_new.argtypes = [C.c_int, C.c_int, C.c_int, C.c_long, _dp, _ip, C.c_long, C.c_long,
                                _ip, _dp, _dp, _dp, C.c_int]
        for name in ["orc_free", "orc_nstep"]:
            getattr(lib, name).argtypes = [C.c_void_p]
        lib.orc_nstep.restype = C.c_long
        lib.orc_info.argtypes = [C.c_void_p, _dp]
        lib.orc_gll.argtypes = [C.c_void_p, _dp, _dp, _dp]
        lib.orc_lattice.argtypes = [C.c_void_p, _dp, _dp, _ip]
        lib.orc_mass_matrix.argtypes = [C.c_void_p, _dp]
        lib.orc_wall_entries.argtypes = [C.c_void_p, _lp, _dp, _dp]
        lib.orc_lap.argtypes = [C.c_void_p, _dp, _dp, C.c_int]
        lib.orc_mu.argtypes = [C.c_void_p, _dp, _dp]
        lib.orc_avg_grad.argtypes = [C.c_void_p, _dp, _dp]
        lib.orc_stream_op.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp]
        lib.orc_density.argtypes = [C.c_void_p, _dp, _dp]
        lib.orc_collide.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp, _dp]
        lib.orc_step.argtypes = [C.c_void_p, C.c_long]
        lib.orc_set_rho.argtypes = [C.c_void_p, _dp]
        lib.orc_set_f.argtypes = [C.c_void_p, _dp]
        lib.orc_get_f.argtypes = [C.c_void_p, _dp]
        lib.orc_init_tanh.argtypes = [C.c_void_p, _dp, C.c_double, C.c_double, C.c_uint64]
        lib.orc_get_rho.argtypes = [C.c_void_p, _dp]
        lib.orc_get_u.argtypes = [C.c_void_p, _dp]
        lib.orc_diag.argtypes = [C.c_void_p, _dp, _dp]
        lib.orc_splitmix64.argtypes = [C.c_uint64]
        lib.orc_splitmix64.restype = C.c_uint64
        lib.orc_set_threads.argtypes = [C.c_int]
        lib.orc_get_threads.restype = C.c_int
        lib.orc_set_threads(1)
        _lib = lib
    return _lib


def set_threads(n: int) -> int:
    """Host threads of the oracle's element and node loops (results do not depend on it);
    returns the count in use."""
    lib = load()
    lib.orc_set_threads(int(n))
    return lib.orc_get_threads()


def _d(a):
    return a.ctypes.data_as(_dp)


class Oracle:
    """One oracle solve.  ``case`` is a :class:`synth.cases.Case` (or any object with
    the same attributes); ``mode=1`` runs pure advection of every population."""

    def __init__(self, case, mode: int = 0, dt: float | None = None):
        lib = load()
        m = case.mesh
        self.case = case
        self.dim, self.N, self.Q = m.dim, m.N, case.lattice
        self.Ng, self.Nl = m.n_global, m.n_local
        self._xyz = np.ascontiguousarray(m.xyz, dtype=np.float64)
        self._gid = np.ascontiguousarray(m.gid, dtype=np.int32)
        self._wf = np.ascontiguousarray(m.wall_face, dtype=np.int32).reshape(-1)
        self._wc = np.ascontiguousarray(m.wall_cos, dtype=np.float64)
        self._wu = np.ascontiguousarray(m.wall_ub, dtype=np.float64).reshape(-1)
        if self._wf.size == 0:  # keep valid pointers
            self._wf = np.zeros(2, np.int32)
            self._wc = np.zeros(1)
            self._wu = np.zeros(3)
        phys = np.array([case.rho_l, case.rho_v, case.delta, case.sigma, case.tau,
                         case.dt if dt is None else dt, case.cfl,
                         float(getattr(case, "nu", 0.0) or 0.0)], dtype=np.float64)
        self._h = lib.orc_new(self.dim, self.N, self.Q, m.E, _d(self._xyz),
                              self._gid.ctypes.data_as(_ip), self.Ng, m.wall_face.shape[0],
                              self._wf.ctypes.data_as(_ip), _d(self._wc), _d(self._wu), _d(phys),
                              mode)
        if not self._h:
            raise ValueError("oracle rejected the mesh (bad sizes or non-positive Jacobian)")
        info = np.zeros(8)
        lib.orc_info(self._h, _d(info))
        self.dt, self.beta, self.kappa, self.omega, self.hmin = info[:5]
        self.nw = int(info[7])

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.orc_free(self._h)
            self._h = None

    # --- tables -------------------------------------------------------------------------
    def gll(self):
        Np = self.N + 1
        x, w, D = np.zeros(Np), np.zeros(Np), np.zeros((Np, Np))
        load().orc_gll(self._h, _d(x), _d(w), _d(D))
        return x, w, D

    def lattice(self):
        ev, tw, opp = np.zeros((self.Q, 3)), np.zeros(self.Q), np.zeros(self.Q, np.int32)
        load().orc_lattice(self._h, _d(ev), _d(tw), opp.ctypes.data_as(_ip))
        return ev, tw, opp

    def mass_matrix(self):
        MA = np.zeros(self.Ng)
        load().orc_mass_matrix(self._h, _d(MA))
        return MA

    def wall_entries(self):
        wl = np.zeros(max(self.nw, 1), dtype=np.int64)
        wsn = np.zeros((max(self.nw, 1), 3))
        ws = np.zeros(max(self.nw, 1))
        load().orc_wall_entries(self._h, wl.ctypes.data_as(_lp), _d(wsn), _d(ws))
        return wl[:self.nw], wsn[:self.nw], ws[:self.nw]

    # --- operators ----------------------------------------------------------------------
    def lap(self, rho, with_wall=True):
        rho = np.ascontiguousarray(rho, dtype=np.float64)
        out = np.zeros(self.Ng)
        load().orc_lap(self._h, _d(rho), _d(out), int(with_wall))
        return out

    def mu(self, rho):
        rho = np.ascontiguousarray(rho, dtype=np.float64)
        out = np.zeros(self.Ng)
        load().orc_mu(self._h, _d(rho), _d(out))
        return out

    def avg_grad(self, phi):
        phi = np.ascontiguousarray(phi, dtype=np.float64)
        out = np.zeros((self.dim, self.Ng))
        load().orc_avg_grad(self._h, _d(phi), _d(out))
        return out

    def stream_op(self, g, rho, mu):
        g = np.ascontiguousarray(g, dtype=np.float64)
        rho = np.ascontiguousarray(rho, dtype=np.float64)
        mu = np.ascontiguousarray(mu, dtype=np.float64)
        out = np.zeros((self.Q, self.Ng))
        load().orc_stream_op(self._h, _d(g), _d(rho), _d(mu), _d(out))
        return out

    def density(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64)
        out = np.zeros(self.Ng)
        load().orc_density(self._h, _d(f), _d(out))
        return out

    def collide(self, f, rho, grho, gmu):
        f, rho = np.ascontiguousarray(f, dtype=np.float64), np.ascontiguousarray(rho, dtype=np.float64)
        grho, gmu = np.ascontiguousarray(grho, dtype=np.float64), np.ascontiguousarray(gmu, dtype=np.float64)
        out = np.zeros((self.Q, self.Ng))
        load().orc_collide(self._h, _d(f), _d(rho), _d(grho), _d(gmu), _d(out))
        return out

    # --- state --------------------------------------------------------------------------
    def set_rho(self, rho):
        rho = np.ascontiguousarray(rho, dtype=np.float64)
        load().orc_set_rho(self._h, _d(rho))

    def init_tanh(self, x0=None, R=None, noise=None, seed=None):
        c = self.case
        x0 = np.array(c.x0 if x0 is None else x0, dtype=np.float64)
        if x0.size < 3:
            x0 = np.concatenate([x0, np.zeros(3 - x0.size)])
        load().orc_init_tanh(self._h, _d(x0), float(c.R if R is None else R),
                             float(c.noise if noise is None else noise),
                             int(c.seed if seed is None else seed))

    def set_f(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64)
        load().orc_set_f(self._h, _d(f))

    def get_f(self):
        f = np.zeros((self.Q, self.Ng))
        load().orc_get_f(self._h, _d(f))
        return f

    def step(self, n=1):
        load().orc_step(self._h, int(n))

    @property
    def nstep(self):
        return load().orc_nstep(self._h)

    def rho(self):
        out = np.zeros(self.Ng)
        load().orc_get_rho(self._h, _d(out))
        return out

    def u(self):
        out = np.zeros((self.dim, self.Ng))
        load().orc_get_u(self._h, _d(out))
        return out

    def diag(self):
        ke, ms = C.c_double(), C.c_double()
        load().orc_diag(self._h, C.byref(ke), C.byref(ms))
        return ke.value, ms.value

"""ctypes binding of libsemlbm.so (the C ABI in include/semlbm.h).

Argument marshalling only: every step of the time loop runs in the library's HIP
kernels.  PyTorch provides the device workspace and the stream.  Importing works
without a GPU; using a solve needs the built library and a HIP device, and fails
loudly otherwise (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsemlbm.so")

SLBM_OK, SLBM_EINVAL, SLBM_ENOMEM, SLBM_EDEVICE, SLBM_ESTATE, SLBM_EDIVERGED = 0, -1, -2, -3, -4, -5
_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ESTATE", -5: "EDIVERGED"}


class SLBMError(RuntimeError):
    def __init__(self, status, msg=""):
        super().__init__(f"slbm {_NAMES.get(status, status)}: {msg}")
        self.status = status


class Params(C.Structure):
    _fields_ = [("lattice", C.c_int), ("N", C.c_int), ("rho_l", C.c_double), ("rho_v", C.c_double),
                ("delta", C.c_double), ("sigma", C.c_double), ("tau", C.c_double),
                ("dt", C.c_double), ("cfl", C.c_double), ("ke_every", C.c_int),
                ("ke_limit", C.c_double), ("seed", C.c_uint64), ("nu", C.c_double)]


class Info(C.Structure):
    _fields_ = [("dt", C.c_double), ("beta", C.c_double), ("kappa", C.c_double),
                ("omega", C.c_double), ("h_min", C.c_double), ("n_elements", C.c_int64),
                ("n_local", C.c_int64), ("n_global", C.c_int64), ("n_wall_nodes", C.c_int64),
                ("step", C.c_int64), ("workspace_bytes", C.c_size_t), ("dim", C.c_int),
                ("Q", C.c_int), ("N", C.c_int), ("tau", C.c_double), ("n_interior", C.c_int64),
                ("fused", C.c_int)]


class WallGeom(C.Structure):
    _fields_ = [("kind", C.c_int), ("point", C.c_double * 3), ("normal", C.c_double * 3),
                ("radius", C.c_double)]


MAX_SHAPES = 4


class BatchShape(C.Structure):
    _fields_ = [("dim", C.c_int), ("order", C.c_int), ("fused", C.c_int), ("members", C.c_int),
                ("elements", C.c_int64), ("n_shapes", C.c_int), ("epb", C.c_int * MAX_SHAPES),
                ("xcd", C.c_int * MAX_SHAPES), ("us_per_step", C.c_double * MAX_SHAPES),
                ("chosen", C.c_int), ("measured", C.c_int), ("lattice", C.c_int)]


class ServerCfg(C.Structure):
    _fields_ = [("arena", C.c_void_p), ("arena_bytes", C.c_size_t), ("hip_stream", C.c_void_p),
                ("max_slots", C.c_int), ("check_every", C.c_int), ("ke_stop", C.c_double),
                ("max_steps", C.c_int64)]


class Request(C.Structure):
    _fields_ = [("params", Params), ("E", C.c_int64), ("xyz", C.c_void_p), ("gid", C.c_void_p),
                ("n_global", C.c_int64), ("n_wall_faces", C.c_int64), ("wall_face", C.c_void_p),
                ("wall_cos", C.c_void_p), ("wall_ub", C.c_void_p), ("x0", C.c_double * 3),
                ("R", C.c_double), ("noise_amp", C.c_double), ("wall", WallGeom),
                ("state_out", C.c_void_p)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int), ("theta_deg", C.c_double), ("ke_max", C.c_double),
                ("steps", C.c_int64), ("t_arrive", C.c_double), ("t_admit", C.c_double),
                ("t_done", C.c_double)]


# every exported entry point of include/semlbm.h: name -> (restype, argtypes)
_vp, _dp, _i64 = C.c_void_p, C.POINTER(C.c_double), C.c_int64
SIGNATURES = {
    "slbm_create": (C.c_int, [C.POINTER(Params), C.POINTER(C.c_void_p)]),
    "slbm_set_mesh": (C.c_int, [_vp, _i64, _vp, _vp, _i64, _i64, _vp, _vp, _vp]),
    "slbm_workspace_bytes": (C.c_size_t, [_vp]),
    "slbm_bind": (C.c_int, [_vp, _vp, C.c_size_t, _vp]),
    "slbm_init_tanh": (C.c_int, [_vp, _dp, C.c_double, C.c_double, C.c_uint64]),
    "slbm_set_rho": (C.c_int, [_vp, _dp]),
    "slbm_get_state": (C.c_int, [_vp, _dp, C.POINTER(C.c_int64)]),
    "slbm_set_state": (C.c_int, [_vp, _dp, _i64]),
    "slbm_step": (C.c_int, [_vp, _i64]),
    "slbm_step_profile": (C.c_int, [_vp, _i64, _dp, C.POINTER(C.c_int64)]),
    "slbm_time_kernel": (C.c_int, [_vp, C.c_int, _i64, _dp]),
    "slbm_get_rho": (C.c_int, [_vp, _dp]),
    "slbm_get_u": (C.c_int, [_vp, _dp]),
    "slbm_kinetic_energy": (C.c_int, [_vp, _dp, _dp]),
    "slbm_contact_angle": (C.c_int, [_vp, C.POINTER(WallGeom), _dp]),
    "slbm_get_info": (C.c_int, [_vp, C.POINTER(Info)]),
    "slbm_get_gll": (C.c_int, [_vp, _dp, _dp, _dp]),
    "slbm_get_mass": (C.c_int, [_vp, _dp]),
    "slbm_last_error": (C.c_char_p, [_vp]),
    "slbm_destroy": (None, [_vp]),
    "slbm_op_mu": (C.c_int, [_vp, _dp, _dp]),
    "slbm_op_grad": (C.c_int, [_vp, _dp, _dp]),
    "slbm_op_stream": (C.c_int, [_vp, _dp, _dp, _dp, _dp]),
    "slbm_op_collide": (C.c_int, [_vp, _dp, _dp, _dp, _dp, _dp]),
    "slbm_batch_create": (C.c_int, [_vp, C.POINTER(C.c_void_p)]),
    "slbm_batch_add": (C.c_int, [_vp, _vp]),
    "slbm_batch_remove": (C.c_int, [_vp, _vp]),
    "slbm_batch_size": (C.c_int, [_vp]),
    "slbm_batch_step": (C.c_int, [_vp, _i64]),
    "slbm_batch_step_static": (C.c_int, [_vp, _i64]),
    "slbm_batch_set_autotune": (C.c_int, [_vp, C.c_int]),
    "slbm_batch_shapes": (C.c_int, [_vp, C.POINTER(BatchShape), C.c_int, C.POINTER(C.c_int)]),
    "slbm_batch_kinetic_energy": (C.c_int, [_vp, _dp, _dp]),
    "slbm_batch_destroy": (None, [_vp]),
    "slbm_server_create": (C.c_int, [C.POINTER(ServerCfg), C.POINTER(C.c_void_p)]),
    "slbm_server_submit": (C.c_int, [_vp, C.POINTER(Request), C.POINTER(C.c_uint64)]),
    "slbm_server_tick": (C.c_int, [_vp, C.POINTER(C.c_int)]),
    "slbm_server_poll": (C.c_int, [_vp, C.c_uint64, C.POINTER(Result)]),
    "slbm_server_drain": (C.c_int, [_vp]),
    "slbm_server_clock": (C.c_double, [_vp]),
    "slbm_server_destroy": (None, [_vp]),
}

_lib = None


def lib():
    """Load libsemlbm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it first "
                               "(python -c 'import __graft_entry__ as g; g.build()')")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp)


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no HIP device: the SEM-LBM library runs on the GPU only")
    return torch


def wall_geom(spec: dict | None) -> WallGeom:
    w = WallGeom()
    if not spec:
        return w
    kinds = {"plane": 0, "circle": 1, "sphere": 2}
    w.kind = kinds[spec["kind"]]
    pt = spec.get("point", spec.get("center", (0.0, 0.0, 0.0)))
    for k, v in enumerate(pt):
        w.point[k] = float(v)
    for k, v in enumerate(spec.get("normal", (0.0, 0.0, 0.0))):
        w.normal[k] = float(v)
    w.radius = float(spec.get("radius", 0.0))
    return w


def make_params(case, ke_every: int = 0, ke_limit: float = 0.0) -> Params:
    p = Params()
    p.lattice = int(case.lattice)
    p.N = int(case.mesh.N)
    p.rho_l, p.rho_v = float(case.rho_l), float(case.rho_v)
    p.delta, p.sigma, p.tau = float(case.delta), float(case.sigma), float(case.tau)
    p.dt, p.cfl = float(case.dt), float(case.cfl)
    p.ke_every = int(ke_every)
    p.ke_limit = float(ke_limit)
    p.seed = int(case.seed)
    p.nu = float(getattr(case, "nu", 0.0) or 0.0)
    return p


class Solve:
    """One bound solve on ``device`` (torch device string) with its own workspace."""

    def __init__(self, case, device="cuda:0", stream=None, ke_every: int = 0,
                 ke_limit: float = 0.0):
        torch = _torch()
        L = lib()
        self.case = case
        m = case.mesh
        self.dim, self.N, self.Q = m.dim, m.N, case.lattice
        self.Ng = m.n_global
        p = make_params(case, ke_every, ke_limit)
        h = C.c_void_p()
        self._check(L.slbm_create(C.byref(p), C.byref(h)), None)
        self._h = h
        xyz = np.ascontiguousarray(m.xyz, dtype=np.float64)
        gid = np.ascontiguousarray(m.gid, dtype=np.int32)
        wf = np.ascontiguousarray(m.wall_face, dtype=np.int32)
        wc = np.ascontiguousarray(m.wall_cos, dtype=np.float64)
        wu = np.ascontiguousarray(m.wall_ub, dtype=np.float64)
        nwf = wf.shape[0]
        self._check(L.slbm_set_mesh(h, m.E, xyz.ctypes.data, gid.ctypes.data, m.n_global, nwf,
                                    wf.ctypes.data if nwf else None,
                                    wc.ctypes.data if nwf else None,
                                    wu.ctypes.data if nwf else None))
        nbytes = L.slbm_workspace_bytes(h)
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) & ~255
        self._check(L.slbm_bind(h, aligned, nbytes, self.stream.cuda_stream))

    def _check(self, st, h=False):
        if st != SLBM_OK:
            msg = ""
            hh = self._h if h is False else h
            if hh:
                msg = lib().slbm_last_error(hh).decode()
            raise SLBMError(st, msg)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.slbm_destroy(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def info(self) -> Info:
        inf = Info()
        self._check(lib().slbm_get_info(self._h, C.byref(inf)))
        return inf

    def init_tanh(self, x0=None, R=None, noise=None, seed=None):
        c = self.case
        x = np.zeros(3)
        src = c.x0 if x0 is None else x0
        x[: len(src)] = src
        self._check(lib().slbm_init_tanh(self._h, _d(x), float(c.R if R is None else R),
                                         float(c.noise if noise is None else noise),
                                         int(c.seed if seed is None else seed)))

    def set_rho(self, rho):
        rho = np.ascontiguousarray(rho, dtype=np.float64)
        self._check(lib().slbm_set_rho(self._h, _d(rho)))

    def set_state(self, f, step=0):
        f = np.ascontiguousarray(f, dtype=np.float64)
        self._check(lib().slbm_set_state(self._h, _d(f), int(step)))

    def get_state(self):
        f = np.zeros((self.Q, self.Ng))
        st = C.c_int64()
        self._check(lib().slbm_get_state(self._h, _d(f), C.byref(st)))
        return f, st.value

    def step(self, n=1):
        self._check(lib().slbm_step(self._h, int(n)))

    KERNEL_KINDS = ("lap", "mu", "grad", "collide", "stream", "rk",
                    "f_mu_grad", "f_collide_stream", "f_rk_lap", "f_mu_stream")

    def step_profile(self, n=1):
        """n steps with per-kernel HIP event timing: {kind: (total_ms, launches)}."""
        ms = np.zeros(len(self.KERNEL_KINDS))
        cnt = np.zeros(len(self.KERNEL_KINDS), dtype=np.int64)
        self._check(lib().slbm_step_profile(self._h, int(n), _d(ms),
                                            cnt.ctypes.data_as(C.POINTER(C.c_int64))))
        return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(self.KERNEL_KINDS) if cnt[i]}

    def time_kernel(self, kind, reps=300):
        """Average ms of one launch of kernel `kind` over reps back-to-back graph launches."""
        ms = C.c_double(0.0)
        self._check(lib().slbm_time_kernel(self._h, self.KERNEL_KINDS.index(kind), int(reps),
                                           C.byref(ms)))
        return ms.value

    def rho(self):
        out = np.zeros(self.Ng)
        self._check(lib().slbm_get_rho(self._h, _d(out)))
        return out

    def u(self):
        out = np.zeros((self.dim, self.Ng))
        self._check(lib().slbm_get_u(self._h, _d(out)))
        return out

    def kinetic_energy(self):
        ke, ms = C.c_double(), C.c_double()
        self._check(lib().slbm_kinetic_energy(self._h, C.byref(ke), C.byref(ms)))
        return ke.value, ms.value

    def contact_angle(self, wall=None):
        w = wall_geom(wall if wall is not None else self.case.wall_geom)
        th = C.c_double()
        self._check(lib().slbm_contact_angle(self._h, C.byref(w), C.byref(th)))
        return th.value

    # operator entry points
    def op_mu(self, rho):
        rho = np.ascontiguousarray(rho, dtype=np.float64)
        out = np.zeros(self.Ng)
        self._check(lib().slbm_op_mu(self._h, _d(rho), _d(out)))
        return out

    def op_grad(self, phi):
        phi = np.ascontiguousarray(phi, dtype=np.float64)
        out = np.zeros((self.dim, self.Ng))
        self._check(lib().slbm_op_grad(self._h, _d(phi), _d(out)))
        return out

    def op_stream(self, g, rho, mu):
        g, rho, mu = (np.ascontiguousarray(a, dtype=np.float64) for a in (g, rho, mu))
        out = np.zeros((self.Q, self.Ng))
        self._check(lib().slbm_op_stream(self._h, _d(g), _d(rho), _d(mu), _d(out)))
        return out

    def op_collide(self, f, rho, grho, gmu):
        f, rho, grho, gmu = (np.ascontiguousarray(a, dtype=np.float64) for a in (f, rho, grho, gmu))
        out = np.zeros((self.Q, self.Ng))
        self._check(lib().slbm_op_collide(self._h, _d(f), _d(rho), _d(grho), _d(gmu), _d(out)))
        return out


class Batch:
    """Several bound solves advanced together (one launch per kernel and (d, N) group)."""

    def __init__(self, stream):
        h = C.c_void_p()
        st = lib().slbm_batch_create(stream.cuda_stream, C.byref(h))
        if st != SLBM_OK:
            raise SLBMError(st, "batch_create")
        self._h = h
        self.members = []

    def add(self, solve: Solve):
        st = lib().slbm_batch_add(self._h, solve.handle)
        if st != SLBM_OK:
            raise SLBMError(st, "batch_add")
        self.members.append(solve)

    def remove(self, solve: Solve):
        st = lib().slbm_batch_remove(self._h, solve.handle)
        if st != SLBM_OK:
            raise SLBMError(st, "batch_remove")
        self.members.remove(solve)

    def step(self, n=1):
        st = lib().slbm_batch_step(self._h, int(n))
        if st != SLBM_OK:
            raise SLBMError(st, "batch_step")

    def step_static(self, n=1):
        """The allocation-free batched step (slbm_batch_step_static)."""
        st = lib().slbm_batch_step_static(self._h, int(n))
        if st != SLBM_OK:
            raise SLBMError(st, "batch_step_static")

    def set_autotune(self, on: bool):
        st = lib().slbm_batch_set_autotune(self._h, 1 if on else 0)
        if st != SLBM_OK:
            raise SLBMError(st, "batch_set_autotune")

    def shapes(self):
        """Launch shapes per group: list of dicts (key, candidates with measured us/step,
        chosen index, whether the choice was timed)."""
        cnt = C.c_int(0)
        st = lib().slbm_batch_shapes(self._h, None, 0, C.byref(cnt))
        if st != SLBM_OK:
            raise SLBMError(st, "batch_shapes")
        arr = (BatchShape * max(cnt.value, 1))()
        st = lib().slbm_batch_shapes(self._h, arr, cnt.value, C.byref(cnt))
        if st != SLBM_OK:
            raise SLBMError(st, "batch_shapes")
        out = []
        for r in arr[:cnt.value]:
            out.append({"dim": r.dim, "lattice": r.lattice, "N": r.order, "fused": bool(r.fused),
                        "members": r.members,
                        "elements": r.elements, "chosen": r.chosen, "measured": bool(r.measured),
                        "shapes": [{"epb": r.epb[k], "xcd": bool(r.xcd[k]), "us_per_step": r.us_per_step[k]}
                                   for k in range(r.n_shapes)]})
        return out

    def kinetic_energy(self):
        n = len(self.members)
        ke, ms = np.zeros(max(n, 1)), np.zeros(max(n, 1))
        st = lib().slbm_batch_kinetic_energy(self._h, _d(ke), _d(ms))
        if st != SLBM_OK:
            raise SLBMError(st, "batch_kinetic_energy")
        return ke[:n], ms[:n]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.slbm_batch_destroy(h)
            self._h = None


class Server:
    """Continuous-batching request loop over a torch-allocated device arena."""

    def __init__(self, arena_bytes, max_slots=64, check_every=100, ke_stop=1e-20,
                 max_steps=50000, device="cuda:0", stream=None):
        torch = _torch()
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.arena = torch.empty(int(arena_bytes) + 256, dtype=torch.uint8, device=self.device)
        cfg = ServerCfg()
        cfg.arena = (self.arena.data_ptr() + 255) & ~255
        cfg.arena_bytes = int(arena_bytes)
        cfg.hip_stream = self.stream.cuda_stream
        cfg.max_slots = int(max_slots)
        cfg.check_every = int(check_every)
        cfg.ke_stop = float(ke_stop)
        cfg.max_steps = int(max_steps)
        h = C.c_void_p()
        st = lib().slbm_server_create(C.byref(cfg), C.byref(h))
        if st != SLBM_OK:
            raise SLBMError(st, "server_create")
        self._h = h
        self._keep = {}

    def submit(self, case, noise: float | None = None, ke_limit: float = 0.0,
               keep_state: bool = False) -> int:
        """Queue a solve of ``case``; ``ke_limit`` > 0 marks it diverged (SLBM_EDIVERGED)
        at the first check with KE_max above it (default limit 1).  With ``keep_state`` the
        final f-bar of a completed request is returned by :meth:`state` ([Q][n_global])."""
        m = case.mesh
        r = Request()
        r.params = make_params(case, 0, ke_limit)
        arrs = dict(xyz=np.ascontiguousarray(m.xyz, dtype=np.float64),
                    gid=np.ascontiguousarray(m.gid, dtype=np.int32),
                    wf=np.ascontiguousarray(m.wall_face, dtype=np.int32),
                    wc=np.ascontiguousarray(m.wall_cos, dtype=np.float64),
                    wu=np.ascontiguousarray(m.wall_ub, dtype=np.float64))
        r.E = m.E
        r.xyz = arrs["xyz"].ctypes.data
        r.gid = arrs["gid"].ctypes.data
        r.n_global = m.n_global
        r.n_wall_faces = m.wall_face.shape[0]
        r.wall_face = arrs["wf"].ctypes.data if r.n_wall_faces else None
        r.wall_cos = arrs["wc"].ctypes.data if r.n_wall_faces else None
        r.wall_ub = arrs["wu"].ctypes.data if r.n_wall_faces else None
        for k, v in enumerate(case.x0):
            r.x0[k] = float(v)
        r.R = float(case.R)
        r.noise_amp = float(case.noise if noise is None else noise)
        r.wall = wall_geom(case.wall_geom)
        out = np.zeros((case.lattice, m.n_global)) if keep_state else None
        r.state_out = out.ctypes.data if keep_state else None
        rid = C.c_uint64()
        st = lib().slbm_server_submit(self._h, C.byref(r), C.byref(rid))
        if st != SLBM_OK:
            raise SLBMError(st, "server_submit")
        if keep_state:
            self._keep[rid.value] = out
        return rid.value

    def state(self, rid):
        """Final f-bar of a request submitted with ``keep_state`` (valid once polled done)."""
        return self._keep[int(rid)]

    def tick(self) -> int:
        pend = C.c_int()
        st = lib().slbm_server_tick(self._h, C.byref(pend))
        if st != SLBM_OK:
            raise SLBMError(st, "server_tick")
        return pend.value

    def poll(self, rid) -> Result:
        res = Result()
        st = lib().slbm_server_poll(self._h, int(rid), C.byref(res))
        if st != SLBM_OK:
            raise SLBMError(st, "server_poll")
        return res

    def drain(self):
        st = lib().slbm_server_drain(self._h)
        if st != SLBM_OK:
            raise SLBMError(st, "server_drain")

    def clock(self) -> float:
        return lib().slbm_server_clock(self._h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.slbm_server_destroy(h)
            self._h = None

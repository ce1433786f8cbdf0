"""Host-side tests of the C ABI (no GPU): symbols, argument checks, call order, and the
host tables (GLL, lumped mass, time step) compared with the oracle bit for bit."""
import ctypes as C
import os
import re

import math

import numpy as np
import pytest

from synth import cases, meshes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "semlbm.h")


@pytest.fixture(scope="module")
def L():
    import paper_2609_00535_amd as P
    try:
        return P.lib()
    except RuntimeError as e:  # library not built in this checkout
        pytest.skip(str(e))


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(slbm_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(L):
    import paper_2609_00535_amd as P
    names = declared_functions()
    assert len(names) >= 30
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(P.SIGNATURES), set(names) ^ set(P.SIGNATURES)


def _create(L, case):
    import paper_2609_00535_amd as P
    p = P.make_params(case)
    h = C.c_void_p()
    assert L.slbm_create(C.byref(p), C.byref(h)) == 0
    return h


def _set_mesh(L, h, m):
    xyz = np.ascontiguousarray(m.xyz)
    gid = np.ascontiguousarray(m.gid, dtype=np.int32)
    wf = np.ascontiguousarray(m.wall_face, dtype=np.int32)
    wc = np.ascontiguousarray(m.wall_cos)
    wu = np.ascontiguousarray(m.wall_ub)
    nwf = wf.shape[0]
    return L.slbm_set_mesh(h, m.E, xyz.ctypes.data, gid.ctypes.data, m.n_global, nwf,
                           wf.ctypes.data if nwf else None, wc.ctypes.data if nwf else None,
                           wu.ctypes.data if nwf else None)


def test_argument_and_order_errors(L):
    import paper_2609_00535_amd as P
    c = cases.c1()
    p = P.make_params(c)
    h = C.c_void_p()
    bad = P.make_params(c)
    bad.lattice = 7
    assert L.slbm_create(C.byref(bad), C.byref(h)) == P.binding.SLBM_EINVAL and not h.value
    bad = P.make_params(c)
    bad.N = 40
    assert L.slbm_create(C.byref(bad), C.byref(h)) == P.binding.SLBM_EINVAL
    bad = P.make_params(c)
    bad.rho_v = 2.0
    assert L.slbm_create(C.byref(bad), C.byref(h)) == P.binding.SLBM_EINVAL
    for nu in (-0.1, float("nan"), float("inf")):
        bad = P.make_params(c)
        bad.nu = nu
        assert L.slbm_create(C.byref(bad), C.byref(h)) == P.binding.SLBM_EINVAL
    bad = P.make_params(c)
    bad.tau = 0.0
    assert L.slbm_create(C.byref(bad), C.byref(h)) == P.binding.SLBM_EINVAL
    ok = P.make_params(c)
    ok.tau, ok.nu = 0.0, 0.05  # a viscosity stands in for tau
    assert L.slbm_create(C.byref(ok), C.byref(h)) == 0
    L.slbm_destroy(h)
    assert L.slbm_create(C.byref(p), C.byref(h)) == 0
    assert L.slbm_workspace_bytes(h) == 0
    assert L.slbm_step(h, 1) == P.binding.SLBM_ESTATE
    m = c.mesh
    gid = np.ascontiguousarray(m.gid, dtype=np.int32).copy()
    gid[3] = m.n_global + 5
    xyz = np.ascontiguousarray(m.xyz)
    assert L.slbm_set_mesh(h, m.E, xyz.ctypes.data, gid.ctypes.data, m.n_global, 0, None, None,
                           None) == P.binding.SLBM_EINVAL
    assert b"out of range" in L.slbm_last_error(h)
    # inverted element -> non-positive Jacobian
    xyz2 = xyz.copy()
    xyz2[0, :, 0] = -xyz2[0, :, 0]
    gid = np.ascontiguousarray(m.gid, dtype=np.int32)
    assert L.slbm_set_mesh(h, m.E, xyz2.ctypes.data, gid.ctypes.data, m.n_global, 0, None, None,
                           None) == P.binding.SLBM_EINVAL
    assert b"Jacobian" in L.slbm_last_error(h)
    assert _set_mesh(L, h, m) == 0
    assert L.slbm_workspace_bytes(h) > 0
    # misaligned / too small workspace
    assert L.slbm_bind(h, 8, 10 ** 9, None) == P.binding.SLBM_EINVAL
    assert L.slbm_bind(h, 4096, 16, None) == P.binding.SLBM_ENOMEM
    assert L.slbm_step(h, 1) == P.binding.SLBM_ESTATE
    assert L.slbm_get_rho(h, np.zeros(m.n_global).ctypes.data_as(C.POINTER(C.c_double))) == \
        P.binding.SLBM_ESTATE
    L.slbm_destroy(h)


@pytest.mark.parametrize("mk", [cases.c1, cases.c2, cases.small_cyl, cases.small_sphere,
                                cases.small_box3d, lambda: cases.order_case(2, 14),
                                lambda: cases.paper_flat(60.0), lambda: cases.paper_isolated(15.0, 4, 16)])
def test_host_tables_match_oracle_bitwise(L, mk):
    """GLL tables, lumped mass, h_min and dt of the library equal the oracle's exactly:
    parity of the time step to 1e-11 needs identical inputs to every kernel."""
    import paper_2609_00535_amd as P
    from oracle import Oracle
    c = mk()
    h = _create(L, c)
    assert _set_mesh(L, h, c.mesh) == 0
    Np = c.N + 1
    x, w, D = np.zeros(Np), np.zeros(Np), np.zeros(Np * Np)
    dp = C.POINTER(C.c_double)
    assert L.slbm_get_gll(h, x.ctypes.data_as(dp), w.ctypes.data_as(dp), D.ctypes.data_as(dp)) == 0
    o = Oracle(c)
    xo, wo, Do = o.gll()
    assert np.array_equal(x, xo) and np.array_equal(w, wo) and np.array_equal(D, Do.reshape(-1))
    MA = np.zeros(c.mesh.n_global)
    assert L.slbm_get_mass(h, MA.ctypes.data_as(dp)) == 0
    assert np.array_equal(MA, o.mass_matrix())
    inf = P.binding.Info()
    assert L.slbm_get_info(h, C.byref(inf)) == 0
    assert inf.dt == o.dt and inf.h_min == o.hmin and inf.beta == o.beta and inf.kappa == o.kappa
    assert inf.omega == o.omega
    if c.nu > 0.0:  # the relaxation time of the case's viscosity at this dt
        assert abs(inf.tau * inf.dt / 3.0 - c.nu) < 1e-15 * c.nu
    assert inf.n_wall_nodes == o.nw
    L.slbm_destroy(h)


def test_kernel_path_rule(L, monkeypatch):
    """slbm_set_mesh picks the fused element kernels up to 2^20 local nodes in 2-D and 2^17
    in 3-D, the separate kernels with the interior-first split above (measured crossovers)."""
    import paper_2609_00535_amd as P
    for v in ("SLBM_UNFUSED", "SLBM_FUSED", "SLBM_NO_SPLIT"):
        monkeypatch.delenv(v, raising=False)
    big2 = cases.small_flat(theta_deg=70.0, nx=183, ny=117, N=6, Lx=8.0 * 183, Ly=8.0 * 117, R=24.0)
    mid2 = cases.small_flat(theta_deg=70.0, nx=92, ny=117, N=6, Lx=8.0 * 92, Ly=8.0 * 117, R=24.0)
    for c, fused in ((cases.small_sphere(n_t=2, n_rad=2, N=4), 1),    # 6,000 local nodes
                     (cases.small_sphere(n_t=4, n_rad=2, N=6), 1),    # 65,856
                     (cases.small_sphere(n_t=6, n_rad=3, N=6), 0),    # 222,264
                     (mid2, 1),                                       # 527,436
                     (big2, 0)):                                      # 1,049,097
        h = _create(L, c)
        assert _set_mesh(L, h, c.mesh) == 0
        inf = P.binding.Info()
        assert L.slbm_get_info(h, C.byref(inf)) == 0
        limit = (1 << 20) if c.mesh.dim == 2 else (1 << 17)
        assert (inf.n_local > limit) == (fused == 0), (c.mesh.E, inf.n_local)
        assert inf.fused == fused, (c.mesh.E, inf.n_local)
        assert (inf.n_interior > 0) == (fused == 0)
        L.slbm_destroy(h)


@pytest.mark.parametrize("theta", [30.0, 60.0, 90.0, 120.0, 150.0])
def test_paper_flat_case_geometry(theta):
    """Inputs of the flat-wall runs: the equilibrium cap has the area of the D = 32 circle
    (counted on a 0.05 grid, not from the segment formula), it meets the wall at theta, it
    stays clear of the other walls, and nu gives La = 122."""
    c = cases.paper_flat(theta)
    xc, yc = c.x0
    h = 0.05
    xs = np.arange(0.0, 128.0, h) + 0.5 * h
    ys = np.arange(0.0, 64.0, h) + 0.5 * h
    X, Y = np.meshgrid(xs, ys)
    inside = (X - xc) ** 2 + (Y - yc) ** 2 < c.R ** 2
    area = inside.sum() * h * h
    assert abs(area - math.pi * 16.0 ** 2) < 2e-3 * math.pi * 16.0 ** 2
    # the cap's edge crosses y = 0 where the circle's tangent makes theta with the wall
    assert abs(math.degrees(math.acos(-yc / c.R)) - theta) < 1e-9
    assert not inside[:, 0].any() and not inside[:, -1].any() and not inside[-1, :].any()
    assert abs(c.sigma * 32.0 / (c.rho_l * c.nu ** 2) - 122.0) < 1e-9
    assert c.N == 16 and c.mesh.E == 128


def test_paper_isolated_case():
    """Inputs of the isolated-droplet runs: the same node count at N = 16 on 4x4 and N = 4
    on 16x16, Cn = 0.063, the La of nu, the droplet clear of the walls."""
    a, b = cases.paper_isolated(61.5, 16, 4), cases.paper_isolated(3.07, 4, 16)
    assert a.mesh.n_global == b.mesh.n_global == 65 * 65
    for c, La in ((a, 61.5), (b, 3.07)):
        assert abs(c.delta / (2.0 * c.R) - 0.063) < 1e-12
        assert abs(c.sigma * 2.0 * c.R / (c.rho_l * c.nu ** 2) - La) < 1e-9
        assert c.x0[0] - c.R > 4.0 * c.delta and c.x0[1] - c.R > 4.0 * c.delta


@pytest.mark.parametrize("theta", [30.0, 90.0, 150.0])
def test_paper_curved_case_geometry(theta):
    """Inputs of the curved-wall runs: the liquid outside the circular wall (area counted
    on a 0.05 grid) equals the D = 25.6 circle, the cap meets the wall at theta (from the
    two outward normals at an intersection point), and nu gives La = 341."""
    c = cases.paper_curved(theta)
    (xc, yc), R = c.x0, c.R
    Rw = c.wall_geom["radius"]
    cx, cy = c.wall_geom["center"]
    h = 0.05
    xs = np.arange(cx - 64.0, cx + 64.0, h) + 0.5 * h
    X, Y = np.meshgrid(xs, xs)
    liquid = ((X - xc) ** 2 + (Y - yc) ** 2 < R * R) & ((X - cx) ** 2 + (Y - cy) ** 2 > Rw * Rw)
    assert abs(liquid.sum() * h * h - math.pi * 12.8 ** 2) < 3e-3 * math.pi * 12.8 ** 2
    # an intersection point P of the two circles, then the contact angle through the liquid
    # from the outward normals there: cos(theta) = n_wall . n_drop
    ux, uy = xc - cx, yc - cy
    d = math.hypot(ux, uy)
    a = (Rw * Rw - R * R + d * d) / (2.0 * d)
    hh = math.sqrt(Rw * Rw - a * a)
    px, py = cx + (a * ux - hh * uy) / d, cy + (a * uy + hh * ux) / d
    assert abs(math.hypot(px - cx, py - cy) - Rw) < 1e-9 and abs(math.hypot(px - xc, py - yc) - R) < 1e-9
    cos_t = ((px - cx) * (px - xc) + (py - cy) * (py - yc)) / (Rw * R)
    assert abs(math.degrees(math.acos(cos_t)) - theta) < 1e-7
    assert abs(c.sigma * 25.6 / (c.rho_l * c.nu ** 2) - 341.0) < 1e-9


def test_mesh_generators_structure():
    """Inputs: shared nodes bitwise equal (no periodic wrap), Jacobians positive."""
    for m in [cases.c2().mesh, cases.small_cyl().mesh, cases.small_sphere().mesh]:
        X = m.xyz.reshape(-1, m.dim)
        g = m.gid.reshape(-1)
        first = m.first_copy_coords()
        assert np.array_equal(X, first[g])
    m = cases.c3().mesh
    X = m.xyz.reshape(-1, 2)
    r = np.hypot(X[:, 0] - 128, X[:, 1] - 128)
    wall_e = m.wall_face[m.wall_face[:, 1] == meshes.FACE_XI_M, 0]
    Np = m.N + 1
    on = m.xyz[wall_e][:, ::Np, :]  # i = 0 nodes of cylinder elements
    assert np.abs(np.hypot(on[..., 0] - 128, on[..., 1] - 128) - 40.0).max() < 1e-12
    assert r.min() > 40.0 - 1e-12


def test_time_kernel_and_wall_face_errors(L):
    """Tracing entry point: argument and call-order errors (no GPU needed); a wall face
    listed twice is rejected at set_mesh."""
    import paper_2609_00535_amd as P
    c = cases.small_flat()
    h = _create(L, c)
    ms = C.c_double(0.0)
    assert L.slbm_time_kernel(h, 99, 10, C.byref(ms)) == P.binding.SLBM_EINVAL
    assert L.slbm_time_kernel(h, 6, 0, C.byref(ms)) == P.binding.SLBM_EINVAL
    assert L.slbm_time_kernel(h, 6, 10, None) == P.binding.SLBM_EINVAL
    assert L.slbm_time_kernel(h, 6, 10, C.byref(ms)) == P.binding.SLBM_ESTATE
    L.slbm_destroy(h)
    m = c.mesh
    h = _create(L, c)
    wf = np.ascontiguousarray(np.concatenate([m.wall_face, m.wall_face[:1]]), dtype=np.int32)
    wc = np.ascontiguousarray(np.concatenate([m.wall_cos, m.wall_cos[:1]]))
    wu = np.ascontiguousarray(np.concatenate([m.wall_ub, m.wall_ub[:1]]))
    xyz = np.ascontiguousarray(m.xyz)
    gid = np.ascontiguousarray(m.gid, dtype=np.int32)
    st = L.slbm_set_mesh(h, m.E, xyz.ctypes.data, gid.ctypes.data, m.n_global, wf.shape[0],
                         wf.ctypes.data, wc.ctypes.data, wu.ctypes.data)
    assert st == P.binding.SLBM_EINVAL and b"duplicate" in L.slbm_last_error(h)
    L.slbm_destroy(h)


def test_batch_tuning_argument_errors(L):
    """Autotuning entry points: argument errors and the empty batch (no GPU needed)."""
    import paper_2609_00535_amd as P
    b = C.c_void_p()
    assert L.slbm_batch_create(None, C.byref(b)) == 0
    assert L.slbm_batch_set_autotune(b, 2) == P.binding.SLBM_EINVAL
    assert L.slbm_batch_set_autotune(None, 1) == P.binding.SLBM_EINVAL
    assert L.slbm_batch_set_autotune(b, 0) == 0 and L.slbm_batch_set_autotune(b, 1) == 0
    cnt = C.c_int(-1)
    assert L.slbm_batch_shapes(b, None, 0, C.byref(cnt)) == 0 and cnt.value == 0
    assert L.slbm_batch_shapes(b, None, 1, C.byref(cnt)) == P.binding.SLBM_EINVAL
    assert L.slbm_batch_shapes(b, None, -1, C.byref(cnt)) == P.binding.SLBM_EINVAL
    assert L.slbm_batch_shapes(b, None, 0, None) == P.binding.SLBM_EINVAL
    L.slbm_batch_destroy(b)


def test_server_config_errors(L):
    """Server creation rejects a missing arena and non-positive slots or check cadence
    (no GPU needed); a valid server that never ran is created and destroyed cleanly."""
    import paper_2609_00535_amd as P
    B = P.binding
    cfg = B.ServerCfg()
    cfg.arena, cfg.arena_bytes, cfg.hip_stream = None, 1 << 20, None
    cfg.max_slots, cfg.check_every, cfg.ke_stop, cfg.max_steps = 4, 100, 1e-20, 1000
    h = C.c_void_p()
    assert L.slbm_server_create(C.byref(cfg), C.byref(h)) == B.SLBM_EINVAL
    cfg.arena = 256
    cfg.max_slots = 0
    assert L.slbm_server_create(C.byref(cfg), C.byref(h)) == B.SLBM_EINVAL
    cfg.max_slots, cfg.check_every = 4, 0
    assert L.slbm_server_create(C.byref(cfg), C.byref(h)) == B.SLBM_EINVAL
    cfg.check_every = 100
    assert L.slbm_server_create(C.byref(cfg), C.byref(h)) == 0 and h.value
    res = B.Result()
    assert L.slbm_server_poll(h, 12345, C.byref(res)) == B.SLBM_EINVAL
    L.slbm_server_destroy(h)


def test_degenerate_inputs(L):
    """An empty mesh is rejected; a batch with no members steps as a no-op."""
    import paper_2609_00535_amd as P
    h = _create(L, cases.c1())
    xyz, gid = np.zeros(1), np.zeros(1, dtype=np.int32)
    assert L.slbm_set_mesh(h, 0, xyz.ctypes.data, gid.ctypes.data, 0, 0, None, None, None) == \
        P.binding.SLBM_EINVAL
    L.slbm_destroy(h)
    b = C.c_void_p()
    assert L.slbm_batch_create(None, C.byref(b)) == 0
    assert L.slbm_batch_step(b, 5) == 0
    L.slbm_batch_destroy(b)

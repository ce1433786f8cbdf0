"""Named, seeded synthetic workloads.

Each case bundles a mesh from :mod:`synth.meshes` with the physical
parameters, the droplet placement and the run length.  The five workloads of
the benchmark suite are ``c1`` .. ``c5``; the ``small_*`` cases are shrunken
versions with the same structure (walls, jitter, curvature) that a plain CPU
implementation finishes in seconds.

Droplet placements on walls follow Young's law for the imposed angle theta
(measured through the liquid): a cap of radius R on a flat wall has its
centre at distance -R cos(theta) from the wall; on a circle/sphere of radius
Rw the centre distance d solves d^2 = Rw^2 + R^2 - 2 R Rw cos(theta).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import meshes

LATTICE_D2Q9 = 9
LATTICE_D3Q19 = 19
LATTICE_D3Q13 = 13


@dataclass
class Case:
    name: str
    mesh: meshes.Mesh
    lattice: int
    rho_l: float = 1.0
    rho_v: float = 0.1
    delta: float = 4.0
    sigma: float = 0.01
    tau: float = 0.5
    cfl: float = 0.4
    dt: float = 0.0               # > 0 overrides cfl
    x0: tuple = (0.0, 0.0)
    R: float = 16.0
    noise: float = 0.0
    seed: int = 1
    steps: int = 1000
    ke_every: int = 100
    wall_geom: dict = field(default_factory=dict)
    theta_deg: float | None = None
    nu: float = 0.0               # > 0: kinematic viscosity to hold (the library sets tau)

    @property
    def N(self) -> int:
        return self.mesh.N

    @property
    def dim(self) -> int:
        return self.mesh.dim


def young_center_distance(Rw: float, R: float, theta_deg: float) -> float:
    """Distance between wall-circle/sphere centre and droplet centre (Young cap)."""
    c = math.cos(math.radians(theta_deg))
    return math.sqrt(Rw * Rw + R * R - 2.0 * R * Rw * c)


def c1() -> Case:
    """D2Q9 isolated droplet: periodic 64x64 box, 8x8 quads, N=4, R=16, 1e-4 noise."""
    m = meshes.box2d(8, 8, 4, 64.0, 64.0, periodic=(True, True), name="c1")
    return Case("c1", m, LATTICE_D2Q9, x0=(32.0, 32.0), R=16.0, noise=1e-4, seed=1,
                steps=1000)


def c2(theta_deg: float = 60.0) -> Case:
    """D2Q9 sessile droplet on a flat wall: 128x64, 32x16 jittered quads, N=6."""
    cb = math.cos(math.radians(theta_deg))
    m = meshes.box2d(32, 16, 6, 128.0, 64.0, periodic=(False, False), jitter=0.2, seed=2,
                     cos_theta={"bottom": cb}, name="c2")
    # cap radius 32 (half the wall length): at 60 deg its height is 16 = 4 delta, so
    # the contact-angle fit still has an arc clear of the 2-delta wall layer
    R = 32.0
    return Case("c2", m, LATTICE_D2Q9, x0=(64.0, -R * cb), R=R, seed=2, steps=10000,
                wall_geom=dict(kind="plane", point=(0.0, 0.0), normal=(0.0, -1.0)),
                theta_deg=theta_deg)


def c2xl(theta_deg: float = 60.0) -> Case:
    """c2's recipe at 16x the element count: 512x256 jittered quads (h = 4) over a 2048x1024
    walled box, N=6, 60-degree bottom wall, cap R=32 at the middle of the bottom wall.
    About 4.7 M global nodes: the working set exceeds the 256 MB Infinity Cache, so the
    2-D step runs from HBM."""
    cb = math.cos(math.radians(theta_deg))
    m = meshes.box2d(512, 256, 6, 2048.0, 1024.0, periodic=(False, False), jitter=0.2, seed=2,
                     cos_theta={"bottom": cb}, name="c2xl")
    R = 32.0
    return Case("c2xl", m, LATTICE_D2Q9, x0=(1024.0, -R * cb), R=R, seed=2, steps=1000,
                wall_geom=dict(kind="plane", point=(0.0, 0.0), normal=(0.0, -1.0)),
                theta_deg=theta_deg)


def c3(theta_deg: float = 90.0, n_az: int = 128, n_rad: int = 16, N: int = 8) -> Case:
    """D2Q9 droplet on a cylinder (R=40) in a 256^2 box: O-grid of 2048 curved quads, N=8."""
    Rc = 40.0
    R = 40.0
    cc = math.cos(math.radians(theta_deg))
    m = meshes.ogrid2d(n_az, n_rad, N, center=(128.0, 128.0), Rc=Rc, half_width=128.0,
                       grading=4.0, jitter=0.1, seed=3, cos_cyl=cc, cos_box=0.0, name="c3")
    d = young_center_distance(Rc, R, theta_deg)
    return Case("c3", m, LATTICE_D2Q9, x0=(128.0, 128.0 + d), R=R, seed=3, steps=20000,
                wall_geom=dict(kind="circle", center=(128.0, 128.0), radius=Rc),
                theta_deg=theta_deg)


def c4(n_t: int = 20, n_rad: int = 10, N: int = 5, theta_deg: float = 90.0,
       lattice: int = LATTICE_D3Q19) -> Case:
    """D3Q19 droplet (R=20) on a sphere (R=30): cubed-sphere shell in a 128^3 box, N=5."""
    Rs, R = 30.0, 20.0
    cs = math.cos(math.radians(theta_deg))
    m = meshes.cubed_sphere3d(n_t, n_rad, N, center=(64.0, 64.0, 64.0), Rs=Rs,
                              half_width=64.0, grading=3.0, jitter=0.1, seed=4,
                              cos_sphere=cs, cos_box=0.0, name="c4")
    d = young_center_distance(Rs, R, theta_deg)
    return Case("c4" if lattice == LATTICE_D3Q19 else "c4q13", m, lattice, x0=(64.0, 64.0, 64.0 + d),
                R=R, seed=4, steps=5000,
                wall_geom=dict(kind="sphere", center=(64.0, 64.0, 64.0), radius=Rs),
                theta_deg=theta_deg)


# ---------------------------------------------------------------------------
# small variants for CPU-speed checks (same structure, fewer nodes)
# ---------------------------------------------------------------------------

def small_flat(theta_deg: float = 60.0, nx: int = 8, ny: int = 4, N: int = 4,
               jitter: float = 0.2, seed: int = 12, Lx: float = 64.0, Ly: float = 32.0,
               R: float = 12.0) -> Case:
    """Flat-wall sessile cap on a jittered walled box (default 64x32)."""
    cb = math.cos(math.radians(theta_deg))
    m = meshes.box2d(nx, ny, N, Lx, Ly, periodic=(False, False), jitter=jitter, seed=seed,
                     cos_theta={"bottom": cb}, name="small_flat")
    return Case("small_flat", m, LATTICE_D2Q9, x0=(0.5 * Lx, -R * cb), R=R, seed=seed,
                steps=200, wall_geom=dict(kind="plane", point=(0.0, 0.0), normal=(0.0, -1.0)),
                theta_deg=theta_deg)


def small_cyl(theta_deg: float = 90.0, n_az: int = 16, n_rad: int = 4, N: int = 5) -> Case:
    """Cylinder O-grid (R=12) in a 80x80 box with a Young cap."""
    Rc, R = 12.0, 12.0
    cc = math.cos(math.radians(theta_deg))
    m = meshes.ogrid2d(n_az, n_rad, N, center=(40.0, 40.0), Rc=Rc, half_width=40.0,
                       grading=2.0, jitter=0.1, seed=13, cos_cyl=cc, cos_box=0.0,
                       name="small_cyl")
    d = young_center_distance(Rc, R, theta_deg)
    return Case("small_cyl", m, LATTICE_D2Q9, x0=(40.0, 40.0 + d), R=R, seed=13, steps=100,
                wall_geom=dict(kind="circle", center=(40.0, 40.0), radius=Rc),
                theta_deg=theta_deg)


def small_sphere(theta_deg: float = 90.0, n_t: int = 2, n_rad: int = 2, N: int = 4) -> Case:
    """Cubed-sphere shell (R=10) in a 48^3 box with a Young cap, D3Q19."""
    Rs, R = 10.0, 8.0
    cs = math.cos(math.radians(theta_deg))
    m = meshes.cubed_sphere3d(n_t, n_rad, N, center=(24.0, 24.0, 24.0), Rs=Rs,
                              half_width=24.0, grading=2.0, jitter=0.1, seed=14,
                              cos_sphere=cs, cos_box=0.0, name="small_sphere")
    d = young_center_distance(Rs, R, theta_deg)
    return Case("small_sphere", m, LATTICE_D3Q19, x0=(24.0, 24.0, 24.0 + d), R=R, seed=14,
                steps=20, wall_geom=dict(kind="sphere", center=(24.0, 24.0, 24.0), radius=Rs),
                theta_deg=theta_deg)


def small_box3d(N: int = 3, n: int = 3, periodic=(True, True, True), jitter: float = 0.0) -> Case:
    """Periodic (or walled) cube of side 24 with a centred droplet, D3Q19."""
    m = meshes.box3d(n, n, n, N, (24.0, 24.0, 24.0), periodic=periodic, jitter=jitter, seed=15,
                     name="small_box3d")
    return Case("small_box3d", m, LATTICE_D3Q19, x0=(12.0, 12.0, 12.0), R=7.0, noise=1e-4,
                seed=15, steps=20)


def moving_walls(dim: int = 2) -> Case:
    """Droplet cap on a wetting wall that slides, under a lid that slides the other way
    (tangential wall velocities u_b of Eq. (9)): 2-D, a jittered 64x32 box of 8x4 quads at
    N = 5; 3-D, a jittered 24^3 box of 3^3 hexes at N = 3, periodic in x and y."""
    cb = math.cos(math.radians(70.0))
    if dim == 2:
        m = meshes.box2d(8, 4, 5, 64.0, 32.0, periodic=(False, False), jitter=0.2, seed=16,
                         cos_theta={"bottom": cb}, ub={"bottom": (-0.004, 0.0), "top": (0.01, 0.0)},
                         name="moving_walls")
        return Case("moving_walls", m, LATTICE_D2Q9, x0=(32.0, -12.0 * cb), R=12.0, seed=16,
                    steps=200, wall_geom=dict(kind="plane", point=(0.0, 0.0), normal=(0.0, -1.0)),
                    theta_deg=70.0)
    m = meshes.box3d(3, 3, 3, 3, (24.0, 24.0, 24.0), periodic=(True, True, False), jitter=0.1,
                     seed=17, cos_theta={"z-": cb},
                     ub={"z-": (-0.004, 0.002, 0.0), "z+": (0.01, 0.005, 0.0)}, name="moving_walls3d")
    return Case("moving_walls3d", m, LATTICE_D3Q19, x0=(12.0, 12.0, -8.0 * cb), R=8.0, seed=17,
                steps=20, wall_geom=dict(kind="plane", point=(0.0, 0.0, 0.0), normal=(0.0, 0.0, -1.0)),
                theta_deg=70.0)


def walled_droplet(nx: int = 8, N: int = 4, L: float = 64.0, R: float = 16.0,
                   delta: float = 6.0) -> Case:
    """Isolated droplet in a closed square box (non-wetting outer walls): the
    equilibration run whose kinetic energy decays to the residual floor."""
    m = meshes.box2d(nx, nx, N, L, L, periodic=(False, False), name="walled_droplet")
    return Case("walled_droplet", m, LATTICE_D2Q9, x0=(0.5 * L, 0.5 * L), R=R, delta=delta,
                steps=10500)


def spreading(theta_deg: float = 60.0, R: float = 24.0) -> Case:
    """Dynamic wetting: a droplet of radius R whose circle just touches a flat wall of
    equilibrium angle theta (16x8 square quads over a 128x64 walled box, N=6), so that it
    spreads (or retracts) from a 180-degree start to its equilibrium cap."""
    cb = math.cos(math.radians(theta_deg))
    m = meshes.box2d(16, 8, 6, 128.0, 64.0, periodic=(False, False), jitter=0.0, seed=21,
                     cos_theta={"bottom": cb}, name="spreading")
    return Case("spreading", m, LATTICE_D2Q9, x0=(64.0, R), R=R, seed=21, steps=30000,
                wall_geom=dict(kind="plane", point=(0.0, 0.0), normal=(0.0, -1.0)),
                theta_deg=theta_deg)


def paper_flat(theta_deg: float = 60.0, N: int = 16, nx: int = 16, ny: int = 8,
               La: float = 122.0) -> Case:
    """The flat-wall parasitic-current test of Sec. 3.1 in lattice units: 16x8 square quads
    over a 128x64 walled box (the domain read as 2 wide by 1 high), N = 16, a droplet of
    diameter D = 32 (half the height) and interface thickness delta = 1.92 (0.03 of the
    height), Laplace number La = sigma D / (rho_l nu^2) = 122.

    The droplet starts as its equilibrium cap: the circular segment at angle theta (through
    the liquid) with the area of the D circle, R^2 (theta - sin theta cos theta) = pi D^2/4.
    `nu` is the kinematic viscosity that gives La; the library sets the relaxation time
    tau = nu / (cs^2 dt) once the time step is known."""
    th = math.radians(theta_deg)
    cb = math.cos(th)
    D, sigma, rho_l = 32.0, 0.01, 1.0
    R = 0.5 * D * math.sqrt(math.pi / (th - math.sin(th) * cb))
    m = meshes.box2d(nx, ny, N, 128.0, 64.0, periodic=(False, False), jitter=0.0, seed=31,
                     cos_theta={"bottom": cb}, name=f"paper_flat_N{N}")
    c = Case(f"paper_flat_{theta_deg:g}", m, LATTICE_D2Q9, rho_l=rho_l, delta=1.92, sigma=sigma,
             x0=(64.0, -R * cb), R=R, seed=31, steps=0,
             wall_geom=dict(kind="plane", point=(0.0, 0.0), normal=(0.0, -1.0)), theta_deg=theta_deg,
             nu=math.sqrt(sigma * D / (rho_l * La)))
    return c


def paper_isolated(La: float = 61.5, N: int = 16, nel: int = 4) -> Case:
    """The boundary-free droplet test of Sec. 3.3 in lattice units: a droplet of diameter
    D = 32 at the centre of a 64x64 box of nel x nel square quads at order N (4x4 at N = 16,
    or 16x16 at N = 4: the same number of nodes), Cahn number delta / D = 0.063, Laplace
    number La = sigma D / (rho_l nu^2).  The box has non-wetting walls, since a fully
    periodic box leaves the uniform-momentum mode undamped.  `nu` gives La; the library
    sets tau = nu / (cs^2 dt) once dt is known."""
    D, sigma, rho_l = 32.0, 0.01, 1.0
    m = meshes.box2d(nel, nel, N, 64.0, 64.0, periodic=(False, False), name=f"paper_isolated_N{N}")
    return Case(f"paper_isolated_La{La:g}_N{N}", m, LATTICE_D2Q9, rho_l=rho_l, delta=0.063 * D,
                sigma=sigma, x0=(32.0, 32.0), R=0.5 * D, seed=33, steps=0,
                nu=math.sqrt(sigma * D / (rho_l * La)))


def lens_area(R: float, Rw: float, d: float) -> float:
    """Area of the intersection of two disks of radii R and Rw whose centres are d apart."""
    if d >= R + Rw:
        return 0.0
    if d <= abs(R - Rw):
        return math.pi * min(R, Rw) ** 2
    a = R * R * math.acos((d * d + R * R - Rw * Rw) / (2.0 * d * R))
    b = Rw * Rw * math.acos((d * d + Rw * Rw - R * R) / (2.0 * d * Rw))
    c = 0.5 * math.sqrt((-d + R + Rw) * (d + R - Rw) * (d - R + Rw) * (d + R + Rw))
    return a + b - c


def paper_curved(theta_deg: float = 90.0, N: int = 11, n_az: int = 32, n_rad: int = 8,
                 La: float = 341.0, jitter: float = 0.1, cn: float = 0.06) -> Case:
    """The curved-wall parasitic-current test of Sec. 3.2 in lattice units: a circular wall
    of diameter D = 25.6 (0.2 of the side) at the centre of a 128x128 walled box, meshed as
    a jittered O-grid (standing in for the paper's unstructured mesh), N = 11, La = 341,
    interface thickness delta = cn D (by default 0.06, the flat-wall test's ratio).

    The droplet starts as its equilibrium cap: the circle meeting the wall at theta (through
    the liquid) whose part outside the wall has the area of a diameter-D circle (bisection
    on its radius).  `nu` gives La; the library sets tau = nu / (cs^2 dt)."""
    D, sigma, rho_l = 25.6, 0.01, 1.0
    Rw, A0 = 0.5 * D, math.pi * (0.5 * D) ** 2
    lo, hi = 1e-3 * Rw, 50.0 * Rw
    for _ in range(200):
        R = 0.5 * (lo + hi)
        d = young_center_distance(Rw, R, theta_deg)
        if math.pi * R * R - lens_area(R, Rw, d) < A0:
            lo = R
        else:
            hi = R
    R = 0.5 * (lo + hi)
    d = young_center_distance(Rw, R, theta_deg)
    cc = math.cos(math.radians(theta_deg))
    m = meshes.ogrid2d(n_az, n_rad, N, center=(64.0, 64.0), Rc=Rw, half_width=64.0,
                       grading=2.0, jitter=jitter, seed=32, cos_cyl=cc, cos_box=0.0,
                       name=f"paper_curved_N{N}")
    return Case(f"paper_curved_{theta_deg:g}", m, LATTICE_D2Q9, rho_l=rho_l, delta=cn * D,
                sigma=sigma, x0=(64.0, 64.0 + d), R=R, seed=32, steps=0,
                wall_geom=dict(kind="circle", center=(64.0, 64.0), radius=Rw),
                theta_deg=theta_deg, nu=math.sqrt(sigma * D / (rho_l * La)))


ORDERS_2D = (2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 14, 16)
ORDERS_3D = (2, 3, 4, 5, 6)


def _lattice_key(dim: int):
    """2 -> (2, D2Q9), 3 -> (3, D3Q19), 13 -> (3, D3Q13)."""
    return (3, LATTICE_D3Q13) if dim == 13 else (dim, LATTICE_D2Q9 if dim == 2 else LATTICE_D3Q19)


def order_case(dim: int, N: int) -> Case:
    """Small walled, jittered mesh of order N for the order sweep: a 70-degree wetting
    wall and a sessile cap, 5x3 quads (2-D) or 2x3x2 hexes (3-D); dim 13 is the 3-D mesh
    with the D3Q13 lattice.  The element counts are not multiples of the wide block sizes,
    so wide launches end ragged."""
    dim, lat = _lattice_key(dim)
    cb = math.cos(math.radians(70.0))
    if dim == 2:
        return small_flat(theta_deg=70.0, nx=5, ny=3, N=N, Lx=40.0, Ly=24.0, R=9.0)
    m = meshes.box3d(2, 3, 2, N, (16.0, 24.0, 16.0), periodic=(True, False, True), jitter=0.15,
                     seed=16, cos_theta={"y-": cb}, name=f"order3d_N{N}")
    R = 7.0
    return Case(f"order3d_N{N}", m, lat, x0=(8.0, -R * cb, 8.0), R=R, seed=16, steps=10,
                wall_geom=dict(kind="plane", point=(0.0, 0.0, 0.0), normal=(0.0, -1.0, 0.0)),
                theta_deg=70.0)


def wide_case(dim: int, N: int) -> Case:
    """Mesh of order N large enough that a single solve launches its element kernels in
    wide blocks (at least 256 blocks of 256 // (N+1)^d elements) with a ragged last block:
    a walled jittered box (2-D, 70-degree wetting bottom wall) or a periodic-x walled-y
    box (3-D; dim 13: with the D3Q13 lattice)."""
    dim, lat = _lattice_key(dim)
    nloc = (N + 1) ** dim
    epb = max(1, 256 // nloc)
    E = 256 * epb + max(1, epb // 2)
    if dim == 2:
        ny = max(2, int(round((E / 2) ** 0.5)))
        nx = -(-E // ny)
        return small_flat(theta_deg=70.0, nx=nx, ny=ny, N=N, Lx=8.0 * nx, Ly=8.0 * ny,
                          R=min(3.0 * ny, 24.0))
    n = max(2, int(round(E ** (1.0 / 3.0))))
    nz = -(-E // (n * n))
    cb = math.cos(math.radians(70.0))
    m = meshes.box3d(n, n, nz, N, (6.0 * n, 6.0 * n, 6.0 * nz), periodic=(True, False, True),
                     jitter=0.1, seed=17, cos_theta={"y-": cb}, name=f"wide3d_N{N}")
    R = 2.0 * n
    return Case(f"wide3d_N{N}", m, lat, x0=(3.0 * n, -R * cb, 3.0 * nz), R=R, seed=17,
                steps=3, wall_geom=dict(kind="plane", point=(0.0, 0.0, 0.0), normal=(0.0, -1.0, 0.0)),
                theta_deg=70.0)


def c4q13() -> Case:
    """c4's mesh and droplet with the paper's 3-D lattice size: D3Q13 (13 populations)."""
    return c4(lattice=LATTICE_D3Q13)


def c4n6() -> Case:
    """c4's mesh and droplet at N = 6 (343 nodes per hex, about 5.27 M global nodes): the
    highest 3-D order, whose streaming kernel runs two nodes on some lanes."""
    c = c4(N=6)
    c.name = "c4n6"
    return c


def flat16() -> Case:
    """2-D N = 16 (289 nodes per quad) on an 85x42-element walled jittered box of 680x336
    with a 70-degree wetting floor, about 1.03 M local nodes (fused kernels, B and D with two
    nodes on some lanes)."""
    c = small_flat(theta_deg=70.0, nx=85, ny=42, N=16, Lx=680.0, Ly=336.0, R=84.0)
    c.name = "flat16"
    return c


CASES = {"c1": c1, "c2": c2, "c3": c3, "c4": c4, "c2xl": c2xl, "c4q13": c4q13, "c4n6": c4n6,
         "flat16": flat16}


def sizes(case: Case) -> dict:
    m = case.mesh
    return dict(E=m.E, N=m.N, n_local=m.n_local, n_global=m.n_global, Q=case.lattice,
                walls=int(m.wall_face.shape[0]))


def request_stream(n_req: int = 256, seed: int = 5):
    """Serving workload: seeded list of 2-D droplet requests.

    Each entry: geometry 'flat' or 'cyl' (p = 1/2), element counts from the
    allowed list, N in {4,6,8}, theta ~ U[30,150] deg, R ~ U[10,30] clipped so
    the cap stays clear of the other walls, and a Poisson arrival time at unit
    mean rate (scale it to the wanted rate).
    """
    rng = np.random.default_rng(seed)
    sizes_ = [(8, 8), (16, 8), (16, 16), (32, 16), (32, 32), (64, 32)]
    out = []
    t = 0.0
    for k in range(n_req):
        t += rng.exponential(1.0)
        geom = "flat" if rng.random() < 0.5 else "cyl"
        nx, ny = sizes_[rng.integers(len(sizes_))]
        N = int(rng.choice([4, 6, 8]))
        theta = float(rng.uniform(30.0, 150.0))
        R = float(rng.uniform(10.0, 30.0))
        out.append(dict(id=k, t_arrive=t, geom=geom, nx=nx, ny=ny, N=N, theta_deg=theta, R=R))
    return out


def request_case(req: dict, delta: float = 4.0) -> Case:
    """Build the Case of one serving request (see :func:`request_stream`)."""
    theta = req["theta_deg"]
    c = math.cos(math.radians(theta))
    R = req["R"]
    N = req["N"]
    nx, ny = req["nx"], req["ny"]
    if req["geom"] == "flat":
        h = 8.0
        Lx, Ly = nx * h, ny * h
        # keep the cap clear of the side and top walls by 2 delta
        Rmax_x = (0.5 * Lx - 2.0 * delta)
        top = Ly - 2.0 * delta
        Rmax_y = top / (1.0 - c) if c < 1.0 else top
        R = min(R, Rmax_x, Rmax_y)
        m = meshes.box2d(nx, ny, N, Lx, Ly, periodic=(False, False), jitter=0.0,
                         cos_theta={"bottom": c}, name="req_flat")
        return Case(f"req{req['id']}", m, LATTICE_D2Q9, delta=delta, x0=(0.5 * Lx, -R * c),
                    R=R, seed=1000 + req["id"], steps=50000,
                    wall_geom=dict(kind="plane", point=(0.0, 0.0), normal=(0.0, -1.0)),
                    theta_deg=theta)
    Rc = R
    half = Rc + 2.0 * R + 3.0 * delta
    n_az = 4 * max(1, nx // 2)
    n_rad = max(1, ny // 2)
    m = meshes.ogrid2d(n_az, n_rad, N, center=(half, half), Rc=Rc, half_width=half,
                       grading=2.0, jitter=0.0, cos_cyl=c, cos_box=0.0, name="req_cyl")
    d = young_center_distance(Rc, R, theta)
    return Case(f"req{req['id']}", m, LATTICE_D2Q9, delta=delta, x0=(half, half + d), R=R,
                seed=1000 + req["id"], steps=50000,
                wall_geom=dict(kind="circle", center=(half, half), radius=Rc), theta_deg=theta)

"""Seeded synthetic spectral-element meshes.

Each generator returns a :class:`Mesh`: the coordinates of every element's
(N+1)^d Gauss-Lobatto-Legendre (GLL) nodes, the local-to-global node map, and
the list of physical wall faces with their imposed contact angle and wall
velocity.  Nothing here evaluates any operator of the lattice Boltzmann method;
the module only places nodes, so the CPU oracle and the GPU library can both be
fed the same inputs without sharing any arithmetic of the method.

Conventions (they are also the library's input format):

* local node index ``n = i + (N+1) j (+ (N+1)^2 k)``, ``i`` along the first
  reference direction xi, ``j`` along eta, ``k`` along zeta; every element map
  has a positive Jacobian (right-handed reference frame);
* faces are numbered ``0..2d-1`` = xi-, xi+, eta-, eta+, zeta-, zeta+;
* nodes shared between elements carry bitwise-equal coordinates, except across
  a periodic wrap, where the copies differ by the period (the global id is
  what identifies them);
* the paper's curved walls are represented isoparametrically: node positions
  come from a smooth map evaluated at GLL points of a (possibly jittered)
  parameter-space element, so wall nodes lie exactly on the circle or sphere.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

FACE_XI_M, FACE_XI_P, FACE_ETA_M, FACE_ETA_P, FACE_ZETA_M, FACE_ZETA_P = range(6)


@dataclass
class Mesh:
    dim: int
    N: int
    xyz: np.ndarray          # [E, (N+1)^d, d] float64
    gid: np.ndarray          # [E, (N+1)^d] int32
    n_global: int
    wall_face: np.ndarray    # [F, 2] int32: (element, face)
    wall_cos: np.ndarray     # [F] float64: cos(theta_eq) of the face
    wall_ub: np.ndarray      # [F, d] float64: wall velocity
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def E(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def nloc(self) -> int:
        return int(self.xyz.shape[1])

    @property
    def n_local(self) -> int:
        return self.E * self.nloc

    def first_copy_coords(self) -> np.ndarray:
        """Coordinates of each global node taken from its lowest local copy."""
        flat_gid = self.gid.reshape(-1)
        flat_xyz = self.xyz.reshape(-1, self.dim)
        out = np.empty((self.n_global, self.dim))
        seen = np.zeros(self.n_global, dtype=bool)
        order = np.arange(flat_gid.size)
        # lowest local index wins: write in reverse so the smallest index is last
        rev = order[::-1]
        out[flat_gid[rev]] = flat_xyz[rev]
        seen[flat_gid] = True
        assert seen.all(), "global ids are not contiguous"
        return out

    def check(self) -> None:
        """Structural self-checks of the input (not of the method)."""
        d, Np = self.dim, self.N + 1
        assert self.xyz.shape == (self.E, Np ** d, d)
        assert self.gid.shape == (self.E, Np ** d)
        assert self.gid.min() == 0 and self.gid.max() == self.n_global - 1
        assert np.unique(self.gid).size == self.n_global
        assert self.wall_face.shape[1] == 2
        assert self.wall_cos.shape == (self.wall_face.shape[0],)
        assert self.wall_ub.shape == (self.wall_face.shape[0], d)


def gll_points(N: int) -> np.ndarray:
    """GLL node positions on [-1, 1], used only to place mesh nodes."""
    if N < 1:
        raise ValueError("N >= 1")
    from numpy.polynomial import legendre as L

    c = np.zeros(N + 1)
    c[N] = 1.0
    r = np.sort(np.real(L.legroots(L.legder(c)))) if N > 1 else np.zeros(0)
    x = np.concatenate([[-1.0], r, [1.0]])
    x = 0.5 * (x - x[::-1])
    x[0], x[-1] = -1.0, 1.0
    if N % 2 == 0:
        x[N // 2] = 0.0
    return x


# ----------------------------------------------------------------------------
# 2-D structured boxes (periodic or walled, optionally jittered)
# ----------------------------------------------------------------------------

def _bilinear(v00, v10, v01, v11, s, t):
    """Bilinear interpolation on [-1,1]^2 (s along first, t along second)."""
    a = (1.0 - s) * (1.0 - t)
    b = (1.0 + s) * (1.0 - t)
    c = (1.0 - s) * (1.0 + t)
    dd = (1.0 + s) * (1.0 + t)
    return 0.25 * (a * v00 + b * v10 + c * v01 + dd * v11)


def box2d(nx: int, ny: int, N: int, Lx: float, Ly: float, *,
          periodic=(False, False), jitter: float = 0.0, seed: int = 0,
          cos_theta=None, ub=None, origin=(0.0, 0.0), name: str = "") -> Mesh:
    """Rectangle [x0, x0+Lx] x [y0, y0+Ly] of nx x ny straight-sided quads.

    ``jitter`` moves every interior vertex (and, along a periodic direction,
    the wrapped vertices consistently) by U[-jitter, jitter] times the element
    width per component, seeded; boundary vertices stay fixed.
    ``cos_theta``/``ub``: dicts keyed by 'bottom', 'right', 'top', 'left'.
    """
    cos_theta = dict(cos_theta or {})
    ub = dict(ub or {})
    px, py = periodic
    hx, hy = Lx / nx, Ly / ny
    vx = origin[0] + hx * np.arange(nx + 1)[:, None] * np.ones((1, ny + 1))
    vy = origin[1] + hy * np.arange(ny + 1)[None, :] * np.ones((nx + 1, 1))
    if jitter > 0.0:
        rng = np.random.default_rng(seed)
        jx = rng.uniform(-jitter, jitter, size=(nx + 1, ny + 1)) * hx
        jy = rng.uniform(-jitter, jitter, size=(nx + 1, ny + 1)) * hy
        movable = np.ones((nx + 1, ny + 1), dtype=bool)
        if not px:
            movable[0, :] = movable[nx, :] = False
        if not py:
            movable[:, 0] = movable[:, ny] = False
        jx = np.where(movable, jx, 0.0)
        jy = np.where(movable, jy, 0.0)
        if px:  # wrapped column equals column 0
            jx[nx, :] = jx[0, :]
            jy[nx, :] = jy[0, :]
        if py:
            jx[:, ny] = jx[:, 0]
            jy[:, ny] = jy[:, 0]
        vx = vx + jx
        vy = vy + jy
    xi = gll_points(N)
    nIx, nIy = nx * N + 1, ny * N + 1
    I = np.arange(nIx)
    ex = np.minimum(I // N, nx - 1)
    p = I - ex * N
    J = np.arange(nIy)
    ey = np.minimum(J // N, ny - 1)
    q = J - ey * N
    EX, EY = np.meshgrid(ex, ey, indexing="ij")
    S, T = np.meshgrid(xi[p], xi[q], indexing="ij")
    X = _bilinear(vx[EX, EY], vx[EX + 1, EY], vx[EX, EY + 1], vx[EX + 1, EY + 1], S, T)
    Y = _bilinear(vy[EX, EY], vy[EX + 1, EY], vy[EX, EY + 1], vy[EX + 1, EY + 1], S, T)
    # wrapped global numbering
    nGx = nx * N if px else nIx
    nGy = ny * N if py else nIy
    Np = N + 1
    E = nx * ny
    xyz = np.empty((E, Np * Np, 2))
    gid = np.empty((E, Np * Np), dtype=np.int64)
    ii, jj = np.meshgrid(np.arange(Np), np.arange(Np), indexing="xy")  # jj rows, ii cols
    ii = ii.reshape(-1)  # n = i + Np*j  -> ii varies fastest
    jj = jj.reshape(-1)
    for eyy in range(ny):
        for exx in range(nx):
            e = exx + nx * eyy
            Ig = exx * N + ii
            Jg = eyy * N + jj
            xyz[e, :, 0] = X[Ig, Jg]
            xyz[e, :, 1] = Y[Ig, Jg]
            gid[e] = (Ig % nGx) + nGx * (Jg % nGy)
    faces, cth, ubs = [], [], []

    def add(side, elems, face):
        for e in elems:
            faces.append((e, face))
            cth.append(float(cos_theta.get(side, 0.0)))
            ubs.append(tuple(ub.get(side, (0.0, 0.0))))

    if not py:
        add("bottom", [exx for exx in range(nx)], FACE_ETA_M)
    if not px:
        add("right", [nx - 1 + nx * eyy for eyy in range(ny)], FACE_XI_P)
    if not py:
        add("top", [exx + nx * (ny - 1) for exx in range(nx)], FACE_ETA_P)
    if not px:
        add("left", [nx * eyy for eyy in range(ny)], FACE_XI_M)
    m = Mesh(2, N, xyz, gid.astype(np.int32), nGx * nGy,
             np.array(faces, dtype=np.int32).reshape(-1, 2),
             np.array(cth, dtype=np.float64),
             np.array(ubs, dtype=np.float64).reshape(-1, 2), name=name,
             meta=dict(kind="box2d", nx=nx, ny=ny, Lx=Lx, Ly=Ly, periodic=periodic,
                       origin=origin, jitter=jitter))
    m.check()
    return m


# ----------------------------------------------------------------------------
# 2-D O-grid around a cylinder inside a square box
# ----------------------------------------------------------------------------

def ogrid2d(n_az: int, n_rad: int, N: int, *, center=(128.0, 128.0), Rc: float = 40.0,
            half_width: float = 128.0, grading: float = 1.0, jitter: float = 0.0,
            seed: int = 0, cos_cyl: float = 0.0, cos_box: float = 0.0,
            name: str = "") -> Mesh:
    """Cylinder of radius ``Rc`` in the square ``center +- half_width``.

    Four O-grid blocks (one per box side), ``n_az`` elements around the whole
    cylinder (a multiple of 4) and ``n_rad`` radially.  The element map is the
    ruled surface between the circle (equiangular) and the box side
    (equispaced), which is the Gordon-Hall transfinite map for straight block
    edges.  ``grading`` > 1 clusters elements toward the cylinder.  Reference
    xi runs radially outward and eta counter-clockwise, so the cylinder is face
    xi- and the box is face xi+.  Interior vertices are jittered in parameter
    space by up to ``jitter`` of the local parametric element size.
    """
    if n_az % 4:
        raise ValueError("n_az must be a multiple of 4")
    cx, cy = center
    per_block = n_az // 4
    xi = gll_points(N)
    # vertex parameters: s in [0, n_az) (periodic), r in [0, n_rad]
    vs = np.arange(n_az + 1, dtype=np.float64)[:, None] * np.ones((1, n_rad + 1))
    vr = np.arange(n_rad + 1, dtype=np.float64)[None, :] * np.ones((n_az + 1, 1))
    if jitter > 0.0:
        rng = np.random.default_rng(seed)
        js = rng.uniform(-jitter, jitter, size=(n_az + 1, n_rad + 1))
        jr = rng.uniform(-jitter, jitter, size=(n_az + 1, n_rad + 1))
        mov = np.ones((n_az + 1, n_rad + 1), dtype=bool)
        mov[:, 0] = mov[:, n_rad] = False
        # keep block-corner radial lines straight (the four diagonals)
        mov[::per_block, :] = False
        js = np.where(mov, js, 0.0)
        jr = np.where(mov, jr, 0.0)
        js[n_az, :] = js[0, :]
        jr[n_az, :] = jr[0, :]
        vs = vs + js
        vr = vr + jr

    def phys(s, r):
        b = np.floor(s / per_block).astype(np.int64)
        b = np.clip(b, 0, 3)
        t = (s - b * per_block) / per_block
        phi = -0.25 * np.pi + (b + t) * (0.5 * np.pi)
        ix = cx + Rc * np.cos(phi)
        iy = cy + Rc * np.sin(phi)
        u = 2.0 * t - 1.0
        # box side point of block b: rotate (1, u) by b quarter turns
        ox = np.where(b == 0, 1.0, np.where(b == 1, -u, np.where(b == 2, -1.0, u)))
        oy = np.where(b == 0, u, np.where(b == 1, 1.0, np.where(b == 2, -u, -1.0)))
        ox = cx + half_width * ox
        oy = cy + half_width * oy
        rr = r / n_rad
        if grading != 1.0:
            rr = (np.power(grading, rr) - 1.0) / (grading - 1.0)
        return (1.0 - rr) * ix + rr * ox, (1.0 - rr) * iy + rr * oy

    Np = N + 1
    nIs, nIr = n_az * N + 1, n_rad * N + 1
    I = np.arange(nIs)
    es = np.minimum(I // N, n_az - 1)
    p = I - es * N
    J = np.arange(nIr)
    er = np.minimum(J // N, n_rad - 1)
    q = J - er * N
    ES, ER = np.meshgrid(es, er, indexing="ij")
    Pp, Qq = np.meshgrid(xi[p], xi[q], indexing="ij")
    # parameter-space element: first local direction = radial (xi), second = azimuth (eta)
    S = _bilinear(vs[ES, ER], vs[ES, ER + 1], vs[ES + 1, ER], vs[ES + 1, ER + 1], Qq, Pp)
    R = _bilinear(vr[ES, ER], vr[ES, ER + 1], vr[ES + 1, ER], vr[ES + 1, ER + 1], Qq, Pp)
    X, Y = phys(S, R)
    # the wrapped azimuthal column is the same physical point as column 0
    X[nIs - 1, :] = X[0, :]
    Y[nIs - 1, :] = Y[0, :]
    nGs = n_az * N
    E = n_az * n_rad
    xyz = np.empty((E, Np * Np, 2))
    gid = np.empty((E, Np * Np), dtype=np.int64)
    n = np.arange(Np * Np)
    li = n % Np  # radial local index
    lj = n // Np  # azimuthal local index
    for a in range(n_az):
        for rj in range(n_rad):
            e = rj + n_rad * a
            Is = a * N + lj
            Ir = rj * N + li
            xyz[e, :, 0] = X[Is, Ir]
            xyz[e, :, 1] = Y[Is, Ir]
            gid[e] = (Is % nGs) * nIr + Ir
    faces, cth = [], []
    for a in range(n_az):
        faces.append((0 + n_rad * a, FACE_XI_M))
        cth.append(cos_cyl)
    for a in range(n_az):
        faces.append((n_rad - 1 + n_rad * a, FACE_XI_P))
        cth.append(cos_box)
    m = Mesh(2, N, xyz, gid.astype(np.int32), nGs * nIr,
             np.array(faces, dtype=np.int32), np.array(cth, dtype=np.float64),
             np.zeros((len(faces), 2)), name=name,
             meta=dict(kind="ogrid2d", n_az=n_az, n_rad=n_rad, center=center, Rc=Rc,
                       half_width=half_width, grading=grading, jitter=jitter))
    m.check()
    return m


# ----------------------------------------------------------------------------
# 3-D structured boxes (periodic or walled)
# ----------------------------------------------------------------------------

def _trilinear(v, s, t, u):
    """v: [2,2,2] corner values (index [a][b][c] for s,t,u = -1/+1)."""
    out = 0.0
    for a, fa in ((0, 1.0 - s), (1, 1.0 + s)):
        for b, fb in ((0, 1.0 - t), (1, 1.0 + t)):
            for c, fc in ((0, 1.0 - u), (1, 1.0 + u)):
                out = out + fa * fb * fc * v[a][b][c]
    return 0.125 * out


def box3d(nx: int, ny: int, nz: int, N: int, L=(1.0, 1.0, 1.0), *,
          periodic=(True, True, True), jitter: float = 0.0, seed: int = 0,
          cos_theta=None, ub=None, origin=(0.0, 0.0, 0.0), name: str = "") -> Mesh:
    """Cuboid of nx x ny x nz trilinear hexes; walls on non-periodic sides.

    ``cos_theta`` and ``ub`` (wall velocity) keys: 'x-', 'x+', 'y-', 'y+', 'z-', 'z+'.
    """
    cos_theta = dict(cos_theta or {})
    ub = dict(ub or {})
    nel = (nx, ny, nz)
    h = [L[a] / nel[a] for a in range(3)]
    shape = (nx + 1, ny + 1, nz + 1)
    V = np.stack(np.meshgrid(*[origin[a] + h[a] * np.arange(nel[a] + 1) for a in range(3)],
                             indexing="ij"), axis=-1)
    if jitter > 0.0:
        rng = np.random.default_rng(seed)
        jit = rng.uniform(-jitter, jitter, size=shape + (3,)) * np.array(h)
        mov = np.ones(shape, dtype=bool)
        for a in range(3):
            if not periodic[a]:
                sl = [slice(None)] * 3
                sl[a] = 0
                mov[tuple(sl)] = False
                sl[a] = nel[a]
                mov[tuple(sl)] = False
        jit = np.where(mov[..., None], jit, 0.0)
        for a in range(3):
            if periodic[a]:
                src = [slice(None)] * 3
                dst = [slice(None)] * 3
                src[a] = 0
                dst[a] = nel[a]
                jit[tuple(dst)] = jit[tuple(src)]
        V = V + jit
    xi = gll_points(N)
    Np = N + 1
    nI = [nel[a] * N + 1 for a in range(3)]
    idx = []
    for a in range(3):
        I = np.arange(nI[a])
        ea = np.minimum(I // N, nel[a] - 1)
        idx.append((ea, xi[I - ea * N]))
    EA, EB, EC = np.meshgrid(idx[0][0], idx[1][0], idx[2][0], indexing="ij")
    S, T, U = np.meshgrid(idx[0][1], idx[1][1], idx[2][1], indexing="ij")
    X = np.empty(tuple(nI) + (3,))
    for c in range(3):
        corners = [[[V[EA + a, EB + b, EC + cc, c] for cc in (0, 1)] for b in (0, 1)] for a in (0, 1)]
        X[..., c] = _trilinear(corners, S, T, U)
    nG = [nel[a] * N if periodic[a] else nI[a] for a in range(3)]
    E = nx * ny * nz
    xyz = np.empty((E, Np ** 3, 3))
    gid = np.empty((E, Np ** 3), dtype=np.int64)
    n = np.arange(Np ** 3)
    li, lj, lk = n % Np, (n // Np) % Np, n // (Np * Np)
    for ez in range(nz):
        for ey in range(ny):
            for ex in range(nx):
                e = ex + nx * (ey + ny * ez)
                Ig, Jg, Kg = ex * N + li, ey * N + lj, ez * N + lk
                xyz[e] = X[Ig, Jg, Kg]
                gid[e] = (Ig % nG[0]) + nG[0] * ((Jg % nG[1]) + nG[1] * (Kg % nG[2]))
    faces, cth, ubs = [], [], []
    for a, (lo, hi) in enumerate((("x-", "x+"), ("y-", "y+"), ("z-", "z+"))):
        if periodic[a]:
            continue
        for ez in range(nz):
            for ey in range(ny):
                for ex in range(nx):
                    e = ex + nx * (ey + ny * ez)
                    ec = (ex, ey, ez)[a]
                    if ec == 0:
                        faces.append((e, 2 * a))
                        cth.append(float(cos_theta.get(lo, 0.0)))
                        ubs.append(tuple(ub.get(lo, (0.0, 0.0, 0.0))))
                    if ec == nel[a] - 1:
                        faces.append((e, 2 * a + 1))
                        cth.append(float(cos_theta.get(hi, 0.0)))
                        ubs.append(tuple(ub.get(hi, (0.0, 0.0, 0.0))))
    m = Mesh(3, N, xyz, gid.astype(np.int32), int(np.prod(nG)),
             np.array(faces, dtype=np.int32).reshape(-1, 2),
             np.array(cth, dtype=np.float64), np.array(ubs, dtype=np.float64).reshape(-1, 3),
             name=name,
             meta=dict(kind="box3d", nel=nel, L=L, periodic=periodic, origin=origin,
                       jitter=jitter))
    m.check()
    return m


# ----------------------------------------------------------------------------
# 3-D cubed-sphere shell: sphere inside a cube
# ----------------------------------------------------------------------------

# cube faces: (normal axis, sign, tangential axis 1, tangential axis 2) chosen so that
# (t1, t2, outward normal) is right-handed
_CUBE_FACES = [
    (0, +1, 1, 2), (0, -1, 2, 1),
    (1, +1, 2, 0), (1, -1, 0, 2),
    (2, +1, 0, 1), (2, -1, 1, 0),
]


def cubed_sphere3d(n_t: int, n_rad: int, N: int, *, center=(64.0, 64.0, 64.0),
                   Rs: float = 30.0, half_width: float = 64.0, grading: float = 1.0,
                   jitter: float = 0.0, seed: int = 0, cos_sphere: float = 0.0,
                   cos_box: float = 0.0, name: str = "") -> Mesh:
    """Sphere of radius ``Rs`` inside the cube ``center +- half_width``.

    Six blocks of ``n_t x n_t`` (equiangular on the sphere, equispaced on the
    cube faces) times ``n_rad`` radial layers, blended linearly along rays.
    Reference xi, eta are the face-tangential directions and zeta is radial
    outward, so the sphere is face zeta- and the box is face zeta+.
    Jitter moves interior radial levels only (seeded, up to ``jitter`` of a
    layer), keeping the tangential structure conforming across block edges.
    """
    M = n_t * N  # lattice points per cube edge minus one
    xi = gll_points(N)
    # global surface lattice: points (a,b,c) in [0,M]^3 on the cube surface
    # parametric position of lattice index I along an edge: element + GLL offset
    I = np.arange(M + 1)
    eI = np.minimum(I // N, n_t - 1)
    par = (eI + 0.5 * (1.0 + xi[I - eI * N])) / n_t  # in [0, 1]
    par[0], par[-1] = 0.0, 1.0
    q = 2.0 * par - 1.0  # in [-1, 1]

    # unique surface points
    key_of = {}
    surf_q = []
    face_pts = []
    for (ax, sg, t1, t2) in _CUBE_FACES:
        A, B = np.meshgrid(np.arange(M + 1), np.arange(M + 1), indexing="ij")
        lat = np.zeros((M + 1, M + 1, 3), dtype=np.int64)
        lat[..., ax] = M if sg > 0 else 0
        lat[..., t1] = A
        lat[..., t2] = B
        keys = (lat[..., 0] * (M + 1) + lat[..., 1]) * (M + 1) + lat[..., 2]
        ids = np.empty((M + 1, M + 1), dtype=np.int64)
        for a in range(M + 1):
            for b in range(M + 1):
                k = int(keys[a, b])
                if k not in key_of:
                    key_of[k] = len(surf_q)
                    surf_q.append(tuple(q[lat[a, b, c]] for c in range(3)))
                ids[a, b] = key_of[k]
        face_pts.append(ids)
    surf_q = np.array(surf_q)  # [Ns, 3] cube-surface coordinates in [-1,1]
    # direction on the sphere (equiangular): tan(pi/4 * q) on tangential axes
    cube_eq = np.where(np.abs(surf_q) == 1.0, surf_q, np.tan(0.25 * np.pi * surf_q))
    dirs = cube_eq / np.linalg.norm(cube_eq, axis=1, keepdims=True)
    Ns = surf_q.shape[0]
    nK = n_rad * N + 1
    K = np.arange(nK)
    eK = np.minimum(K // N, n_rad - 1)
    kpar = eK + 0.5 * (1.0 + xi[K - eK * N])  # in [0, n_rad]
    if jitter > 0.0:
        rng = np.random.default_rng(seed)
        lev = np.arange(n_rad + 1, dtype=np.float64)
        lev[1:-1] += rng.uniform(-jitter, jitter, size=n_rad - 1)
        kpar = lev[eK] + 0.5 * (1.0 + xi[K - eK * N]) * (lev[eK + 1] - lev[eK])
    rr = kpar / n_rad
    rr[0], rr[-1] = 0.0, 1.0
    if grading != 1.0:
        rr = (np.power(grading, rr) - 1.0) / (grading - 1.0)
    c = np.asarray(center, dtype=np.float64)
    inner = c[None, :] + Rs * dirs                     # [Ns, 3]
    outer = c[None, :] + half_width * surf_q           # [Ns, 3]
    Np = N + 1
    E = 6 * n_t * n_t * n_rad
    xyz = np.empty((E, Np ** 3, 3))
    gid = np.empty((E, Np ** 3), dtype=np.int64)
    n = np.arange(Np ** 3)
    li, lj, lk = n % Np, (n // Np) % Np, n // (Np * Np)
    e = 0
    faces = []
    for f in range(6):
        ids = face_pts[f]
        for kr in range(n_rad):
            for b in range(n_t):
                for a in range(n_t):
                    sidx = ids[a * N + li, b * N + lj]
                    Kg = kr * N + lk
                    w = rr[Kg][:, None]
                    xyz[e] = (1.0 - w) * inner[sidx] + w * outer[sidx]
                    gid[e] = sidx * nK + Kg
                    if kr == 0:
                        faces.append((e, FACE_ZETA_M))
                    if kr == n_rad - 1:
                        faces.append((e, FACE_ZETA_P))
                    e += 1
    faces = np.array(faces, dtype=np.int32)
    cth = np.where(faces[:, 1] == FACE_ZETA_M, cos_sphere, cos_box).astype(np.float64)
    m = Mesh(3, N, xyz, gid.astype(np.int32), Ns * nK, faces, cth,
             np.zeros((faces.shape[0], 3)), name=name,
             meta=dict(kind="cubed_sphere3d", n_t=n_t, n_rad=n_rad, center=center, Rs=Rs,
                       half_width=half_width, grading=grading, jitter=jitter))
    m.check()
    return m

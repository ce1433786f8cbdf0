"""Geometric contact-angle measurement (test infrastructure only).

The paper measures the equilibrium angle "geometrically" with an external
method it does not restate (Sec. 3.1).  Reading used here: collect the points
where the density crosses the mid value (rho_l + rho_v)/2 by linear
interpolation between neighbouring GLL nodes along element lines, drop those
within two interface widths of the wall, fit a circle (sphere in 3-D) by the
algebraic least-squares method of Kasa (1976), and intersect it with the wall:

* plane with outward fluid normal n through p0: cos(theta) = ((c - p0).n) / R;
* circle/sphere of radius Rw centred at cw, droplet centre at distance d:
  cos(theta) = (Rw^2 + R^2 - d^2) / (2 R Rw)  (law of cosines at the contact
  line), theta measured through the liquid.
"""
from __future__ import annotations

import numpy as np


def interface_points(xyz, gid, N, rho, level):
    """Mid-density crossings along element lines, one per global node pair."""
    E, nloc, dim = xyz.shape
    Np = N + 1
    pts = []
    seen = set()
    for e in range(E):
        for a in range(dim):
            s = Np ** a
            for n in range(nloc):
                if (n // s) % Np == N:
                    continue
                g1, g2 = int(gid[e, n]), int(gid[e, n + s])
                key = (min(g1, g2), max(g1, g2))
                if key in seen:
                    continue
                r1, r2 = rho[g1] - level, rho[g2] - level
                if r1 == 0.0 and r2 == 0.0:
                    continue
                if r1 * r2 > 0.0:
                    continue
                seen.add(key)
                t = r1 / (r1 - r2)
                pts.append(xyz[e, n] + t * (xyz[e, n + s] - xyz[e, n]))
    return np.array(pts).reshape(-1, dim)


def fit_circle(pts):
    """Kasa algebraic fit: |x|^2 + b.x + c = 0 in least squares -> (centre, radius)."""
    dim = pts.shape[1]
    A = np.concatenate([pts, np.ones((pts.shape[0], 1))], axis=1)
    rhs = -np.sum(pts * pts, axis=1)
    sol, *_ = np.linalg.lstsq(A, rhs, rcond=None)
    c = -0.5 * sol[:dim]
    R = np.sqrt(np.dot(c, c) - sol[dim])
    return c, R


def wall_distance(pts, wall):
    kind = wall["kind"]
    if kind == "plane":
        n = np.asarray(wall["normal"], dtype=np.float64)
        p0 = np.asarray(wall["point"], dtype=np.float64)
        return np.abs((pts - p0) @ n)
    c = np.asarray(wall["center"], dtype=np.float64)
    return np.linalg.norm(pts - c, axis=1) - wall["radius"]


def angle_from_fit(c, R, wall):
    kind = wall["kind"]
    if kind == "plane":
        n = np.asarray(wall["normal"], dtype=np.float64)
        p0 = np.asarray(wall["point"], dtype=np.float64)
        cth = float(np.dot(c - p0, n)) / R
    else:
        cw = np.asarray(wall["center"], dtype=np.float64)
        Rw = float(wall["radius"])
        d = float(np.linalg.norm(c - cw))
        cth = (Rw * Rw + R * R - d * d) / (2.0 * R * Rw)
    return float(np.degrees(np.arccos(np.clip(cth, -1.0, 1.0))))


def contact_angle(mesh, rho, rho_l, rho_v, delta, wall):
    """Contact angle in degrees of the droplet described by ``rho`` (global nodes)."""
    level = 0.5 * (rho_l + rho_v)
    pts = interface_points(mesh.xyz, mesh.gid, mesh.N, np.asarray(rho), level)
    keep = wall_distance(pts, wall) >= 2.0 * delta
    pts = pts[keep]
    if pts.shape[0] < mesh.dim + 2:
        raise ValueError("too few interface points for a fit")
    c, R = fit_circle(pts)
    return angle_from_fit(c, R, wall), c, R

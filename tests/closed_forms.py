"""Independent closed forms used to pin the oracle.

Nothing here calls the oracle or the GPU library.  Each helper is derived
from geometry rather than from the clip procedure the oracle uses:

* ``tent_value``: the column density of one tetrahedron under orthographic
  projection is a pyramid ("tent") over its projected silhouette.  It is
  zero on the silhouette boundary, linear on each triangle (apex, edge) and
  peaks at the apex, where the ray is longest; because the integral of
  rho*dl over the image plane is the tetrahedron's mass m, the peak value is
  3 m / A_sil (pyramid volume = area * height / 3).  The apex is the
  projected vertex that falls inside the other three (triangle silhouette)
  or the crossing of the two diagonals (quadrilateral silhouette).  No 3D
  volume and no ray clipping enter.
* ``cube_chord``: the length of a line inside an axis-aligned box (slab
  method), for the undisplaced lattice seen from a rotated direction.
* ``points_in_tets``: barycentric containment, for Monte-Carlo ray sums.
"""
from __future__ import annotations

import numpy as np

TET_TABLE = ((1, 0, 2, 4), (3, 1, 2, 4), (3, 5, 1, 4), (3, 6, 5, 4), (3, 2, 6, 4), (3, 7, 5, 6))


def cross2(a, b):
    return a[..., 0] * b[..., 1] - a[..., 1] * b[..., 0]


def _inside_triangle(p, a, b, c):
    d1, d2, d3 = cross2(b - a, p - a), cross2(c - b, p - b), cross2(a - c, p - c)
    neg = (d1 < 0) or (d2 < 0) or (d3 < 0)
    pos = (d1 > 0) or (d2 > 0) or (d3 > 0)
    return not (neg and pos)


def tent_geometry(P2):
    """Silhouette hull (counter-clockwise), apex and area of 4 projected points."""
    P2 = np.asarray(P2, dtype=np.float64)
    for a in range(4):
        o = [b for b in range(4) if b != a]
        if _inside_triangle(P2[a], P2[o[0]], P2[o[1]], P2[o[2]]):
            hull = P2[o]
            apex = P2[a].copy()
            break
    else:
        c = P2.mean(axis=0)
        ang = np.arctan2(P2[:, 1] - c[1], P2[:, 0] - c[0])
        hull = P2[np.argsort(ang)]
        # crossing of the diagonals hull[0]-hull[2] and hull[1]-hull[3]
        d1, d2 = hull[2] - hull[0], hull[3] - hull[1]
        s = cross2(hull[1] - hull[0], d2) / cross2(d1, d2)
        apex = hull[0] + s * d1
    area = 0.5 * sum(cross2(hull[i], hull[(i + 1) % len(hull)]) for i in range(len(hull)))
    if area < 0:
        hull = hull[::-1]
        area = -area
    return hull, apex, area


def tent_value(P2, mass, pts):
    """rho*dl of one tetrahedron at 2D points ``pts`` (N, 2), from its projection."""
    hull, apex, area = tent_geometry(P2)
    pts = np.asarray(pts, dtype=np.float64).reshape(-1, 2)
    peak = 3.0 * mass / area
    lam = np.full(pts.shape[0], np.inf)
    n = len(hull)
    for i in range(n):
        e0, e1 = hull[i], hull[(i + 1) % n]
        den = cross2(e1 - e0, apex - e0)
        lam = np.minimum(lam, cross2(e1 - e0, pts - e0) / den)
    return peak * np.maximum(lam, 0.0)


def cube_chord(origin, direction, lo=0.0, hi=1.0):
    """Length of {origin + t*direction} inside [lo, hi]^3 (direction unit)."""
    tmin, tmax = -np.inf, np.inf
    for a in range(3):
        if direction[a] == 0:
            if origin[a] < lo or origin[a] > hi:
                return 0.0
            continue
        t1 = (lo - origin[a]) / direction[a]
        t2 = (hi - origin[a]) / direction[a]
        tmin = max(tmin, min(t1, t2))
        tmax = min(tmax, max(t1, t2))
    return max(0.0, tmax - tmin)


def lattice_tets(x, y, z, n, box=1.0):
    """Unwrapped tetrahedra (6 n^3, 4, 3) of a periodic n^3 lattice, numpy only.

    Corner c = a + 2b + 4c of cube (i, j, k) is tracer ((i+a)%n, (j+b)%n,
    (k+c)%n); corners move to the periodic image nearest corner 0, an offset
    of exactly half the box going in the positive direction.
    """
    X = np.stack([x, y, z], axis=1).astype(np.float64).reshape(n, n, n, 3)  # [k, j, i]
    corners = []
    for c in range(8):
        a, b, cc = c & 1, (c >> 1) & 1, (c >> 2) & 1
        corners.append(np.roll(X, shift=(-cc, -b, -a), axis=(0, 1, 2)).reshape(-1, 3))
    base = corners[0]
    un = [base]
    for c in range(1, 8):
        e = corners[c] - base
        e -= box * np.ceil(e / box - 0.5)   # offset in (-L/2, L/2]
        un.append(base + e)
    un = np.stack(un, axis=1)  # (cubes, 8, 3), cube id = i + n(j + n k)
    tets = np.stack([un[:, list(t), :] for t in TET_TABLE], axis=1)  # (cubes, 6, 4, 3)
    return tets.reshape(-1, 4, 3)


def signed_volumes(tets):
    a = tets[:, 1] - tets[:, 0]
    b = tets[:, 2] - tets[:, 0]
    c = tets[:, 3] - tets[:, 0]
    return np.einsum("ij,ij->i", a, np.cross(b, c)) / 6.0


def points_in_tets(pts, tets):
    """Boolean (P, T): point p inside (closed) tetrahedron t, by barycentric signs."""
    v0 = tets[:, 0]
    M = np.stack([tets[:, 1] - v0, tets[:, 2] - v0, tets[:, 3] - v0], axis=2)  # (T,3,3)
    Minv = np.linalg.inv(M)
    d = pts[:, None, :] - v0[None, :, :]                   # (P,T,3)
    lam = np.einsum("tij,ptj->pti", Minv, d)
    l0 = 1.0 - lam.sum(axis=2)
    return (lam >= 0).all(axis=2) & (l0 >= 0)

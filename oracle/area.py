"""Area-average mode of the FP64 oracle (test infrastructure only).

Only the test suite may import this module; the GPU library never does, and
this module imports nothing from it.

The point-sampled oracle (``tess_oracle.c``) evaluates the column density of
the density-projections subsection (Eq. ``Eqn:TetProjection``: each
tetrahedron adds rho = m / |V| times the length of the view ray inside it) at
pixel centres.  This mode averages the same quantity over each pixel square
instead:

    I_area(ix, iy) = (1 / A_pix) * sum_T rho_T * integral over the pixel of dl_T(u, v) du dv.

It is exact, with no sampling: dl_T is the length of the ray at (u, v) inside
the convex tetrahedron, t_exit - t_entry, where t_exit is the least and
t_entry the greatest of the ray's crossings with the back and front face
planes (clamped at zero length).  Each crossing is an affine function of
(u, v), and two faces' crossings can only trade places along the projection
of the edge they share; the clamp acts on the silhouette, also made of
projected edges.  So dl_T is affine on every cell of the arrangement of the
six projected edge lines, and each cell's integral is its area times dl_T at
its centroid.  The cells inside one pixel come from splitting the pixel
square by the six lines (convex polygon clipping), and dl_T at a centroid is
the per-ray clip itself (the oracle's steps for a face plane: outward normal
n, offset h = n . y_b, crossing t = (h - n_u u - n_v v) / n_d).

Plain Python loops: for inputs of a few hundred tetrahedra and images of a
few thousand pixels.  Orthographic views only (rows of ``rot`` = screen u,
screen v, depth), with or without periodic image wrap.
"""
from __future__ import annotations

from typing import Dict, List, Sequence, Tuple

import numpy as np


def _view_frame(view: Dict):
    rot = np.asarray(view["rot"], dtype=np.float64).reshape(3, 3)
    center = np.asarray(view["center"], dtype=np.float64)
    W, H = int(view["width"]), int(view["height"])
    du = float(view["extent"][0]) / W
    dv = float(view["extent"][1]) / H
    u0 = -0.5 * float(view["extent"][0])
    v0 = -0.5 * float(view["extent"][1])
    return rot, center, W, H, du, dv, u0, v0


def face_planes(y: np.ndarray) -> List[Tuple[np.ndarray, float]]:
    """Outward face planes (n, h) of the tetrahedron with view-frame vertices
    y (4, 3): the face opposite vertex a has normal n = (y_c - y_b) x (y_d -
    y_b), turned so that n . (y_a - y_b) < 0, and offset h = n . y_b."""
    planes = []
    for a in range(4):
        b, c, d = [k for k in range(4) if k != a]
        n = np.cross(y[c] - y[b], y[d] - y[b])
        if np.dot(n, y[a] - y[b]) > 0:
            n = -n
        planes.append((n, float(np.dot(n, y[b]))))
    return planes


def ray_interval(planes, pu: float, pv: float) -> Tuple[float, float]:
    """The depths (t_entry, t_exit) where the ray (pu, pv, t) enters and leaves
    the tetrahedron; t_entry >= t_exit when it misses.  A face parallel to the
    ray excludes it when the ray lies outside (and, on the face plane, by the
    half-open rule: inside iff n_u < 0, or n_u = 0 and n_v < 0)."""
    lo, hi = -np.inf, np.inf
    for n, h in planes:
        s = h - n[0] * pu - n[1] * pv
        if n[2] > 0:
            hi = min(hi, s / n[2])
        elif n[2] < 0:
            lo = max(lo, s / n[2])
        elif s < 0 or (s == 0 and not (n[0] < 0 or (n[0] == 0 and n[1] < 0))):
            return 0.0, 0.0
    return lo, hi


def chord(planes, pu: float, pv: float) -> float:
    lo, hi = ray_interval(planes, pu, pv)
    return max(0.0, hi - lo) if np.isfinite(lo) and np.isfinite(hi) else 0.0


def _split(poly: List[Tuple[float, float]], a: float, b: float, c: float):
    """The parts of a convex polygon with a u + b v + c >= 0 and <= 0."""
    pos, neg = [], []
    m = len(poly)
    for i in range(m):
        p, q = poly[i], poly[(i + 1) % m]
        fp = a * p[0] + b * p[1] + c
        fq = a * q[0] + b * q[1] + c
        if fp >= 0:
            pos.append(p)
        if fp <= 0:
            neg.append(p)
        if (fp > 0 and fq < 0) or (fp < 0 and fq > 0):
            t = fp / (fp - fq)
            x = (p[0] + t * (q[0] - p[0]), p[1] + t * (q[1] - p[1]))
            pos.append(x)
            neg.append(x)
    return pos, neg


def _area_centroid(poly):
    """Signed area and centroid of a simple polygon (shoelace)."""
    A = cx = cy = 0.0
    m = len(poly)
    for i in range(m):
        x0, y0 = poly[i]
        x1, y1 = poly[(i + 1) % m]
        cr = x0 * y1 - x1 * y0
        A += cr
        cx += (x0 + x1) * cr
        cy += (y0 + y1) * cr
    A *= 0.5
    if A == 0.0:
        return 0.0, 0.0, 0.0
    return A, cx / (6.0 * A), cy / (6.0 * A)


def _cells(square, lines):
    cells = [square]
    for (a, b, c) in lines:
        nxt = []
        for poly in cells:
            p, n = _split(poly, a, b, c)
            for part in (p, n):
                if len(part) >= 3:
                    nxt.append(part)
        cells = nxt
    return cells


def pixel_integrals(y: np.ndarray, du: float, dv: float, u0: float, v0: float):
    """For a tetrahedron with view-frame vertices y (4, 3): the integral of
    dl over each pixel square its projection meets, as {(ix, iy): value}
    with unwrapped pixel indices (pixel (ix, iy) covers [u0 + ix du, u0 +
    (ix + 1) du] x [v0 + iy dv, ...])."""
    planes = face_planes(y)
    pu, pv = y[:, 0], y[:, 1]
    lines = []
    for i in range(4):
        for j in range(i + 1, 4):
            a = pv[j] - pv[i]
            b = pu[i] - pu[j]
            if a == 0.0 and b == 0.0:
                continue
            lines.append((a, b, -(a * pu[i] + b * pv[i])))
    ix0 = int(np.floor((pu.min() - u0) / du))
    ix1 = int(np.floor((pu.max() - u0) / du))
    iy0 = int(np.floor((pv.min() - v0) / dv))
    iy1 = int(np.floor((pv.max() - v0) / dv))
    out = {}
    for iy in range(iy0, iy1 + 1):
        ya, yb = v0 + iy * dv, v0 + (iy + 1) * dv
        for ix in range(ix0, ix1 + 1):
            xa, xb = u0 + ix * du, u0 + (ix + 1) * du
            total = 0.0
            for cell in _cells([(xa, ya), (xb, ya), (xb, yb), (xa, yb)], lines):
                A, cx, cy = _area_centroid(cell)
                if A > 0.0:
                    total += A * chord(planes, cx, cy)
            if total != 0.0:
                out[(ix, iy)] = total
    return out


def project_tets_area(verts, mass, view: Dict) -> np.ndarray:
    """Area-average image (H, W) of an explicit tetrahedron list, verts
    (T, 4, 3) world coordinates, mass (T,) or a scalar; each tetrahedron
    carries rho = m / |V| (Eqs. Eqn:TetVolume and Eqn-rho_loc).  With
    view["wrap"] the window is periodic, otherwise pixels outside it are
    dropped."""
    rot, center, W, H, du, dv, u0, v0 = _view_frame(view)
    wrap = bool(view.get("wrap", 0))
    verts = np.asarray(verts, dtype=np.float64).reshape(-1, 4, 3)
    mass = np.broadcast_to(np.asarray(mass, dtype=np.float64), (verts.shape[0],))
    img = np.zeros((H, W), dtype=np.float64)
    for T in range(verts.shape[0]):
        x = verts[T]
        vol = np.dot(x[1] - x[0], np.cross(x[2] - x[0], x[3] - x[0])) / 6.0
        if vol == 0.0:
            continue
        rho = mass[T] / abs(vol)
        y = (x - center) @ rot.T
        for (ix, iy), val in pixel_integrals(y, du, dv, u0, v0).items():
            if wrap:
                ix, iy = ix % W, iy % H
            elif not (0 <= ix < W and 0 <= iy < H):
                continue
            img[iy, ix] += rho * val / (du * dv)
    return img


def lattice_tets(x, y, z, dims: Sequence[int], box=(1.0, 1.0, 1.0), periodic: bool = True):
    """All tetrahedra of a lattice as (T, 4, 3) unwrapped vertices, from the
    oracle's own cube gather (every cube's six tetrahedra)."""
    from oracle import cube_tets
    nc = int(np.prod([d if periodic else d - 1 for d in dims]))
    out = []
    for cube in range(nc):
        v, _ = cube_tets(x, y, z, dims, cube, box=box, periodic=periodic)
        out.append(v)
    return np.concatenate(out, axis=0)


def dirichlet_deposits(verts, mass, view: Dict, per_tet: int, seed: int = 0) -> np.ndarray:
    """Monte Carlo counterpart of the area mode: per_tet points drawn
    uniformly in each tetrahedron (barycentric weights Dirichlet(1, 1, 1, 1)),
    each depositing m / per_tet into the pixel its projection falls in;
    returned as a column density (deposits / pixel area)."""
    rot, center, W, H, du, dv, u0, v0 = _view_frame(view)
    wrap = bool(view.get("wrap", 0))
    verts = np.asarray(verts, dtype=np.float64).reshape(-1, 4, 3)
    mass = np.broadcast_to(np.asarray(mass, dtype=np.float64), (verts.shape[0],))
    rng = np.random.default_rng(seed)
    img = np.zeros((H, W), dtype=np.float64)
    for T in range(verts.shape[0]):
        w = rng.dirichlet(np.ones(4), size=per_tet)
        p = (w @ verts[T] - center) @ rot.T
        ix = np.floor((p[:, 0] - u0) / du).astype(np.int64)
        iy = np.floor((p[:, 1] - v0) / dv).astype(np.int64)
        if wrap:
            ix, iy = ix % W, iy % H
        else:
            keep = (ix >= 0) & (ix < W) & (iy >= 0) & (iy < H)
            ix, iy = ix[keep], iy[keep]
        np.add.at(img, (iy, ix), mass[T] / per_tet)
    return img / (du * dv)

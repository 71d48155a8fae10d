"""Pins of the FP64 oracle against things other than itself.

Each test checks the oracle against a closed form, an invariant or brute
force derived independently (``closed_forms.py``), chosen so that a plausible
slip in the oracle (a corner numbering, a table entry, a sign, a dropped face,
the unwrap, the pixel-centre convention, the wrap logic) fails one of them.
"""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W
from closed_forms import (TET_TABLE, cube_chord, lattice_tets, points_in_tets,
                          signed_volumes, tent_value)


def corner_xyz(n):
    return np.array([[(c & 1), (c >> 1) & 1, (c >> 2) & 1] for c in range(8)], dtype=np.float64)


# ---------------------------------------------------------------- C1: table
def test_c1_undisplaced_volumes_equal_and_negative():
    # Table {1,0,2,4} ... {3,7,5,6} with corners n = a + 2b + 4c: six tets of
    # equal volume Delta^3/6, all with the same (negative) orientation.
    n = 4  # spacing exact in FP32
    x, y, z = W.undisplaced(n)
    for cube in (0, 21, 63):
        _, vols = O.cube_tets(x, y, z, (n, n, n), cube)
        np.testing.assert_allclose(vols, -(1.0 / n) ** 3 / 6.0, rtol=1e-12, atol=0)


def test_c1_tets_tile_the_cube_without_overlap():
    n = 2
    x, y, z = W.undisplaced(n)
    verts, vols = O.cube_tets(x, y, z, (n, n, n), 0)
    rng = np.random.default_rng(5)
    pts = rng.uniform(0.0, 0.5, size=(20000, 3))
    inside = points_in_tets(pts, verts)
    assert np.all(inside.sum(axis=1) == 1)
    assert abs(np.abs(vols).sum() - 0.5 ** 3) < 1e-15


def test_c1_face_diagonals_match_neighbours():
    # Boundary triangles on opposite cube faces coincide after translation,
    # so neighbouring cubes share their face diagonals (no cracks).
    C = corner_xyz(1)
    for axis in range(3):
        sets = {0: set(), 1: set()}
        for t in TET_TABLE:
            for drop in range(4):
                face = [t[m] for m in range(4) if m != drop]
                coord = C[face, axis]
                if np.all(coord == coord[0]):
                    key = tuple(sorted(tuple(np.delete(C[f], axis)) for f in face))
                    sets[int(coord[0])].add(key)
        assert len(sets[0]) == 2 and sets[0] == sets[1]


def _hull_area(pts):
    """Area of the convex hull of 2D points (monotone chain)."""
    P = sorted(set(map(tuple, np.asarray(pts, dtype=np.float64))))
    if len(P) < 3:
        return 0.0

    def half(seq):
        h = []
        for p in seq:
            while len(h) >= 2 and ((h[-1][0] - h[-2][0]) * (p[1] - h[-2][1])
                                   - (h[-1][1] - h[-2][1]) * (p[0] - h[-2][0])) <= 0:
                h.pop()
            h.append(p)
        return h
    hull = half(P)[:-1] + half(P[::-1])[:-1]
    return 0.5 * abs(sum(hull[i][0] * hull[(i + 1) % len(hull)][1]
                         - hull[(i + 1) % len(hull)][0] * hull[i][1] for i in range(len(hull))))


def test_c1_z_projected_areas():
    # z-projected silhouettes of the six undisplaced tets: 1/2, 1, 1/2, 1, 1/2,
    # 1/2 of the unit square, 4 in total (each column crosses the cube in 4 tets'
    # worth of silhouette, a fact the undisplaced constant-density pin relies on).
    C = corner_xyz(1)
    areas = [_hull_area(C[list(t), :2]) for t in TET_TABLE]
    assert areas == [0.5, 1.0, 0.5, 1.0, 0.5, 0.5]


# ------------------------------------------------- C2: single-tet closed form
def _random_tets(rng, count, scale=0.3):
    out = []
    while len(out) < count:
        v = rng.uniform(0.2, 0.8, size=(4, 3))
        v = v.mean(axis=0) + (v - v.mean(axis=0)) * scale / 0.3
        if abs(signed_volumes(v[None])[0]) > 1e-4:
            out.append(v)
    return np.array(out)


def test_c2_single_tet_matches_tent_closed_form_z_view():
    rng = np.random.default_rng(11)
    view = W.rotated_view(np.eye(3), 48, 40, side=1.0, center=(0.5, 0.5, 0.5))
    for v in _random_tets(rng, 25):
        img, st = O.project_tets(v[None], [0.7], view)
        jj, ii = np.mgrid[0:40, 0:48]
        pu = -0.5 + (ii + 0.5) / 48.0
        pv = -0.5 + (jj + 0.5) / 40.0
        ref = tent_value(v[:, :2] - 0.5, 0.7, np.stack([pu.ravel(), pv.ravel()], 1)).reshape(40, 48)
        np.testing.assert_allclose(img, ref, rtol=0, atol=1e-10 * ref.max())
        assert st["tets"] == 1 and st["fragments"] == int((ref > 0).sum())


def test_c2_single_tet_matches_tent_rotated_views():
    rng = np.random.default_rng(12)
    Rs = W.random_rotations(10, seed=77)
    for v, R in zip(_random_tets(rng, 10), Rs):
        view = W.rotated_view(R, 40, 36, side=1.6)
        img, _ = O.project_tets(v[None], [1.3], view)
        y = (v - 0.5) @ R.T
        jj, ii = np.mgrid[0:36, 0:40]
        pu = -0.8 + (ii + 0.5) * 1.6 / 40
        pv = -0.8 + (jj + 0.5) * 1.6 / 36
        ref = tent_value(y[:, :2], 1.3, np.stack([pu.ravel(), pv.ravel()], 1)).reshape(36, 40)
        np.testing.assert_allclose(img, ref, rtol=0, atol=1e-10 * ref.max())


@pytest.mark.parametrize("n", [2, 3, 8, 100])
def test_c2_corner_tet_pixel_sum(n):
    # Corner tet with legs of n pixels: sum of I * A_pix = m (1 - 1/n^2) exactly.
    v = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=np.float64)
    view = W.rotated_view(np.eye(3), n, n, side=1.0, center=(0.5, 0.5, 0.5))
    m = 0.25
    img, _ = O.project_tets(v[None], [m], view)
    total = img.sum() / (n * n)
    assert math.isclose(total, m * (1 - 1.0 / n ** 2), rel_tol=1e-13)


# ------------------------------------------------ C3: undisplaced lattice
@pytest.mark.parametrize("n,w,h", [(2, 2, 4), (4, 16, 16), (4, 12, 20), (8, 24, 16)])
def test_c3_undisplaced_column_density_is_one(n, w, h):
    x, y, z = W.undisplaced(n)
    img, st = O.project_region(x, y, z, (n, n, n), W.z_view(w, h))
    np.testing.assert_allclose(img, 1.0, rtol=0, atol=1e-13)
    assert st["tets"] == 6 * n ** 3 and st["inverted"] == 0


def test_c3_tie_rule_rays_on_vertical_faces():
    # Pixel centres on the lattice planes x = j/n (but not on any edge): the
    # half-open rule must let exactly one of the two face-sharing tets count.
    n = 4
    x, y, z = W.undisplaced(n)
    img, _ = O.project_region(x, y, z, (n, n, n), W.z_view(2, 10))
    np.testing.assert_allclose(img, 1.0, rtol=0, atol=1e-13)


def test_c3_rotated_view_equals_cube_chord():
    d = 5  # non-periodic lattice of vertices at i/4 covering [0, 1]^3
    r = np.arange(d) / (d - 1)
    qz, qy, qx = np.meshgrid(r, r, r, indexing="ij")
    x, y, z = (a.ravel().astype(np.float32) for a in (qx, qy, qz))
    R = W.random_rotations(3, seed=9)
    for rot in R:
        view = W.rotated_view(rot, 24, 20, side=2.0)
        img, st = O.project_region(x, y, z, (d, d, d), view, periodic=False)
        ref = np.zeros_like(img)
        for j in range(20):
            for i in range(24):
                pu = -1 + (i + 0.5) * 2 / 24
                pv = -1 + (j + 0.5) * 2 / 20
                origin = np.array([0.5, 0.5, 0.5]) + pu * rot[0] + pv * rot[1]
                ref[j, i] = cube_chord(origin, rot[2])
        np.testing.assert_allclose(img, ref, rtol=0, atol=1e-12)
        assert st["tets"] == 6 * (d - 1) ** 3


# --------------------------------------- C4: line-of-sight-only displacement
def test_c4_z_only_displacement_keeps_column_density():
    n = 8
    q = W.lattice_q(n)
    f = 0.25 * np.sin(2 * np.pi * q[:, 2]) * (1 + 0.5 * np.cos(2 * np.pi * q[:, 0])) \
        + 0.1 * np.sin(2 * np.pi * (2 * q[:, 1] + q[:, 2]))
    x = q[:, 0].astype(np.float32)
    y = q[:, 1].astype(np.float32)
    z = W.wrap_to_f32(q[:, 2] + f, 1.0)
    img, st = O.project_region(x, y, z, (n, n, n), W.z_view(32, 24))
    assert st["inverted"] > 0          # shell crossing happened
    np.testing.assert_allclose(img, 1.0, rtol=0, atol=1e-11)


# ------------------ Q: projected quantity q = rho^p (p = 0 path length, 2 rho^2)
@pytest.mark.parametrize("quantity,power", [("unit", 0), ("density", 1), ("density2", 2)])
def test_q_undisplaced_lattice_projects_mass_power(quantity, power):
    # rho = M everywhere and every ray crosses a column of length 1
    n, M = 4, 3.0
    xyz = W.undisplaced(n)
    view = dict(W.z_view(16, 12), quantity=quantity)
    img, _ = O.project_region(*xyz, (n, n, n), view, total_mass=M)
    np.testing.assert_allclose(img, M ** power, rtol=1e-13, atol=0)


@pytest.mark.parametrize("quantity", ["unit", "density2"])
def test_q_z_only_layers_closed_forms(quantity):
    # z = q_z + A sin(2 pi q_z) with A > 1/(2 pi): flat layers k of signed
    # thickness dz_k, some inverted (shell crossing). Every ray crosses each
    # layer once: sum dl = sum |dz_k|, and with rho_k = M / (n |dz_k|),
    # sum rho^2 dl = M^2 / n^2 * sum 1 / |dz_k|.
    n, M, A = 8, 2.0, 0.3
    q = W.lattice_q(n)
    x = q[:, 0].astype(np.float32)
    y = q[:, 1].astype(np.float32)
    z = W.wrap_to_f32(q[:, 2] + A * np.sin(2 * np.pi * q[:, 2]), 1.0)
    zk = z.reshape(n, n, n)[:, 0, 0].astype(np.float64)        # layer k at column (0, 0)
    dz = np.roll(zk, -1) - zk
    dz -= np.ceil(dz - 0.5)                                      # nearest periodic image
    assert (dz < 0).any()
    view = dict(W.z_view(16, 12), quantity=quantity)
    img, st = O.project_region(x, y, z, (n, n, n), view, total_mass=M)
    assert st["inverted"] > 0
    want = np.abs(dz).sum() if quantity == "unit" else M ** 2 / n ** 2 * (1.0 / np.abs(dz)).sum()
    np.testing.assert_allclose(img, want, rtol=1e-12, atol=0)


# ---------------------------------- S: depth slab (clamped front/back fragments)
@pytest.mark.parametrize("slab", [(-0.5, 0.5), (-0.25, 0.1), (0.2, 0.45), (0.49, 0.7)])
def test_s_undisplaced_lattice_slab_is_its_thickness(slab):
    # z-view: depth t = z - 1/2 and the lattice fills t in [-1/2, 1/2]; every
    # ray's chord inside the slab is its overlap with that range, at rho = M
    n, M = 4, 3.0
    view = dict(W.z_view(16, 12), slab=slab)
    img, _ = O.project_region(*W.undisplaced(n), (n, n, n), view, total_mass=M)
    want = M * max(0.0, min(slab[1], 0.5) - max(slab[0], -0.5))
    np.testing.assert_allclose(img, want, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("slab", [(-0.3, 0.2), (0.0, 0.05), (-0.6, -0.2)])
def test_s_z_only_layers_slab_closed_form(slab):
    # flat layers k from z_k to z_k + dz_k (unwrapped from the cube's corner 0,
    # dz_k < 0 for inverted ones) at rho_k = M / (n |dz_k|): the slab keeps
    # the part of each layer with z - 1/2 in [s0, s1]
    n, M, A = 8, 2.0, 0.3
    q = W.lattice_q(n)
    x = q[:, 0].astype(np.float32)
    y = q[:, 1].astype(np.float32)
    z = W.wrap_to_f32(q[:, 2] + A * np.sin(2 * np.pi * q[:, 2]), 1.0)
    zk = z.reshape(n, n, n)[:, 0, 0].astype(np.float64)
    dz = np.roll(zk, -1) - zk
    dz -= np.ceil(dz - 0.5)
    lo, hi = np.minimum(zk, zk + dz) - 0.5, np.maximum(zk, zk + dz) - 0.5
    overlap = np.clip(np.minimum(hi, slab[1]) - np.maximum(lo, slab[0]), 0.0, None)
    want = (M / (n * np.abs(dz)) * overlap).sum()
    view = dict(W.z_view(16, 12), slab=slab)
    img, _ = O.project_region(x, y, z, (n, n, n), view, total_mass=M)
    np.testing.assert_allclose(img, want, rtol=1e-12, atol=1e-14)


def test_s_slabs_partition_the_projection():
    # slabs that tile the depth axis add up to the unclipped projection, and
    # one slab around everything is the unclipped projection
    n = 8
    xyz = W.zeldovich(n, 3, 4.0, seed=9)
    R = W.random_rotations(1, seed=17)[0]
    view = W.rotated_view(R, 48, 40)
    full, st = O.project_region(*xyz, (n, n, n), view)
    cuts = np.linspace(-1.5, 1.5, 7)
    parts = [O.project_region(*xyz, (n, n, n), dict(view, slab=(a, b)))[0] for a, b in zip(cuts[:-1], cuts[1:])]
    np.testing.assert_allclose(sum(parts), full, rtol=0, atol=1e-12 * np.abs(full).max())
    assert all((p >= 0).all() for p in parts) and sum(p.sum() > 0 for p in parts) >= 3
    whole, _ = O.project_region(*xyz, (n, n, n), dict(view, slab=(-10.0, 10.0)))
    np.testing.assert_array_equal(whole, full)


# ------------------------------------------ K: centroid splatting (approximate)
def _splat_tet(scale=1.0, at=(0.5, 0.5)):
    # a tetrahedron with |V| = scale^3 * 1e-3 / 6 * 6 = scale^3 * 1e-3 whose
    # centroid projects onto (at) in a z-view of the unit box
    e = 0.1 * scale * np.cbrt(6.0)
    v = np.array([[0, 0, 0], [e, 0, 0], [0, e, 0], [0, 0, e]], dtype=np.float64)
    v += np.array([at[0], at[1], 0.5]) - v.mean(axis=0)
    return v


def test_k_splat_carries_the_mass_within_two_h():
    # h = |V|^(1/3) = 0.1 = 51.2 px at 512^2: the kernel's pixel sum is its
    # integral (1) to well below 1e-6, so the image holds the mass m
    view = W.z_view(512)
    m = 0.37
    v = _splat_tet(at=(0.5 + 0.3 / 512, 0.5 - 0.2 / 512))
    img, st = O.splat_tets(v[None], m, view)
    np.testing.assert_allclose(img.sum() / 512 ** 2, m, rtol=1e-6)
    yy, xx = np.nonzero(img)
    c = v.mean(axis=0)
    r = np.hypot((xx + 0.5) / 512 - c[0], (yy + 0.5) / 512 - c[1])
    assert r.max() < 0.2 and r.max() > 0.19 and st["fragments"] == len(xx)


def test_k_splat_size_is_the_cube_root_of_the_volume():
    # scaling the tetrahedron by s keeps the mass and divides the peak by s^2
    view = W.z_view(256)
    peaks = [O.splat_tets(_splat_tet(scale=s, at=(0.5 + 0.5 / 256, 0.5 + 0.5 / 256))[None], 1.0, view)[0].max()
             for s in (1.0, 2.0)]
    np.testing.assert_allclose(peaks[0] / peaks[1], 4.0, rtol=1e-12)


def test_k_undisplaced_lattice_splats_around_the_column_density():
    # periodic image: the mass is kept up to the point sampling of kernels
    # with h = 4.4 px (a Riemann sum, ~1e-5); a uniform lattice of splats
    # (h = |V|^(1/3), 0.55 of the lattice spacing) ripples around the
    # uniform column density M by about 16 %
    n, M = 8, 2.0
    img, st = O.splat_image(*W.undisplaced(n), (n, n, n), W.z_view(64), total_mass=M)
    np.testing.assert_allclose(img.mean(), M, rtol=1e-4)
    assert np.abs(img / M - 1).max() < 0.2 and st["tets"] == 6 * n ** 3


# ------------------------------------------------------------ P: perspective
def box_chords(view):
    """Length of every pixel's camera half-line inside the unit box, by the
    slab method (independent of the tetrahedra)."""
    R = np.asarray(view["rot"], dtype=np.float64).reshape(3, 3)
    c = np.asarray(view["center"], dtype=np.float64)
    W_, H_ = view["width"], view["height"]
    pu = -0.5 * view["extent"][0] + (np.arange(W_) + 0.5) * (view["extent"][0] / W_)
    pv = -0.5 * view["extent"][1] + (np.arange(H_) + 0.5) * (view["extent"][1] / H_)
    U, V = np.meshgrid(pu, pv)
    d = np.stack([U, V, np.ones_like(U)], -1) @ R          # world directions, rows of R^T
    with np.errstate(divide="ignore", invalid="ignore"):
        t0 = (0.0 - c) / d
        t1 = (1.0 - c) / d
    lo = np.where(d != 0, np.minimum(t0, t1), np.where((c >= 0) & (c <= 1), -np.inf, np.inf))
    hi = np.where(d != 0, np.maximum(t0, t1), np.where((c >= 0) & (c <= 1), np.inf, -np.inf))
    s_in = np.maximum(lo.max(-1), 0.0)
    s_out = hi.min(-1)
    return np.maximum(s_out - s_in, 0.0) * np.linalg.norm(d, axis=-1)


@pytest.mark.parametrize("camera,rot_seed", [((0.4, 0.55, -1.3), None), ((0.3, 0.62, 0.45), 3),
                                              ((1.9, -0.7, 1.6), 5)])
def test_p_undisplaced_lattice_is_the_box_chord(camera, rot_seed):
    # periodic unit lattice, M = 1: density 1 exactly filling [0, 1]^3, so every
    # pixel holds the length of its camera half-line inside the box; the
    # camera outside, inside (half-line cut at the camera), and oblique
    n = 8
    R = np.eye(3) if rot_seed is None else W.random_rotations(1, seed=rot_seed)[0]
    if camera[0] > 1.0:  # look back at the box centre
        f = np.array([0.5, 0.5, 0.5]) - np.array(camera)
        f /= np.linalg.norm(f)
        u = np.cross([0.0, 0.0, 1.0], f)
        u /= np.linalg.norm(u)
        R = np.stack([u, np.cross(f, u), f])
    view = W.perspective_view(R, camera, 40, 32, extent=(1.6, 1.3))
    img, st = O.project_region(*W.undisplaced(n), (n,) * 3, view)
    ref = box_chords(view)
    assert ref.max() > 0.5
    np.testing.assert_allclose(img, ref, rtol=1e-12, atol=1e-13)


def test_p_far_camera_is_the_orthographic_projection():
    # a camera 1e6 box lengths away with a window of the box's size there sees
    # nearly parallel rays: the orthographic image to ~W / (2 D) of a pixel
    n = 12
    xyz = W.zeldovich(n, 3, 1.5)
    D = 1e6
    ortho = W.z_view(32)
    ortho["wrap"] = 0
    persp = W.perspective_view(np.eye(3), (0.5, 0.5, 0.5 - D), 32, extent=(1.0 / D, 1.0 / D))
    a, _ = O.project_region(*xyz, (n,) * 3, ortho)
    b, _ = O.project_region(*xyz, (n,) * 3, persp)
    cov = a > 1e-3 * a.mean()
    assert cov.mean() > 0.5
    np.testing.assert_allclose(b[cov], a[cov], rtol=1e-4)
    assert abs(b.sum() / a.sum() - 1.0) < 1e-5


def test_h_hybrid_limits_are_the_exact_and_the_billboard_images():
    # the near/far hybrid: a sphere larger than the scene draws every
    # tetrahedron exactly, radius 0 draws every one as a billboard
    n = 8
    xyz = W.zeldovich(n, 3, 2.0)
    base = W.perspective_view(np.eye(3), (0.45, 0.52, -1.2), 40, 32, extent=(1.2, 1.0))
    exact, _ = O.project_region(*xyz, (n,) * 3, base)
    bills, sb = O.project_region(*xyz, (n,) * 3, dict(base, method="centroids"))
    far, _ = O.project_region(*xyz, (n,) * 3, dict(base, method="hybrid", lod_radius=1e9))
    near, _ = O.project_region(*xyz, (n,) * 3, dict(base, method="hybrid", lod_radius=0.0))
    np.testing.assert_array_equal(far, exact)
    np.testing.assert_array_equal(near, bills)
    mid, _ = O.project_region(*xyz, (n,) * 3, dict(base, method="hybrid", lod_radius=1.9))
    assert not np.array_equal(mid, exact) and not np.array_equal(mid, bills)
    assert sb["fragments"] > 0


def test_h_billboard_carries_q_v_over_z_squared():
    # the window integral of one billboard's kernel is 1 / z_c^2 (the plane at
    # depth z_c maps to the window scaled by 1 / z_c), so a far billboard sums
    # to q |V| / z_c^2 times the pixel area
    v = np.array([[0.0, 0.0, 0.0], [0.3, 0.0, 0.0], [0.0, 0.3, 0.0], [0.0, 0.0, 0.3]]) + [0.1, -0.05, 4.0]
    vol = abs(np.linalg.det(v[1:] - v[0])) / 6.0
    zc = v[:, 2].mean()
    view = dict(W.perspective_view(np.eye(3), (0.0, 0.0, 0.0), 160, 160, extent=(0.5, 0.5)), method="centroids")
    img, st = O.project_tets(v[None], 0.7, view)
    du = dv = 0.5 / 160
    total = img.sum() * du * dv
    assert abs(total * zc ** 2 / 0.7 - 1.0) < 2e-3      # q |V| = rho |V| = m
    # and the hybrid takes it exactly inside its sphere
    img2, _ = O.project_tets(v[None], 0.7, dict(view, method="hybrid", lod_radius=5.0))
    ex, _ = O.project_tets(v[None], 0.7, dict(view, method="tessellation"))
    np.testing.assert_array_equal(img2, ex)
    assert vol > 0


def test_h_far_camera_billboards_are_the_orthographic_splats():
    n = 10
    xyz = W.zeldovich(n, 3, 1.5)
    D = 1e6
    ortho = dict(W.z_view(32), wrap=0, method="centroids")
    persp = W.perspective_view(np.eye(3), (0.5, 0.5, 0.5 - D), 32, extent=(1.0 / D, 1.0 / D))
    a, _ = O.splat_image(*xyz, (n,) * 3, ortho)
    b, _ = O.project_region(*xyz, (n,) * 3, dict(persp, method="centroids"))
    cov = a > 1e-3 * a.mean()
    np.testing.assert_allclose(b[cov], a[cov], rtol=1e-4)


def test_p_perspective_needs_no_wrap_and_no_slab():
    n = 4
    xyz = W.undisplaced(n)
    for extra in ({"wrap": 1}, {"slab": (0.1, 0.3)}):
        view = W.perspective_view(np.eye(3), (0.5, 0.5, -1.0), 8)
        view.update(extra)
        with pytest.raises(Exception):
            O.project_region(*xyz, (n,) * 3, view)


def test_c4_near_degenerate_tets():
    # z = q_z - A sin(2 pi q_z + phi): the first cell layer has thickness
    # 1/n - 2 A sin(pi/n) = delta/n for A = (1 - delta)/(2 n sin(pi/n)),
    # phi = -pi/n, so its tets are almost flat; the column density stays 1.
    n, delta = 16, 1e-4
    q = W.lattice_q(n)
    A = (1 - delta) / (2 * n * np.sin(np.pi / n))
    f = A * np.sin(2 * np.pi * q[:, 2] - np.pi / n)
    z = W.wrap_to_f32(q[:, 2] - f, 1.0)
    x = q[:, 0].astype(np.float32)
    y = q[:, 1].astype(np.float32)
    tets = lattice_tets(x, y, z, n)
    V = np.abs(signed_volumes(tets))
    assert V.min() < 1e-3 * V.mean()
    img, st = O.project_region(x, y, z, (n, n, n), W.z_view(48, 32))
    assert st["zero_volume"] == 0
    np.testing.assert_allclose(img, 1.0, rtol=0, atol=1e-9)


# ----------------------------------------------------------- C5: mass
def test_c5_point_sampled_mass_converges():
    x, y, z = W.random_lattice(4, 0.08, seed=3)
    errs = []
    for w in (16, 64, 256):
        img, _ = O.project_region(x, y, z, (4, 4, 4), W.z_view(w))
        errs.append(abs(img.mean() - 1.0))
    assert errs[2] < errs[0] and errs[2] < 2e-3


# ------------------------------------------- area-average mode (C2, C5, C6)
def _random_tet(rng, lo=0.2, hi=0.8):
    while True:
        v = rng.uniform(lo, hi, size=(4, 3))
        if abs(np.linalg.det(v[1:] - v[0])) > 1e-3:
            return v


def test_c2_area_mode_single_tet_carries_its_mass_exactly():
    # the integral of dl over the projection is the volume, so a tetrahedron
    # inside the window deposits exactly m (any view, any shape)
    from oracle import area as A
    rng = np.random.default_rng(11)
    for k in range(6):
        v = _random_tet(rng)
        m = rng.uniform(0.5, 2.0)
        if k % 2:
            view = W.rotated_view(W.random_rotations(1, seed=30 + k)[0], 19, 23, side=1.6)
        else:
            view = W.z_view(24, 20)
        img = A.project_tets_area(v[None], m, view)
        apix = view["extent"][0] * view["extent"][1] / (view["width"] * view["height"])
        assert abs(img.sum() * apix - m) <= 1e-12 * m, k


def test_c2_area_mode_pixel_is_the_mean_of_the_tent():
    # an area-mode pixel against a fine midpoint average of the independent
    # tent closed form of rho * dl over the pixel square
    from oracle import area as A
    rng = np.random.default_rng(12)
    v = _random_tet(rng)
    m = 1.0
    w = 8
    img = A.project_tets_area(v[None], m, W.z_view(w))
    s = 240
    for (j, i) in zip(*np.nonzero(img > 0.05 * img.max())):
        g = (np.arange(s) + 0.5) / s
        uu, vv = np.meshgrid((i + g) / w, (j + g) / w)
        mean = tent_value(v[:, :2], m, np.stack([uu.ravel(), vv.ravel()], 1)).mean()
        assert abs(mean - img[j, i]) <= 4e-3 * img.max(), (i, j, mean, img[j, i])


def test_c5_area_mode_mass_is_exact():
    # a displaced periodic lattice under the wrapped z-view: the area mode
    # carries the total mass exactly (point sampling only converges to it)
    from oracle import area as A
    n = 3
    x, y, z = W.random_lattice(n, 0.1, seed=5)
    tets = A.lattice_tets(x, y, z, (n, n, n))
    assert tets.shape == (6 * n ** 3, 4, 3)
    mass = 1.0 / len(tets)
    for w, h in ((9, 9), (13, 7)):
        img = A.project_tets_area(tets, mass, W.z_view(w, h))
        assert abs(img.mean() - 1.0) <= 1e-12, (w, h, img.mean())
        pt, _ = O.project_region(x, y, z, (n, n, n), W.z_view(w, h))
        assert abs(pt.mean() - 1.0) > 1e-9  # the point mode is not exact at this resolution


def test_c6_area_mode_against_dirichlet_deposits():
    # K points uniform in each tetrahedron (Dirichlet(1,1,1,1) weights), each
    # depositing m/K in the pixel its projection falls in: every pixel within
    # 5 sigma of the area mode, and the normalised squared deviations average
    # about 1
    from oracle import area as A
    n = 2
    x, y, z = W.random_lattice(n, 0.12, seed=7)
    tets = A.lattice_tets(x, y, z, (n, n, n))
    mass = 1.0 / len(tets)
    view = W.z_view(7, 6)
    ref = A.project_tets_area(tets, mass, view)
    K = 20000
    mc = A.dirichlet_deposits(tets, mass, view, K, seed=3)
    apix = 1.0 / (7 * 6)
    # variance per pixel: sum over tets of (m/K)^2 K p (1 - p) / apix^2
    var = np.zeros_like(ref)
    rot, center = np.eye(3), np.array([0.5, 0.5, 0.5])
    for tv in tets:
        one = A.project_tets_area(tv[None], mass, view)
        p = one * apix / mass
        var += (mass / K) ** 2 * K * p * (1.0 - p) / apix ** 2
    zs = (mc - ref) / np.sqrt(np.maximum(var, 1e-300))
    assert np.abs(zs).max() < 5.0, np.abs(zs).max()
    assert 0.4 < float((zs ** 2).mean()) < 2.0
    assert abs(mc.mean() - 1.0) < 1e-12


# ------------------------------------- C8: the entry/exit form of the sum
def test_c8_entry_exit_form_and_its_fp32_cancellation():
    # Eq. Eqn:TetSum writes a pixel as sum rho (t_exit - t_ref) - sum rho
    # (t_entry - t_ref) over the tetrahedra the ray meets: in FP64 it is the
    # projection (against the oracle's point mode); with the depths measured
    # from a reference far in front (a camera 10^4 box lengths away) and the
    # terms summed in FP32, the two sums cancel and the error reaches
    # eps * (distance / chord) * sqrt(terms), far above the 1e-4 bar
    from oracle import area as A
    n = 3
    x, y, z = W.random_lattice(n, 0.1, seed=6)
    tets = A.lattice_tets(x, y, z, (n, n, n))
    mass = 1.0 / len(tets)
    w = 9
    img, _ = O.project_region(x, y, z, (n, n, n), W.z_view(w))
    t_ref = -1.0e4
    planes, rhos = [], []
    for tv in tets:
        for sx in (-1, 0, 1):
            for sy in (-1, 0, 1):
                yv = tv + np.array([sx, sy, 0.0]) - 0.5
                vol = np.dot(yv[1] - yv[0], np.cross(yv[2] - yv[0], yv[3] - yv[0])) / 6.0
                planes.append(A.face_planes(yv))
                rhos.append(mass / abs(vol))
    worst64, worst32, pred = 0.0, 0.0, 0.0
    for (j, i) in [(0, 0), (4, 4), (7, 2), (3, 8)]:
        pu, pv = (i + 0.5) / w - 0.5, (j + 0.5) / w - 0.5
        ex, en = [], []
        for pl, r in zip(planes, rhos):
            lo, hi = A.ray_interval(pl, pu, pv)
            if np.isfinite(lo) and np.isfinite(hi) and hi > lo:
                ex.append(r * (hi - t_ref))
                en.append(r * (lo - t_ref))
        ref = img[j, i]
        f64 = sum(ex) - sum(en)
        e32 = np.float32(0.0)
        n32 = np.float32(0.0)
        for a in ex:
            e32 = np.float32(e32 + np.float32(a))
        for a in en:
            n32 = np.float32(n32 + np.float32(a))
        worst64 = max(worst64, abs(f64 - ref) / ref)
        worst32 = max(worst32, abs(float(e32 - n32) - ref) / ref)
        pred = max(pred, 2.0 ** -24 * abs(t_ref) * max(rhos) * math.sqrt(2 * len(ex)) / ref)
    assert worst64 < 1e-9, worst64
    assert worst32 > 1e-3, worst32          # the cancellation: ten times the per-pixel bar and more
    assert worst32 < 50 * pred, (worst32, pred)


# ------------------------------------------------- C6: Monte Carlo on rays
def test_c6_monte_carlo_along_rays():
    n = 2
    x, y, z = W.random_lattice(n, 0.12, seed=21)
    tets = lattice_tets(x, y, z, n)
    mass = 1.0 / len(tets)
    rho = mass / np.abs(signed_volumes(tets))
    imgs = []
    for sx in (-1, 0, 1):
        for sy in (-1, 0, 1):
            imgs.append(tets + np.array([sx, sy, 0.0]))
    tets9 = np.concatenate(imgs)
    rho9 = np.tile(rho, 9)
    wpx = 6
    img, _ = O.project_region(x, y, z, (n, n, n), W.z_view(wpx))
    rng = np.random.default_rng(4)
    K = 6000
    zlo, zhi = tets9[:, :, 2].min(), tets9[:, :, 2].max()
    for (j, i) in [(0, 0), (2, 3), (5, 5), (1, 4)]:
        pu, pv = (i + 0.5) / wpx, (j + 0.5) / wpx
        t = rng.uniform(zlo, zhi, size=K)
        pts = np.stack([np.full(K, pu), np.full(K, pv), t], axis=1)
        dens = points_in_tets(pts, tets9).astype(np.float64) @ rho9
        est = dens.mean() * (zhi - zlo)
        sig = dens.std(ddof=1) / math.sqrt(K) * (zhi - zlo)
        assert abs(est - img[j, i]) <= 4 * sig + 1e-12, (i, j, est, img[j, i], sig)


# ----------------------------------------------- C7: brute force, all pairs
def test_c7_brute_force_all_pairs_wrap():
    n = 3
    x, y, z = W.random_lattice(n, 0.1, seed=8)
    tets = lattice_tets(x, y, z, n)
    mass = 1.0 / len(tets)
    w, h = 14, 9
    img, st = O.project_region(x, y, z, (n, n, n), W.z_view(w, h))
    jj, ii = np.mgrid[0:h, 0:w]
    pts = np.stack([((ii + 0.5) / w).ravel(), ((jj + 0.5) / h).ravel()], 1)
    ref = np.zeros(h * w)
    frags = 0
    for tv in tets:
        for sx in (-1, 0, 1):
            for sy in (-1, 0, 1):
                val = tent_value(tv[:, :2] + np.array([sx, sy]), mass, pts)
                ref += val
                frags += int((val > 0).sum())
    np.testing.assert_allclose(img.ravel(), ref, rtol=1e-10, atol=0)
    assert st["fragments"] == frags


def test_c7_brute_force_all_pairs_rotated_no_wrap():
    n = 3
    x, y, z = W.random_lattice(n, 0.1, seed=9)
    tets = lattice_tets(x, y, z, n)
    mass = 1.0 / len(tets)
    R = W.random_rotations(1, seed=5)[0]
    w, h = 17, 13
    view = W.rotated_view(R, w, h, side=1.4)
    img, _ = O.project_region(x, y, z, (n, n, n), view)
    jj, ii = np.mgrid[0:h, 0:w]
    pts = np.stack([(-0.7 + (ii + 0.5) * 1.4 / w).ravel(), (-0.7 + (jj + 0.5) * 1.4 / h).ravel()], 1)
    ref = np.zeros(h * w)
    for tv in tets:
        yv = (tv - 0.5) @ R.T
        ref += tent_value(yv[:, :2], mass, pts)
    np.testing.assert_allclose(img.ravel(), ref, rtol=1e-10, atol=1e-12)


# ------------------------------------------------- C9: order independence
def test_c9_order_independence():
    n = 4
    x, y, z = W.random_lattice(n, 0.15, seed=12)
    tets = lattice_tets(x, y, z, n)
    view = W.rotated_view(np.eye(3), 32, 32, side=1.0, center=(0.5, 0.5, 0.5))
    m = np.full(len(tets), 1.0 / len(tets))
    a, _ = O.project_tets(tets, m, view)
    perm = np.random.default_rng(1).permutation(len(tets))
    b, _ = O.project_tets(tets[perm], m, view)
    np.testing.assert_allclose(a, b, rtol=1e-13, atol=0)


def test_region_mode_is_thread_count_independent(tiny_lattice):
    x, y, z = tiny_lattice
    v = W.z_view(96, 80)
    a, sa = O.project_region(x, y, z, (32, 32, 32), v, nthreads=1)
    b, sb = O.project_region(x, y, z, (32, 32, 32), v, nthreads=5)
    assert np.array_equal(a, b) and sa == sb


# ------------------------------------------------------- C10: dyadic shift
def test_c10_dyadic_shift_is_cyclic_shift():
    n, w = 8, 64
    x, y, z = W.zeldovich(n, 3, 2.0)
    x = (np.round(x.astype(np.float64) * 2 ** 24) / 2 ** 24).astype(np.float32)
    x[x >= 1] -= 1
    k = 5
    xs = x.astype(np.float64) + k / w
    xs[xs >= 1] -= 1
    xs = xs.astype(np.float32)
    assert np.array_equal(xs.astype(np.float64), np.mod(x.astype(np.float64) + k / w, 1.0))
    a, _ = O.project_region(x, y, z, (n, n, n), W.z_view(w))
    b, _ = O.project_region(xs, y, z, (n, n, n), W.z_view(w))
    np.testing.assert_allclose(np.roll(a, k, axis=1), b, rtol=1e-12, atol=0)


# ------------------------------------------ mode consistency and edge cases
def test_pixel_and_crop_modes_agree_with_full_image(tiny_lattice):
    x, y, z = tiny_lattice
    v = W.z_view(128, 96)
    full, st = O.project_region(x, y, z, (32, 32, 32), v)
    crop, _ = O.project_region(x, y, z, (32, 32, 32), v, crop=(100, 7, 28, 40))
    np.testing.assert_allclose(crop, full[7:47, 100:128], rtol=1e-14, atol=0)
    rng = np.random.default_rng(0)
    px = rng.integers(0, 128, 300)
    py = rng.integers(0, 96, 300)
    vals, _ = O.project_pixels(x, y, z, (32, 32, 32), v, px, py)
    np.testing.assert_allclose(vals, full[py, px], rtol=1e-14, atol=0)
    assert st["fragments"] > 0


def test_single_pixel_image_and_minimum_lattice():
    x, y, z = W.random_lattice(2, 0.05, seed=2)
    img, st = O.project_region(x, y, z, (2, 2, 2), W.z_view(1, 1))
    assert img.shape == (1, 1) and np.isfinite(img).all() and st["tets"] == 48


def test_invalid_arguments_rejected():
    x, y, z = W.undisplaced(2)
    bad = W.z_view(0)
    with pytest.raises(RuntimeError):
        O.project_region(x, y, z, (2, 2, 2), bad)
    with pytest.raises(RuntimeError):
        O.project_region(x, y, z, (1, 2, 2), W.z_view(4))

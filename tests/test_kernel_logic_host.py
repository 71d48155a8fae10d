"""The kernels' per-tetrahedron code (tess_tet.h), compiled for the host and
driven by plain loops in the kernels' order of work, against the FP64 oracle.
Runs without a GPU; it checks the arithmetic and control flow the HIP kernels
share (setup, footprint, walls, the row spans and their second differences,
tile lists and work items), not the kernels' scheduling."""
import numpy as np
import pytest

import oracle as O
import workloads as W

hostcheck = pytest.importorskip("hostcheck")


def rel(a, b):
    tau = 1e-6 * np.abs(b).mean()
    return (np.abs(a - b) / np.maximum(np.abs(b), tau)).max()


@pytest.mark.parametrize("n,w,h", [(4, 16, 16), (8, 24, 40), (4, 2, 10), (2, 6, 4), (4, 7, 5)])
def test_undisplaced_lattice_is_one(n, w, h):
    # every ray crosses exactly one cube layer per lattice step: column density 1,
    # with pixel centres on cube faces and tetrahedron faces seen edge-on
    img, _, st = hostcheck.pipeline(*W.undisplaced(n), (n, n, n), W.z_view(w, h), tile_rows=3,
                                    tile_cols=max(16, w // 2))
    np.testing.assert_allclose(img, 1.0, rtol=0, atol=1e-12)
    assert st["tets"] == 6 * n ** 3


def test_z_only_displacement_is_one():
    n = 16
    q = W.lattice_q(n)
    A = (1 - 1e-4) / (2 * n * np.sin(np.pi / n))
    f = A * np.sin(2 * np.pi * q[:, 2] - np.pi / n) + 0.05 * np.sin(2 * np.pi * (q[:, 0] + 2 * q[:, 2]))
    xyz = (q[:, 0].astype(np.float32), q[:, 1].astype(np.float32), W.wrap_to_f32(q[:, 2] - f, 1.0))
    img, _, _ = hostcheck.pipeline(*xyz, (n, n, n), W.z_view(64, 48))
    np.testing.assert_allclose(img, 1.0, rtol=0, atol=1e-10)


@pytest.mark.parametrize("rows,cols,chunk", [(8, 200, 4096), (4, 64, 100), (16, 16, 37), (1, 200, 4096),
                                             (3, 37, 1000)])
def test_zeldovich_wrap_matches_oracle_any_tiling(rows, cols, chunk):
    n = 16
    xyz = W.zeldovich(n, 5, 6.0, seed=99)
    view = W.z_view(200, 136)
    img, img32, st = hostcheck.pipeline(*xyz, (n, n, n), view, tile_rows=rows, tile_cols=cols, chunk=chunk)
    ref, ost = O.project_region(*xyz, (n, n, n), view)
    # FP64 row sums: rounding grows along a row, ~1e-9 at its end here
    assert rel(img, ref) < 1e-8
    assert rel(img32.astype(np.float64), ref) < 1e-6
    assert st["tets"] == ost["tets"] and st["inverted"] == ost["inverted"]
    assert st["fragments"] == ost["fragments"]


@pytest.mark.parametrize("quantity", ["unit", "density2"])
@pytest.mark.parametrize("view_kind", ["z", "rotated"])
def test_projected_quantities_match_oracle(quantity, view_kind):
    # q = 1 and q = rho^2: the density footprint with its mass scaled per
    # tetrahedron; shell crossing and a rotated window without wrap
    n = 12
    xyz = W.zeldovich(n, 4, 6.0, seed=5)
    if view_kind == "z":
        view = dict(W.z_view(96, 72), quantity=quantity)
    else:
        view = dict(W.rotated_view(W.random_rotations(1, seed=3)[0], 80, 64), quantity=quantity)
    img, _, st = hostcheck.pipeline(*xyz, (n, n, n), view, tile_rows=8, tile_cols=40, chunk=500,
                                    total_mass=2.0)
    ref, ost = O.project_region(*xyz, (n, n, n), view, total_mass=2.0)
    assert np.abs(img - ref).max() < 1e-8 * np.abs(ref).max()
    # empty pixels of the rotated window hold only FP64 noise of the row sums,
    # which scales with the image's maximum (a rho^2 image peaks at ~1000x its
    # mean): held to 1e-12 of the maximum, the other pixels to the usual bar
    empty = ref == 0.0
    assert np.abs(img[empty]).max(initial=0.0) <= 1e-12 * np.abs(ref).max()
    assert rel(np.where(empty, 0.0, img), ref) < (1e-8 if view_kind == "z" else 1e-5)
    assert st["fragments"] == ost["fragments"]
    assert st["fp64_dets"] == st["tets"] + st["zero_volume"]


@pytest.mark.parametrize("view_kind,slab", [("z", (-0.2, 0.15)), ("z", (0.3, 0.9)), ("rotated", (-0.4, 0.1))])
def test_depth_slab_matches_oracle(view_kind, slab):
    # the face form: chords clipped to the slab, front/back face envelopes
    n = 12
    xyz = W.zeldovich(n, 4, 6.0, seed=5)
    base = W.z_view(96, 72) if view_kind == "z" else W.rotated_view(W.random_rotations(1, seed=3)[0], 80, 64)
    view = dict(base, slab=slab)
    img, _, st = hostcheck.pipeline(*xyz, (n, n, n), view, tile_rows=8, tile_cols=40, chunk=500)
    ref, ost = O.project_region(*xyz, (n, n, n), view)
    assert np.abs(img - ref).max() < 1e-8 * np.abs(ref).max()
    assert rel(img, ref) < (1e-8 if view_kind == "z" else 1e-5)  # empty pixels: FP64 row-sum noise
    assert st["tets"] == ost["tets"]
    assert abs(st["fragments"] - ost["fragments"]) <= 1e-6 * ost["fragments"] + 4


def test_depth_slab_undisplaced_walls_closed_form():
    # every face parallel to z is a wall; the slab keeps rho (s1 - s0)
    n, M = 4, 3.0
    view = dict(W.z_view(16, 12), slab=(-0.25, 0.1))
    img, _, _ = hostcheck.pipeline(*W.undisplaced(n), (n, n, n), view, total_mass=M, tile_rows=4, tile_cols=8)
    np.testing.assert_allclose(img, M * 0.35, rtol=1e-12)


def test_depth_slabs_add_up_to_the_projection():
    n = 10
    xyz = W.zeldovich(n, 3, 5.0, seed=21)
    view = W.z_view(64, 48)
    full, _, _ = hostcheck.pipeline(*xyz, (n, n, n), view, tile_rows=8, tile_cols=32)
    cuts = np.linspace(-1.2, 1.2, 9)
    parts = [hostcheck.pipeline(*xyz, (n, n, n), dict(view, slab=(a, b)), tile_rows=8, tile_cols=32)[0]
             for a, b in zip(cuts[:-1], cuts[1:])]
    np.testing.assert_allclose(sum(parts), full, rtol=0, atol=1e-9 * np.abs(full).max())


def test_depth_slab_with_density_squared():
    n = 12
    xyz = W.zeldovich(n, 4, 6.0, seed=5)
    view = dict(W.z_view(96, 72), slab=(-0.3, 0.2), quantity="density2")
    img, _, _ = hostcheck.pipeline(*xyz, (n, n, n), view, tile_rows=8, tile_cols=40, total_mass=2.0)
    ref, _ = O.project_region(*xyz, (n, n, n), view, total_mass=2.0)
    assert rel(img, ref) < 1e-8


@pytest.mark.parametrize("view_kind,quantity", [("z", "density"), ("rotated", "density"), ("z", "density2")])
def test_centroid_splats_match_oracle(view_kind, quantity):
    # the centroid method: kernel values added directly (no row sums)
    n = 12
    xyz = W.zeldovich(n, 4, 6.0, seed=5)
    base = W.z_view(96, 72) if view_kind == "z" else W.rotated_view(W.random_rotations(1, seed=3)[0], 80, 64)
    view = dict(base, method="centroids", quantity=quantity)
    img, _, st = hostcheck.pipeline(*xyz, (n, n, n), view, tile_rows=8, tile_cols=40, chunk=500)
    ref, ost = O.splat_image(*xyz, (n, n, n), view)
    assert np.abs(img - ref).max() <= 1e-12 * np.abs(ref).max()
    assert st["fragments"] == ost["fragments"] and st["tets"] == ost["tets"]


@pytest.mark.parametrize("camera,quantity", [((0.45, 0.52, -1.4), "density"), ((0.37, 0.58, 0.41), "density"),
                                             ((0.37, 0.58, 0.41), "unit"), ((0.61, 0.3, -0.9), "density2")])
def test_perspective_matches_oracle(camera, quantity):
    # a camera outside the volume and one inside it (half-lines cut at the
    # camera, tetrahedra behind it skipped, ones around it on every pixel)
    n = 12
    xyz = W.zeldovich(n, 4, 3.0, seed=9)
    R = W.random_rotations(1, seed=4)[0] if camera[2] > 0 else np.eye(3)
    view = dict(W.perspective_view(R, camera, 72, 56, extent=(1.5, 1.2)), quantity=quantity)
    img, _, st = hostcheck.pipeline(*xyz, (n, n, n), view, tile_rows=8, tile_cols=40, chunk=500)
    ref, ost = O.project_region(*xyz, (n, n, n), view)
    assert np.abs(img - ref).max() <= 1e-11 * np.abs(ref).max()
    assert st["fragments"] == ost["fragments"] and st["tets"] == ost["tets"]


@pytest.mark.parametrize("method,radius", [("centroids", 0.0), ("hybrid", 0.9), ("hybrid", 1.6)])
def test_perspective_billboards_and_hybrid_match_oracle(method, radius):
    # billboards under the perspective camera, alone and beyond the hybrid's
    # sphere (exact inside it); camera inside the volume for radius 0.9
    n = 12
    xyz = W.zeldovich(n, 4, 3.0, seed=9)
    camera = (0.41, 0.55, 0.3) if radius < 1.0 else (0.45, 0.52, -1.2)
    view = dict(W.perspective_view(np.eye(3), camera, 72, 56, extent=(1.5, 1.2)), method=method, lod_radius=radius)
    img, _, st = hostcheck.pipeline(*xyz, (n, n, n), view, tile_rows=8, tile_cols=40, chunk=500)
    ref, ost = O.project_region(*xyz, (n, n, n), view)
    assert np.abs(img - ref).max() <= 1e-11 * np.abs(ref).max()
    assert st["fragments"] == ost["fragments"] and st["tets"] == ost["tets"]


def test_tallest_tiles_match_oracle():
    # 256-row tiles (the largest the library accepts): row offsets of up to 255
    # inside a tile, footprints taller than the lattice spacing wrapping in y
    n = 16
    xyz = W.zeldovich(n, 5, 6.0, seed=7)
    view = W.z_view(64, 300)
    img, _, st = hostcheck.pipeline(*xyz, (n, n, n), view, tile_rows=256, tile_cols=64, chunk=4096)
    ref, ost = O.project_region(*xyz, (n, n, n), view)
    assert rel(img, ref) < 1e-8
    assert st["fragments"] == ost["fragments"]


@pytest.mark.parametrize("rows,cols", [(8, 50), (5, 16), (2, 17)])
def test_rotated_view_without_wrap_matches_oracle(rows, cols):
    n = 8
    xyz = W.random_lattice(n, 0.2, seed=4)
    R = W.random_rotations(1, seed=3)[0]
    view = W.rotated_view(R, 50, 44)
    img, _, st = hostcheck.pipeline(*xyz, (n, n, n), view, tile_rows=rows, tile_cols=cols)
    ref, ost = O.project_region(*xyz, (n, n, n), view)
    assert np.abs(img - ref).max() < 1e-8 * np.abs(ref).max()
    assert rel(img, ref) < 1e-5  # empty pixels hold only FP64 noise of the row sums
    assert st["fragments"] == ost["fragments"]


@pytest.mark.parametrize("crease_div", [0.0, None, 1e-30])
def test_crease_and_line_forms_agree(crease_div):
    # every footprint in line form, the library's split, every one in crease form
    n = 16
    xyz = W.zeldovich(n, 5, 4.0, seed=5)
    view = W.rotated_view(W.random_rotations(1, seed=31)[0], 96, 80)
    img, _, st = hostcheck.pipeline(*xyz, (n, n, n), view, tile_rows=4, tile_cols=32, crease_div=crease_div)
    ref, ost = O.project_region(*xyz, (n, n, n), view)
    if crease_div == 0.0:
        assert st["crease_records"] == 0
    elif crease_div is None:
        assert 0 < st["crease_records"] < st["tets"]
        assert rel(img, ref) < 1e-5
    else:
        assert st["crease_records"] > 0.95 * st["tets"]
    assert np.abs(img - ref).max() < 1e-8 * np.abs(ref).max()
    assert st["fragments"] == ost["fragments"]


def test_non_periodic_lattice_matches_oracle():
    n = 9
    xyz = W.random_lattice(n, 0.3, seed=7)
    R = W.random_rotations(2, seed=5)[1]
    view = W.rotated_view(R, 61, 47, side=1.6)
    img, _, st = hostcheck.pipeline(*xyz, (n, n, n), view, periodic=False, tile_rows=4, tile_cols=32)
    ref, ost = O.project_region(*xyz, (n, n, n), view, periodic=False)
    assert np.abs(img - ref).max() < 1e-8 * np.abs(ref).max()
    assert st["tets"] == ost["tets"] and st["fragments"] == ost["fragments"]


def test_fp64_determinants_give_the_same_image():
    n = 8
    xyz = W.zeldovich(n, 3, 8.0, seed=1)
    view = W.z_view(40, 40)
    a, _, sa = hostcheck.pipeline(*xyz, (n, n, n), view, precision=0)
    b, _, sb = hostcheck.pipeline(*xyz, (n, n, n), view, precision=1)
    assert sb["fp64_dets"] == sb["tets"] + sb["zero_volume"] and sa["fp64_dets"] < sb["fp64_dets"]
    # the footprint uses projected vertices only; the determinant decides sign and V == 0
    assert sa["inverted"] == sb["inverted"] and sa["tets"] == sb["tets"]
    np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("w,h", [(1, 1), (1, 5), (7, 1)])
def test_degenerate_image_sizes(w, h):
    n = 6
    xyz = W.zeldovich(n, 2, 3.0, seed=2)
    view = W.z_view(w, h)
    img, _, st = hostcheck.pipeline(*xyz, (n, n, n), view, tile_rows=2, tile_cols=16)
    ref, ost = O.project_region(*xyz, (n, n, n), view)
    assert rel(img, ref) < 1e-8
    assert st["fragments"] == ost["fragments"]


def test_minimum_lattice_and_huge_footprints():
    # n = 2 with strong displacement: footprints wider than the image, many periodic copies
    n = 2
    xyz = W.random_lattice(n, 0.45, seed=11)
    view = W.z_view(23, 19)
    img, _, st = hostcheck.pipeline(*xyz, (n, n, n), view, tile_rows=4, tile_cols=16)
    ref, ost = O.project_region(*xyz, (n, n, n), view)
    assert rel(img, ref) < 1e-8
    assert st["fragments"] == ost["fragments"]


@pytest.mark.parametrize("wrap", [1, 0])
def test_edge_form_equals_per_tetrahedron_form(wrap):
    # strongly shell-crossed lattice: many tetrahedra reach across the
    # periodic seam (wrap) or past the image's columns (no wrap); the creases
    # summed per mesh edge give the per-tetrahedron image to rounding and the
    # same fragment count, and under wrap nearly every crease-form
    # tetrahedron goes to its edges (all but those about as wide as the image)
    n = 24
    xyz = W.zeldovich(n, 8, 8.0, seed=13)
    view = W.z_view(192, 160) if wrap else W.rotated_view(W.random_rotations(1, seed=6)[0], 150, 130)
    a, _, sa = hostcheck.pipeline(*xyz, (n, n, n), view, tile_rows=8, tile_cols=64, edges=True)
    b, _, sb = hostcheck.pipeline(*xyz, (n, n, n), view, tile_rows=8, tile_cols=64, edges=False)
    assert np.abs(a - b).max() < 1e-9 * np.abs(b).max()
    assert sa["fragments"] == sb["fragments"] and sa["crease_records"] == sb["crease_records"]
    if wrap:
        assert sa["edged"] > 0.99 * sa["crease_records"]
    else:
        assert 0 < sa["edged"] < sa["crease_records"]
    ref, ost = O.project_region(*xyz, (n, n, n), view)
    assert np.abs(a - ref).max() < 1e-8 * np.abs(ref).max()
    assert sa["fragments"] == ost["fragments"]


@pytest.mark.parametrize("wrap", [True, False])
@pytest.mark.parametrize("rows,cols", [(8, 64), (32, 512), (3, 37), (1, 200)])
def test_edge_form_short_loop_without_counts(wrap, rows, cols):
    # the edge raster's loop without the fragment count (the library's
    # default without stats): the same image as the counting loop and the
    # oracle's, on a strongly shell-crossed lattice with many tetrahedra
    # across the periodic seam
    n = 24
    xyz = W.zeldovich(n, 8, 8.0, seed=13)
    view = W.z_view(192, 160) if wrap else W.rotated_view(W.random_rotations(1, seed=6)[0], 150, 130)
    a, _, _ = hostcheck.pipeline(*xyz, (n, n, n), view, tile_rows=rows, tile_cols=cols, edges=True)
    c, _, _ = hostcheck.pipeline(*xyz, (n, n, n), view, tile_rows=rows, tile_cols=cols, edges="no_counts")
    assert np.abs(c - a).max() < 1e-9 * np.abs(a).max()
    # the first copy's kinks drawn from the edge job, the rest by the pair
    # routine that skips them: the same terms in the same order
    s, _, _ = hostcheck.pipeline(*xyz, (n, n, n), view, tile_rows=rows, tile_cols=cols, edges="split")
    assert np.array_equal(s, c)
    ref, _ = O.project_region(*xyz, (n, n, n), view)
    # FP64 row sums: ~1e-12 at the ends of rows, also on empty pixels of the
    # rotated window (the contract's 1e-4 against its 1e-6-of-the-mean floor)
    assert np.abs(c - ref).max() < 1e-8 * np.abs(ref).max()
    assert rel(c, ref) < 1e-4


@pytest.mark.parametrize("edges", [False, True])
def test_tile_columns_leave_no_residual_slope(edges):
    # a kink whose two second-difference entries fall in two tiles is drawn
    # by both; they must compute it identically (in the record's frame), or
    # the entries no longer add up to its slope change and the row sums leave
    # a slope on the empty pixels right of the footprints.  A rotated window
    # (empty pixels) with 2 pixels per lattice cell, one tile per row against
    # 16- to 256-column tiles: the same image to FP64 rounding, empty pixels
    # included
    n = 32
    xyz = W.zeldovich(n, 8, 2.0, seed=17)
    view = W.rotated_view(W.random_rotations(1, seed=5)[0], 128, 112)
    one, _, _ = hostcheck.pipeline(*xyz, (n, n, n), view, tile_rows=16, tile_cols=128, edges=edges)
    ref, _ = O.project_region(*xyz, (n, n, n), view)
    for cols in (64, 37, 16):
        img, _, _ = hostcheck.pipeline(*xyz, (n, n, n), view, tile_rows=16, tile_cols=cols, edges=edges)
        assert np.abs(img - one).max() < 1e-12 * np.abs(one).max(), cols
        assert rel(img, ref) < 1e-5, cols


def test_fast_floor_division_is_exact():
    # the binning's and the raster's floor division of pixel coordinates by
    # tile and image sizes takes the FP32 reciprocal plus one correction; it
    # must be exact even with the reciprocal a few ulp off
    import ctypes
    f = hostcheck.lib().hc_floor_div_check
    f.restype = ctypes.c_int64
    for ulps in (0, 1, 4):
        assert f(ulps) == 0, ulps

@pytest.mark.parametrize("case", ["wrap", "rotated", "density2", "steep", "undisplaced"])
def test_edge_setup_common_path_equals_general_setup(case):
    # The edge form's setup takes the common tetrahedron directly (its six
    # slope changes from the silhouette set alone, a steep one's line-form
    # record from its silhouette edges' face functions) and leaves the rest
    # to the general code.  Run every tetrahedron through the general code
    # instead: the slots, records, image and counts must not change, bit for
    # bit.  "steep" lowers the crease form's slope bound so that many
    # footprints keep the line form; "undisplaced" has faces seen edge-on
    # (walls), which only the general code takes.
    n = 16
    kw = {}
    if case == "undisplaced":
        xyz = W.undisplaced(n)
        view = W.z_view(96)
    else:
        xyz = W.zeldovich(n, 4, 4.0, seed=7)
        if case == "rotated":
            view = W.rotated_view(W.random_rotations(1, seed=3)[0], 120, 110)
        elif case == "density2":
            view = dict(W.z_view(128), quantity="density2")
        else:
            view = W.z_view(128)
        if case == "steep":
            kw["crease_div"] = 128 / 4.0
    fast = hostcheck.pipeline(*xyz, (n, n, n), view, edges=True, **kw)
    general = hostcheck.pipeline(*xyz, (n, n, n), view, edges="general", **kw)
    assert np.array_equal(fast[0], general[0]) and np.array_equal(fast[1], general[1])
    assert fast[2] == general[2]
    assert fast[2]["edged"] > 0
    if case == "steep":
        assert fast[2]["crease_records"] < 0.95 * fast[2]["tets"]  # many line-form records

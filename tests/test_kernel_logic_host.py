"""The kernels' per-tetrahedron code (tess_tet.h), compiled for the host and
driven by plain loops, against the FP64 oracle.  Runs without a GPU; it checks
the arithmetic and control flow the HIP kernels share (setup, footprint,
walls, strip evaluation, tile culling), not the kernels' scheduling."""
import numpy as np
import pytest

import oracle as O
import workloads as W

hostcheck = pytest.importorskip("hostcheck")


def rel(a, b):
    tau = 1e-6 * np.abs(b).mean()
    return (np.abs(a - b) / np.maximum(np.abs(b), tau)).max()


@pytest.mark.parametrize("n,w,h", [(4, 16, 16), (8, 24, 40), (4, 2, 10), (2, 6, 4)])
def test_undisplaced_lattice_is_one(n, w, h):
    img, st = hostcheck.project(*W.undisplaced(n), (n, n, n), W.z_view(w, h))
    np.testing.assert_allclose(img, 1.0, rtol=0, atol=1e-6)
    assert st["culled_but_covered"] == 0


def test_z_only_displacement_is_one():
    n = 16
    q = W.lattice_q(n)
    A = (1 - 1e-4) / (2 * n * np.sin(np.pi / n))
    f = A * np.sin(2 * np.pi * q[:, 2] - np.pi / n) + 0.05 * np.sin(2 * np.pi * (q[:, 0] + 2 * q[:, 2]))
    xyz = (q[:, 0].astype(np.float32), q[:, 1].astype(np.float32), W.wrap_to_f32(q[:, 2] - f, 1.0))
    img, st = hostcheck.project(*xyz, (n, n, n), W.z_view(64, 48))
    np.testing.assert_allclose(img, 1.0, rtol=0, atol=1e-5)


@pytest.mark.parametrize("tile", [16, 32, 64])
def test_zeldovich_wrap_matches_oracle(tile):
    n = 16
    xyz = W.zeldovich(n, 5, 6.0, seed=99)
    view = W.z_view(200, 136)
    img, st = hostcheck.project(*xyz, (n, n, n), view, tile=tile)
    ref, ost = O.project_region(*xyz, (n, n, n), view)
    assert rel(img, ref) < 1e-4
    assert st["tets"] == ost["tets"] and st["inverted"] == ost["inverted"]
    assert st["fragments"] == ost["fragments"]
    assert st["culled_but_covered"] == 0


def test_fp64_footprints_match_oracle_tightly():
    n = 8
    xyz = W.random_lattice(n, 0.2, seed=4)
    R = W.random_rotations(1, seed=3)[0]
    view = W.rotated_view(R, 50, 44)
    img, st = hostcheck.project(*xyz, (n, n, n), view, fp64_cond=-1.0)
    ref, _ = O.project_region(*xyz, (n, n, n), view)
    assert rel(img, ref) < 1e-10
    assert st["fp64_tets"] > 0

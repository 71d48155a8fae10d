"""Host-side checks of the C ABI that need no GPU: the library loads, every
symbol declared in include/tess.h is exported, and argument validation
rejects bad descriptors and views before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "tess.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tess_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def tess():
    import paper_1208_3206_amd as t
    return t


def test_every_declared_symbol_is_exported(tess):
    names = declared_functions()
    assert "tess_project" in names and "tess_build" in names
    for n in names:
        assert hasattr(tess.lib(), n), n
    assert set(names) == set(tess.EXPORTS)


def test_binding_structs_match_the_library(tess):
    # the ctypes mirrors must have the C layouts' sizes (a mismatch would
    # make the library read or write past the binding's buffers)
    mirrors = [tess.TessBuildDesc, tess.TessView, tess.TessTune, tess.TessStats, tess.TessRefineDesc]
    for which, cls in enumerate(mirrors):
        assert tess.lib().tess_struct_size(which) == ctypes.sizeof(cls), cls.__name__
    assert tess.lib().tess_struct_size(99) == 0


def test_version_and_empty_error(tess):
    assert tess.version() >= 100
    assert isinstance(tess.last_error(), str)


def test_build_desc_validation(tess):
    d = tess.build_desc((8, 8, 8))
    tess.check_build_desc(d)
    for field, value in (("total_mass", -1.0), ("precision", 7), ("periodic", 3)):
        bad = tess.build_desc((8, 8, 8))
        setattr(bad, field, value)
        with pytest.raises(tess.TessError) as ei:
            tess.check_build_desc(bad)
        assert ei.value.status == tess.TESS_EINVAL
    bad = tess.build_desc((1, 8, 8))
    with pytest.raises(tess.TessError):
        tess.check_build_desc(bad)
    bad = tess.build_desc((8, 8, 8), box=(1.0, 0.0, 1.0))
    with pytest.raises(tess.TessError):
        tess.check_build_desc(bad)


def test_view_validation(tess):
    d = tess.build_desc((8, 8, 8))
    tess.check_view(W.z_view(64), d)
    R = W.random_rotations(1)[0]
    tess.check_view(W.rotated_view(R, 64), d)
    cases = [
        dict(W.z_view(64), width=0),
        dict(W.z_view(64), height=20000),
        dict(W.z_view(64), extent=[1.0, -1.0]),
        dict(W.z_view(64), rot=[1, 0, 0, 0, 1, 0, 0, 0, 1.1]),
        dict(W.rotated_view(R, 64), wrap=1),            # wrap with a rotated view
        dict(W.z_view(64), extent=[1.0, 0.5]),           # wrap with extent != box
        dict(W.z_view(64), center=[0.5, float("nan"), 0.5]),
    ]
    for v in cases:
        with pytest.raises(tess.TessError) as ei:
            tess.check_view(v, d)
        assert ei.value.status == tess.TESS_EINVAL, v
    nonper = tess.build_desc((8, 8, 8), periodic=False)
    with pytest.raises(tess.TessError):
        tess.check_view(W.z_view(64), nonper)
    # permuted axes are fine for wrap (projection along x)
    xview = dict(W.z_view(32), rot=[0, 1, 0, 0, 0, 1, 1, 0, 0])
    tess.check_view(xview, d)
    # the projected quantity: 0 density, 1 unit, 2 density^2; nothing else
    for name in ("density", "unit", "density2"):
        tess.check_view(dict(W.z_view(64), quantity=name), d)
    v = tess.make_view(W.z_view(64))
    v.quantity = 3
    assert tess.lib().tess_check_view(ctypes.byref(v), None) == tess.TESS_EINVAL
    # drawing methods, and no slab with centroids
    tess.check_view(dict(W.z_view(64), method="centroids"), d)
    for bad in (dict(W.z_view(64), method="centroids", slab=(0.0, 0.1)),):
        with pytest.raises(tess.TessError):
            tess.check_view(bad, d)
    v = tess.make_view(W.z_view(64))
    v.method = 2
    assert tess.lib().tess_check_view(ctypes.byref(v), None) == tess.TESS_EINVAL
    v.method, v.projection = 0, 2
    assert tess.lib().tess_check_view(ctypes.byref(v), None) == tess.TESS_EINVAL
    # perspective: no wrap, no slab, the tessellation method
    persp = W.perspective_view(np.eye(3), (0.5, 0.5, -1.0), 64)
    tess.check_view(persp, d)
    tess.check_view(dict(persp, method="centroids"), d)
    tess.check_view(dict(persp, method="hybrid", lod_radius=0.3), d)
    for bad in (dict(persp, wrap=1), dict(persp, slab=(0.0, 0.1)), dict(W.z_view(64), method="hybrid"),
                dict(persp, method="hybrid", lod_radius=-1.0),
                dict(persp, method="hybrid", lod_radius=float("inf"))):
        with pytest.raises(tess.TessError):
            tess.check_view(bad, d)
    v = tess.make_view(W.z_view(64))
    v.method = 3
    assert tess.lib().tess_check_view(ctypes.byref(v), None) == tess.TESS_EINVAL
    # depth slabs: finite and ordered
    tess.check_view(dict(W.z_view(64), slab=(-0.1, 0.2)), d)
    for bad in ((0.2, 0.2), (0.3, -0.1), (float("nan"), 0.1), (-float("inf"), 0.0)):
        with pytest.raises(tess.TessError):
            tess.check_view(dict(W.z_view(64), slab=bad), d)


def test_null_arguments_rejected_without_gpu(tess):
    L = tess.lib()
    st = L.tess_project(None, None, None, None, None, None)
    assert st == tess.TESS_EINVAL
    assert "NULL" in tess.last_error()
    st = L.tess_build(None, None, None, None, None, None, None)
    assert st == tess.TESS_EINVAL

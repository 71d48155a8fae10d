"""FP64 CPU oracle (test infrastructure only).

This package is the reference the GPU library is checked against.  Only the
test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import it; the GPU library never does, and this package
imports nothing from the GPU library.

``tess_oracle.c`` computes the column-density projection by exact FP64
ray-tetrahedron clipping (see its header for the steps and the paper
passages they follow).  This module only compiles it, loads it with ctypes
and marshals numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Dict, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tess_oracle.c")
_LIB = os.path.join(_HERE, "libtess_oracle.so")


class OrcProblem(ctypes.Structure):
    _fields_ = [
        ("dims", ctypes.c_int32 * 3),
        ("box", ctypes.c_double * 3),
        ("periodic", ctypes.c_int32),
        ("total_mass", ctypes.c_double),
        ("rot", ctypes.c_double * 9),
        ("center", ctypes.c_double * 3),
        ("extent", ctypes.c_double * 2),
        ("width", ctypes.c_int32),
        ("height", ctypes.c_int32),
        ("wrap", ctypes.c_int32),
        ("qpow", ctypes.c_int32),
        ("slab", ctypes.c_int32),
        ("slab_t", ctypes.c_double * 2),
        ("perspective", ctypes.c_int32),
        ("method", ctypes.c_int32),
        ("lod_radius", ctypes.c_double),
    ]

# projected per-tetrahedron value q = rho^p by name (view["quantity"])
QUANTITY_POWER = {"density": 1, "unit": 0, "density2": 2}


class OrcStats(ctypes.Structure):
    _fields_ = [("tets", ctypes.c_int64), ("zero_volume", ctypes.c_int64),
                ("inverted", ctypes.c_int64), ("fragments", ctypes.c_int64)]

    def as_dict(self) -> Dict[str, int]:
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP64, OpenMP).  Returns the library path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
               "-fno-fast-math", "-ffp-contract=off", _SRC, "-o", _LIB + ".tmp%x" % os.getpid(), "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp%x" % os.getpid(), _LIB)  # (a file per process: parallel test workers)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        fptr = P(ctypes.c_float)
        dptr = P(ctypes.c_double)
        L.orc_project_region.argtypes = [P(OrcProblem), fptr, fptr, fptr, ctypes.c_int32,
                                         ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                         dptr, P(OrcStats), ctypes.c_int32]
        L.orc_project_pixels.argtypes = [P(OrcProblem), fptr, fptr, fptr, ctypes.c_int64,
                                         P(ctypes.c_int32), P(ctypes.c_int32), dptr,
                                         P(OrcStats), ctypes.c_int32]
        L.orc_project_tets.argtypes = [P(OrcProblem), ctypes.c_int64, dptr, dptr, dptr,
                                       P(OrcStats)]
        L.orc_cube_tets.argtypes = [P(OrcProblem), fptr, fptr, fptr, ctypes.c_int64, dptr, dptr]
        for f in (L.orc_project_region, L.orc_project_pixels, L.orc_project_tets,
                  L.orc_cube_tets):
            f.restype = ctypes.c_int
        _lib = L
    return _lib


def _problem(dims: Sequence[int], view: Dict, box=(1.0, 1.0, 1.0), periodic: bool = True,
             total_mass: float = 1.0) -> OrcProblem:
    p = OrcProblem()
    for a in range(3):
        p.dims[a] = int(dims[a])
        p.box[a] = float(box[a])
        p.center[a] = float(view["center"][a])
    for r in range(9):
        p.rot[r] = float(view["rot"][r])
    p.extent[0], p.extent[1] = float(view["extent"][0]), float(view["extent"][1])
    p.periodic = 1 if periodic else 0
    p.total_mass = float(total_mass)
    p.width, p.height = int(view["width"]), int(view["height"])
    p.wrap = 1 if view.get("wrap", 0) else 0
    p.qpow = QUANTITY_POWER[view.get("quantity", "density")]
    slab = view.get("slab")
    p.slab = 1 if slab is not None else 0
    if slab is not None:
        p.slab_t[0], p.slab_t[1] = float(slab[0]), float(slab[1])
    p.perspective = 1 if view.get("projection", "orthographic") == "perspective" else 0
    if p.perspective:  # orthographic centroids go through splat_image / splat_tets
        p.method = {"tessellation": 0, "centroids": 1, "hybrid": 2}[view.get("method", "tessellation")]
        p.lod_radius = float(view.get("lod_radius", 0.0))
    return p


def _f32(a) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with status {rc}")


def default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def project_region(x, y, z, dims, view: Dict, crop: Optional[Tuple[int, int, int, int]] = None,
                   box=(1.0, 1.0, 1.0), periodic: bool = True, total_mass: float = 1.0,
                   nthreads: Optional[int] = None) -> Tuple[np.ndarray, Dict[str, int]]:
    """FP64 image (or crop (x0, y0, w, h) of it), shape (h, w)."""
    x, y, z = _f32(x), _f32(y), _f32(z)
    p = _problem(dims, view, box, periodic, total_mass)
    if crop is None:
        crop = (0, 0, p.width, p.height)
    cx, cy, cw, ch = (int(c) for c in crop)
    out = np.empty((ch, cw), dtype=np.float64)
    st = OrcStats()
    rc = lib().orc_project_region(ctypes.byref(p), _ptr(x, ctypes.c_float), _ptr(y, ctypes.c_float),
                                  _ptr(z, ctypes.c_float), cx, cy, cw, ch,
                                  _ptr(out, ctypes.c_double), ctypes.byref(st),
                                  int(nthreads or default_threads()))
    _check(rc, "project_region")
    return out, st.as_dict()


def project_pixels(x, y, z, dims, view: Dict, px, py, box=(1.0, 1.0, 1.0), periodic: bool = True,
                   total_mass: float = 1.0, nthreads: Optional[int] = None
                   ) -> Tuple[np.ndarray, Dict[str, int]]:
    """FP64 projection at the listed pixels (column px[s], row py[s])."""
    x, y, z = _f32(x), _f32(y), _f32(z)
    px = np.ascontiguousarray(px, dtype=np.int32)
    py = np.ascontiguousarray(py, dtype=np.int32)
    p = _problem(dims, view, box, periodic, total_mass)
    out = np.empty(px.shape[0], dtype=np.float64)
    st = OrcStats()
    rc = lib().orc_project_pixels(ctypes.byref(p), _ptr(x, ctypes.c_float), _ptr(y, ctypes.c_float),
                                  _ptr(z, ctypes.c_float), int(px.shape[0]),
                                  _ptr(px, ctypes.c_int32), _ptr(py, ctypes.c_int32),
                                  _ptr(out, ctypes.c_double), ctypes.byref(st),
                                  int(nthreads or default_threads()))
    _check(rc, "project_pixels")
    return out, st.as_dict()


def splat_image(x, y, z, dims, view: Dict, box=(1.0, 1.0, 1.0), periodic: bool = True,
                total_mass: float = 1.0) -> Tuple[np.ndarray, Dict[str, int]]:
    """Centroid splatting of the lattice (FP64 image)."""
    x, y, z = _f32(x), _f32(y), _f32(z)
    p = _problem(dims, view, box, periodic, total_mass)
    out = np.empty((p.height, p.width), dtype=np.float64)
    st = OrcStats()
    rc = lib().orc_splat_image(ctypes.byref(p), _ptr(x, ctypes.c_float), _ptr(y, ctypes.c_float),
                               _ptr(z, ctypes.c_float), _ptr(out, ctypes.c_double), ctypes.byref(st))
    _check(rc, "splat_image")
    return out, st.as_dict()


def splat_tets(verts, mass, view: Dict) -> Tuple[np.ndarray, Dict[str, int]]:
    """Centroid splats of an explicit tetrahedron list, verts (T, 4, 3), mass (T,)."""
    verts = np.ascontiguousarray(verts, dtype=np.float64).reshape(-1, 4, 3)
    mass = np.ascontiguousarray(np.broadcast_to(np.asarray(mass, dtype=np.float64), (verts.shape[0],)))
    p = _problem((2, 2, 2), view)
    out = np.empty((p.height, p.width), dtype=np.float64)
    st = OrcStats()
    rc = lib().orc_splat_tets(ctypes.byref(p), int(verts.shape[0]), _ptr(verts, ctypes.c_double),
                              _ptr(mass, ctypes.c_double), _ptr(out, ctypes.c_double), ctypes.byref(st))
    _check(rc, "splat_tets")
    return out, st.as_dict()


def project_tets(verts, mass, view: Dict) -> Tuple[np.ndarray, Dict[str, int]]:
    """Projection of an explicit tetrahedron list, verts (T, 4, 3) world, mass (T,)."""
    verts = np.ascontiguousarray(verts, dtype=np.float64).reshape(-1, 4, 3)
    mass = np.ascontiguousarray(np.broadcast_to(np.asarray(mass, dtype=np.float64),
                                                (verts.shape[0],)))
    p = _problem((2, 2, 2), view)
    out = np.empty((p.height, p.width), dtype=np.float64)
    st = OrcStats()
    rc = lib().orc_project_tets(ctypes.byref(p), int(verts.shape[0]), _ptr(verts, ctypes.c_double),
                                _ptr(mass, ctypes.c_double), _ptr(out, ctypes.c_double),
                                ctypes.byref(st))
    _check(rc, "project_tets")
    return out, st.as_dict()


def cube_tets(x, y, z, dims, cube: int, box=(1.0, 1.0, 1.0), periodic: bool = True
              ) -> Tuple[np.ndarray, np.ndarray]:
    """Unwrapped vertices (6, 4, 3) and signed volumes (6,) of one lattice cube."""
    x, y, z = _f32(x), _f32(y), _f32(z)
    from workloads import z_view  # view fields are unused here
    p = _problem(dims, z_view(4), box, periodic)
    verts = np.empty((6, 4, 3), dtype=np.float64)
    vols = np.empty(6, dtype=np.float64)
    rc = lib().orc_cube_tets(ctypes.byref(p), _ptr(x, ctypes.c_float), _ptr(y, ctypes.c_float),
                             _ptr(z, ctypes.c_float), int(cube), _ptr(verts, ctypes.c_double),
                             _ptr(vols, ctypes.c_double))
    _check(rc, "cube_tets")
    return verts, vols

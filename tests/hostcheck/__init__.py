"""Builds and loads the host-compiled run of the kernels' per-tetrahedron code."""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SRC = os.path.join(HERE, "hostcheck.cpp")
HDR = os.path.join(ROOT, "paper_1208_3206_amd", "csrc", "tess_tet.h")
LIB = os.path.join(HERE, "libhostcheck.so")
_lib = None


def build():
    newest = max(os.path.getmtime(SRC), os.path.getmtime(HDR),
                 os.path.getmtime(os.path.join(ROOT, "paper_1208_3206_amd", "csrc", "tess_internal.h")))
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < newest:
        cmd = ["/opt/rocm/bin/hipcc", "-x", "hip", "--offload-arch=gfx950", "-O2", "-std=c++17",
               "-fPIC", "-shared", "-I", os.path.join(ROOT, "paper_1208_3206_amd", "csrc"),
               "-I", os.path.join(ROOT, "include"), SRC, "-o", LIB + ".tmp%x" % os.getpid()]
        # (a file of its own per process: parallel test workers may all
        # rebuild after a header change, and each replaces the library whole)
        subprocess.run(cmd, check=True, capture_output=True)
        os.replace(LIB + ".tmp%x" % os.getpid(), LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = ctypes.CDLL(LIB)
        _lib.hc_pipeline.restype = ctypes.c_int
    return _lib


def pipeline(x, y, z, dims, view, periodic=True, total_mass=1.0, precision=0, tile_rows=8,
             tile_cols=None, chunk=4096, crease_div=None, edges=True):
    """The GPU pipeline's own per-tetrahedron code run on the CPU, in the
    kernels' order of work.  Returns the FP64 image before rounding, the FP32
    image and the counters.  crease_div: footprints steeper than the mean
    pixel value / crease_div per pixel keep the line form (the library uses
    width / 64); 0 puts every footprint in line form.  edges: the library's
    edge form for plain pyramids (False: every crease per tetrahedron;
    "no_counts": the edge form's raster without its fragment count, which is
    then not comparable; "split": as "no_counts", with each pair's first
    tile copy drawn from its edge job, row by row, as the GPU's 16-lane
    groups do, and the rest by the pair routine that skips that copy;
    "general": the edge form with every tetrahedron set up by the general
    code, without the common-case path)."""
    P = ctypes.POINTER
    x, y, z = (np.ascontiguousarray(a, dtype=np.float32) for a in (x, y, z))
    W, H = int(view["width"]), int(view["height"])
    if tile_cols is None:
        tile_cols = W
    if crease_div is None:
        crease_div = W / 64.0
    out64 = np.zeros((H, W), dtype=np.float64)
    out32 = np.zeros((H, W), dtype=np.float32)
    st = np.zeros(10, dtype=np.int64)
    d = (ctypes.c_int32 * 3)(*[int(v) for v in dims])
    rot = (ctypes.c_double * 9)(*[float(v) for v in view["rot"]])
    cen = (ctypes.c_double * 3)(*[float(v) for v in view["center"]])
    ext = (ctypes.c_double * 2)(*[float(v) for v in view["extent"]])
    rc = lib().hc_pipeline(x.ctypes.data_as(P(ctypes.c_float)), y.ctypes.data_as(P(ctypes.c_float)),
                           z.ctypes.data_as(P(ctypes.c_float)), d, int(periodic), ctypes.c_double(total_mass),
                           int(precision), rot, cen, ext, W, H, int(view.get("wrap", 0)), int(tile_rows),
                           int(tile_cols), int(chunk), ctypes.c_double(crease_div),
                           {"unit": 0, "density": 1, "density2": 2}[view.get("quantity", "density")],
                           (ctypes.c_double * 2)(*view["slab"]) if view.get("slab") is not None else None,
                           1 if view.get("method", "tessellation") == "centroids" else 0,
                           1 if view.get("projection", "orthographic") == "perspective" else 0,
                           1 if view.get("method", "tessellation") == "hybrid" else 0,
                           ctypes.c_double(float(view.get("lod_radius", 0.0))),
                           {"no_counts": 2, "split": 3, "general": 4}.get(edges, 1 if edges else 0),
                           out64.ctypes.data_as(P(ctypes.c_double)),
                           out32.ctypes.data_as(P(ctypes.c_float)), st.ctypes.data_as(P(ctypes.c_longlong)))
    if rc != 0:
        raise RuntimeError(f"hostcheck pipeline failed: {rc}")
    keys = ("tets", "zero_volume", "inverted", "fp64_dets", "fragments", "spans", "pairs", "items",
            "crease_records", "edged")
    return out64, out32, dict(zip(keys, (int(v) for v in st)))

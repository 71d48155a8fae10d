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
               "-I", os.path.join(ROOT, "include"), SRC, "-o", LIB + ".tmp"]
        subprocess.run(cmd, check=True, capture_output=True)
        os.replace(LIB + ".tmp", LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = ctypes.CDLL(LIB)
        _lib.hc_project.restype = ctypes.c_int
    return _lib


def project(x, y, z, dims, view, periodic=True, total_mass=1.0, fp64_cond=256.0, tile=32):
    P = ctypes.POINTER
    x, y, z = (np.ascontiguousarray(a, dtype=np.float32) for a in (x, y, z))
    W, H = int(view["width"]), int(view["height"])
    out = np.zeros((H, W), dtype=np.float64)
    st = np.zeros(6, dtype=np.int64)
    d = (ctypes.c_int32 * 3)(*[int(v) for v in dims])
    rot = (ctypes.c_double * 9)(*[float(v) for v in view["rot"]])
    cen = (ctypes.c_double * 3)(*[float(v) for v in view["center"]])
    ext = (ctypes.c_double * 2)(*[float(v) for v in view["extent"]])
    rc = lib().hc_project(x.ctypes.data_as(P(ctypes.c_float)), y.ctypes.data_as(P(ctypes.c_float)),
                          z.ctypes.data_as(P(ctypes.c_float)), d, int(periodic), ctypes.c_double(total_mass),
                          rot, cen, ext, W, H, int(view.get("wrap", 0)), ctypes.c_double(fp64_cond),
                          int(tile), out.ctypes.data_as(P(ctypes.c_double)),
                          st.ctypes.data_as(P(ctypes.c_longlong)))
    if rc != 0:
        raise RuntimeError(f"hostcheck failed: {rc}")
    keys = ("tets", "zero_volume", "inverted", "fp64_tets", "fragments", "culled_but_covered")
    return out, dict(zip(keys, (int(v) for v in st)))


def pipeline(x, y, z, dims, view, periodic=True, total_mass=1.0, fp64_cond=256.0, tile=32, chunk=4096):
    """The GPU pipeline's own code run on the CPU: float32 image and stats."""
    P = ctypes.POINTER
    x, y, z = (np.ascontiguousarray(a, dtype=np.float32) for a in (x, y, z))
    W, H = int(view["width"]), int(view["height"])
    out = np.zeros((H, W), dtype=np.float32)
    st = np.zeros(5, dtype=np.int64)
    d = (ctypes.c_int32 * 3)(*[int(v) for v in dims])
    rot = (ctypes.c_double * 9)(*[float(v) for v in view["rot"]])
    cen = (ctypes.c_double * 3)(*[float(v) for v in view["center"]])
    ext = (ctypes.c_double * 2)(*[float(v) for v in view["extent"]])
    rc = lib().hc_pipeline(x.ctypes.data_as(P(ctypes.c_float)), y.ctypes.data_as(P(ctypes.c_float)),
                           z.ctypes.data_as(P(ctypes.c_float)), d, int(periodic), ctypes.c_double(total_mass),
                           rot, cen, ext, W, H, int(view.get("wrap", 0)), ctypes.c_double(fp64_cond),
                           int(tile), int(chunk), out.ctypes.data_as(P(ctypes.c_float)),
                           st.ctypes.data_as(P(ctypes.c_longlong)))
    if rc != 0:
        raise RuntimeError(f"hostcheck pipeline failed: {rc}")
    keys = ("tets", "fp64_tets", "pairs", "items", "fragments")
    return out, dict(zip(keys, (int(v) for v in st)))

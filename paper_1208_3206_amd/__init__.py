"""Python binding of the MI355X tessellation projector (libtess.so).

Argument marshalling only: every step of the projection runs in the HIP
kernels of ``libtess.so``; this module turns torch tensors into device
pointers and the current torch stream into a HIP stream, and calls the C ABI
declared in ``include/tess.h`` under the same names.  PyTorch is used for
device memory and streams only.

Importing this package loads the compiled library and fails loudly if it is
missing; there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Dict, List, Optional, Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtess.so")

TESS_OK, TESS_EINVAL, TESS_ENOMEM, TESS_EHIP, TESS_ENOTSUP, TESS_ECAPACITY, TESS_ERANGE = (
    0, -1, -2, -3, -4, -5, -6)
PREC_FP32, PREC_FP64 = 0, 1
_STATUS = {0: "TESS_OK", -1: "TESS_EINVAL", -2: "TESS_ENOMEM", -3: "TESS_EHIP",
           -4: "TESS_ENOTSUP", -5: "TESS_ECAPACITY", -6: "TESS_ERANGE"}


class TessBuildDesc(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int32 * 3), ("box", ctypes.c_double * 3),
                ("periodic", ctypes.c_int32), ("total_mass", ctypes.c_double),
                ("precision", ctypes.c_int32), ("det_v0_frac", ctypes.c_double),
                ("det_cond_k", ctypes.c_double), ("copy_positions", ctypes.c_int32)]


class TessView(ctypes.Structure):
    _fields_ = [("rot", ctypes.c_double * 9), ("center", ctypes.c_double * 3),
                ("extent", ctypes.c_double * 2), ("width", ctypes.c_int32),
                ("height", ctypes.c_int32), ("wrap", ctypes.c_int32),
                ("quantity", ctypes.c_int32), ("slab", ctypes.c_int32),
                ("slab_t", ctypes.c_double * 2), ("method", ctypes.c_int32),
                ("projection", ctypes.c_int32), ("lod_radius", ctypes.c_double)]

# tess_method by name (view["method"], default "tessellation")
METHODS = {"tessellation": 0, "centroids": 1, "hybrid": 2}

# tess_projection by name (view["projection"], default "orthographic")
PROJECTIONS = {"orthographic": 0, "perspective": 1}

# tess_quantity by name (view["quantity"], default "density")
QUANTITIES = {"density": 0, "unit": 1, "density2": 2}


class TessTune(ctypes.Structure):
    _fields_ = [("tile_rows", ctypes.c_int32), ("tile_cols", ctypes.c_int32),
                ("chunk", ctypes.c_int32), ("block", ctypes.c_int32),
                ("form", ctypes.c_int32), ("no_counts", ctypes.c_int32),
                ("pair_capacity", ctypes.c_uint64), ("workspace_limit", ctypes.c_uint64),
                ("own_capacity", ctypes.c_uint64)]


# tess_form by name (make_tune(form=...))
FORMS = {"auto": 0, "per_tetrahedron": 1, "edges": 2}


class TessStats(ctypes.Structure):
    _fields_ = [("tets", ctypes.c_uint64), ("zero_volume", ctypes.c_uint64),
                ("inverted", ctypes.c_uint64), ("fp64_dets", ctypes.c_uint64),
                ("degenerate", ctypes.c_uint64), ("fragments", ctypes.c_uint64),
                ("spans", ctypes.c_uint64),
                ("bin_pairs", ctypes.c_uint64), ("max_bin", ctypes.c_uint32),
                ("work_items", ctypes.c_uint32), ("tile_rows", ctypes.c_int32),
                ("tile_cols", ctypes.c_int32), ("chunk", ctypes.c_int32),
                ("block", ctypes.c_int32), ("ms", ctypes.c_float),
                ("setup_ms", ctypes.c_float), ("bin_ms", ctypes.c_float),
                ("raster_ms", ctypes.c_float), ("finalize_ms", ctypes.c_float),
                ("kinks", ctypes.c_uint64), ("overflow", ctypes.c_uint32),
                ("own_records", ctypes.c_uint32)]

    def as_dict(self) -> Dict:
        return {k: (float(getattr(self, k)) if k.endswith("ms") else int(getattr(self, k)))
                for k, _ in self._fields_}


class TessRefineDesc(ctypes.Structure):
    _fields_ = [("r", ctypes.c_int32), ("mode", ctypes.c_int32), ("steps", ctypes.c_int32),
                ("batch", ctypes.c_int32), ("rff_sigma", ctypes.c_double), ("lr0", ctypes.c_double),
                ("lr1", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("rff_B", ctypes.c_void_p), ("weights_in", ctypes.c_void_p),
                ("weights_out", ctypes.c_void_p)]


class TessRefineReport(ctypes.Structure):
    _fields_ = [("loss_first", ctypes.c_double), ("loss_last", ctypes.c_double),
                ("train_ms", ctypes.c_float), ("infer_ms", ctypes.c_float),
                ("fine_tracers", ctypes.c_int64)]

    def as_dict(self) -> Dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


MLP_PARAMS = 66435
MLP_FREQS = 64
REFINE_LINEAR, REFINE_MLP, REFINE_MLP_RAW = 0, 1, 2


class TessError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {_STATUS.get(status, status)}: {msg}")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build the HIP library first "
            "(python -c 'import __graft_entry__ as g; g.build()')")
    # torch ships its own HIP runtime; load it first so that the library binds
    # to the same one (two runtimes in one process do not share the device)
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    L.tess_build_desc_default.argtypes = [P(TessBuildDesc)]
    L.tess_build.argtypes = [P(TessBuildDesc), vp, vp, vp, vp, vp, P(vp)]
    L.tess_free.argtypes = [vp]
    L.tess_free.restype = None
    L.tess_project.argtypes = [vp, P(TessView), P(TessTune), vp, P(TessStats), vp]
    L.tess_project_batch.argtypes = [P(vp), ctypes.c_int32, P(TessView), ctypes.c_int32,
                                     P(TessTune), vp, P(TessStats), vp]
    L.tess_check_view.argtypes = [P(TessView), P(TessBuildDesc)]
    L.tess_check_build_desc.argtypes = [P(TessBuildDesc)]
    L.tess_refine_desc_default.argtypes = [P(TessRefineDesc)]
    L.tess_refine.argtypes = [vp, P(TessRefineDesc), P(vp), P(TessRefineReport), vp]
    L.tess_mlp_loss_grad.argtypes = [vp, vp, vp, vp, ctypes.c_int64, P(ctypes.c_double), vp, vp, vp]
    L.tess_mlp_adam.argtypes = [vp, vp, vp, vp, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                ctypes.c_double, ctypes.c_double, vp]
    L.tess_lattice_positions.argtypes = [vp, vp, vp, vp, vp]
    L.tess_mlp_forward.argtypes = [vp, vp, vp, ctypes.c_int64, vp, vp]
    L.tess_project_noalloc.argtypes = [vp, P(TessView), P(TessTune), vp, vp]
    L.tess_last_error.argtypes = []
    L.tess_last_error.restype = ctypes.c_char_p
    L.tess_version.argtypes = []
    L.tess_version.restype = ctypes.c_int32
    L.tess_struct_size.argtypes = [ctypes.c_int32]
    L.tess_struct_size.restype = ctypes.c_uint64
    for f in (L.tess_build_desc_default, L.tess_build, L.tess_project, L.tess_project_batch,
              L.tess_check_view, L.tess_check_build_desc, L.tess_refine_desc_default,
              L.tess_refine, L.tess_mlp_loss_grad, L.tess_mlp_adam, L.tess_lattice_positions,
              L.tess_project_noalloc, L.tess_mlp_forward):
        f.restype = ctypes.c_int
    return L


_lib = _load()

# names exported by the C ABI (checked against include/tess.h by the tests)
EXPORTS = ("tess_build_desc_default", "tess_build", "tess_free", "tess_project",
           "tess_project_batch", "tess_check_view", "tess_check_build_desc",
           "tess_last_error", "tess_version", "tess_struct_size", "tess_refine_desc_default", "tess_refine",
           "tess_mlp_loss_grad", "tess_mlp_adam", "tess_lattice_positions", "tess_project_noalloc",
           "tess_mlp_forward")


def lib():
    return _lib


def last_error() -> str:
    return _lib.tess_last_error().decode()


def version() -> int:
    return int(_lib.tess_version())


def _check(rc: int, where: str):
    if rc != TESS_OK:
        raise TessError(rc, where, last_error())


# ------------------------------------------------------------ descriptors
def build_desc(dims: Sequence[int], box=(1.0, 1.0, 1.0), periodic: bool = True,
               total_mass: float = 1.0, precision: str = "fp32", det_v0_frac: float = 1e-6,
               det_cond_k: float = 1e3, copy_positions: bool = False) -> TessBuildDesc:
    d = TessBuildDesc()
    _check(_lib.tess_build_desc_default(ctypes.byref(d)), "tess_build_desc_default")
    for a in range(3):
        d.dims[a] = int(dims[a])
        d.box[a] = float(box[a])
    d.periodic = 1 if periodic else 0
    d.total_mass = float(total_mass)
    d.precision = {"fp32": PREC_FP32, "fp64": PREC_FP64}[precision]
    d.det_v0_frac = float(det_v0_frac)
    d.det_cond_k = float(det_cond_k)
    d.copy_positions = 1 if copy_positions else 0
    return d


def make_view(view: Dict) -> TessView:
    """Converts a view dict (rot, center, extent, width, height, wrap, optional
    quantity: "density", "unit" or "density2", optional slab: (t0, t1),
    optional method: "tessellation", "centroids" or "hybrid" (with
    lod_radius), optional projection: "orthographic" or "perspective", with
    center the camera) to the C struct."""
    v = TessView()
    for i in range(9):
        v.rot[i] = float(view["rot"][i])
    for i in range(3):
        v.center[i] = float(view["center"][i])
    v.extent[0], v.extent[1] = float(view["extent"][0]), float(view["extent"][1])
    v.width, v.height = int(view["width"]), int(view["height"])
    v.wrap = 1 if view.get("wrap", 0) else 0
    v.quantity = QUANTITIES[view.get("quantity", "density")]
    slab = view.get("slab")
    v.slab = 1 if slab is not None else 0
    if slab is not None:
        v.slab_t[0], v.slab_t[1] = float(slab[0]), float(slab[1])
    v.method = METHODS[view.get("method", "tessellation")]
    v.projection = PROJECTIONS[view.get("projection", "orthographic")]
    v.lod_radius = float(view.get("lod_radius", 0.0))
    return v


def make_tune(tile_rows: int = 0, tile_cols: int = 0, chunk: int = 0, block: int = 0,
              form: str = "auto", pair_capacity: int = 0, counts: bool = True,
              workspace_limit: int = 0, own_capacity: int = 0) -> TessTune:
    """Raster parameters; 0 (and form "auto") means automatic.  counts=False:
    calls with stats skip the edge form's fragment count (timings only)."""
    t = TessTune()
    t.tile_rows, t.tile_cols, t.chunk, t.block = int(tile_rows), int(tile_cols), int(chunk), int(block)
    t.form = FORMS[form]
    t.no_counts = 0 if counts else 1
    t.pair_capacity = int(pair_capacity)
    t.workspace_limit = int(workspace_limit)
    t.own_capacity = int(own_capacity)
    return t


def check_view(view: Dict, desc: Optional[TessBuildDesc] = None):
    """Host-only validation of a view (no GPU needed); raises TessError."""
    v = make_view(view)
    _check(_lib.tess_check_view(ctypes.byref(v), ctypes.byref(desc) if desc is not None else None),
           "tess_check_view")


def check_build_desc(desc: TessBuildDesc):
    _check(_lib.tess_check_build_desc(ctypes.byref(desc)), "tess_check_build_desc")


# ---------------------------------------------------------------- handles
def _stream_handle(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _dev_f32(t, n: int, name: str):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32
            and t.is_contiguous() and t.numel() == n):
        raise ValueError(f"{name} must be a contiguous CUDA float32 tensor of {n} elements")
    return t


class Lattice:
    """A lattice handle (tess_build).  Keeps the position tensors alive."""

    def __init__(self, x, y, z, dims: Sequence[int], ids=None, stream=None, **desc_kw):
        import torch
        self.desc = build_desc(dims, **desc_kw)
        n = int(dims[0]) * int(dims[1]) * int(dims[2])
        self._tensors = [_dev_f32(x, n, "x"), _dev_f32(y, n, "y"), _dev_f32(z, n, "z")]
        if ids is not None:
            if not (isinstance(ids, torch.Tensor) and ids.is_cuda and ids.dtype == torch.int64
                    and ids.is_contiguous() and ids.numel() == n):
                raise ValueError("ids must be a contiguous CUDA int64 tensor")
            self._tensors.append(ids)
        h = ctypes.c_void_p()
        rc = _lib.tess_build(ctypes.byref(self.desc), x.data_ptr(), y.data_ptr(), z.data_ptr(),
                             ids.data_ptr() if ids is not None else None, _stream_handle(stream),
                             ctypes.byref(h))
        _check(rc, "tess_build")
        self.handle = h
        self.dims = tuple(int(d) for d in dims)

    def positions(self, stream=None):
        """Copies of the handle's positions (x, y, z CUDA float32 tensors, tracer-id order)."""
        import torch
        n = int(self.dims[0]) * int(self.dims[1]) * int(self.dims[2])
        out = [torch.empty(n, dtype=torch.float32, device="cuda") for _ in range(3)]
        _check(_lib.tess_lattice_positions(self.handle, out[0].data_ptr(), out[1].data_ptr(), out[2].data_ptr(),
                                           _stream_handle(stream)), "tess_lattice_positions")
        return out

    def free(self):
        if getattr(self, "handle", None):
            _lib.tess_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def build(x, y, z, dims: Sequence[int], ids=None, stream=None, **desc_kw) -> Lattice:
    return Lattice(x, y, z, dims, ids=ids, stream=stream, **desc_kw)


def project(lat: Lattice, view: Dict, out=None, tune: Optional[TessTune] = None,
            stats: bool = False, stream=None):
    """Column-density image (float32 CUDA tensor [H, W]); with stats, also a dict."""
    import torch
    v = make_view(view)
    if out is None:
        out = torch.empty((v.height, v.width), dtype=torch.float32, device="cuda")
    if not (out.is_cuda and out.dtype == torch.float32 and out.is_contiguous()
            and out.numel() == v.width * v.height):
        raise ValueError("out must be a contiguous CUDA float32 tensor of height*width elements")
    st = TessStats()
    rc = _lib.tess_project(lat.handle, ctypes.byref(v), ctypes.byref(tune) if tune is not None else None,
                           out.data_ptr(), ctypes.byref(st) if stats else None, _stream_handle(stream))
    _check(rc, "tess_project")
    return (out, st.as_dict()) if stats else out


def project_noalloc(lat: Lattice, view: Dict, out, tune: Optional[TessTune] = None, stream=None):
    """tess_project_noalloc into `out` (float32 CUDA tensor [H, W]); allocates nothing."""
    v = make_view(view)
    if not (out.is_cuda and out.dtype.itemsize == 4 and out.is_floating_point() and out.is_contiguous()
            and out.numel() == v.width * v.height):
        raise ValueError("out must be a contiguous CUDA float32 tensor of height*width elements")
    _check(_lib.tess_project_noalloc(lat.handle, ctypes.byref(v), ctypes.byref(tune) if tune is not None else None,
                                     out.data_ptr(), _stream_handle(stream)), "tess_project_noalloc")
    return out


def project_batch(lats: List[Lattice], views: List[Dict], out=None, tune: Optional[TessTune] = None,
                  stats: bool = False, stream=None):
    """Images [n_snaps, n_views, H, W] of every (snapshot, view) pair."""
    import torch
    vs = (TessView * len(views))(*[make_view(v) for v in views])
    hs = (ctypes.c_void_p * len(lats))(*[l.handle for l in lats])
    H, W = vs[0].height, vs[0].width
    if out is None:
        out = torch.empty((len(lats), len(views), H, W), dtype=torch.float32, device="cuda")
    if not (out.is_cuda and out.dtype == torch.float32 and out.is_contiguous()
            and out.numel() == len(lats) * len(views) * H * W):
        raise ValueError("out has the wrong shape or type")
    st = TessStats()
    rc = _lib.tess_project_batch(hs, len(lats), vs, len(views),
                                 ctypes.byref(tune) if tune is not None else None, out.data_ptr(),
                                 ctypes.byref(st) if stats else None, _stream_handle(stream))
    _check(rc, "tess_project_batch")
    return (out, st.as_dict()) if stats else out


# ------------------------------------------------------------- refinement
class _Owned(Lattice):
    """A lattice handle whose positions the library owns (from tess_refine)."""

    def __init__(self, handle, dims):  # noqa: D401 - plain holder
        self.handle = handle
        self.dims = tuple(dims)
        self._tensors = []


def refine(lat: Lattice, r: int = 4, mode: str = "mlp", steps: int = 10000, batch: int = 8192,
           rff_sigma: float = 8.0, lr0: float = 1e-2, lr1: float = 1e-5, seed: int = 2,
           rff_B=None, weights_in=None, want_weights: bool = False, stream=None):
    """Refined lattice (tess_refine); returns (lattice, report dict[, weights])."""
    import numpy as np
    d = TessRefineDesc()
    _check(_lib.tess_refine_desc_default(ctypes.byref(d)), "tess_refine_desc_default")
    d.r, d.steps, d.batch = int(r), int(steps), int(batch)
    d.mode = {"linear": REFINE_LINEAR, "mlp": REFINE_MLP, "mlp_raw": REFINE_MLP_RAW}[mode]
    d.rff_sigma, d.lr0, d.lr1, d.seed = float(rff_sigma), float(lr0), float(lr1), int(seed)
    keep = []
    if rff_B is not None:
        b = np.ascontiguousarray(rff_B, dtype=np.float32).reshape(-1)
        keep.append(b)
        d.rff_B = b.ctypes.data
    if weights_in is not None:
        w = np.ascontiguousarray(weights_in, dtype=np.float32).reshape(-1)
        keep.append(w)
        d.weights_in = w.ctypes.data
    wout = np.empty(MLP_PARAMS, dtype=np.float32) if want_weights else None
    if wout is not None:
        d.weights_out = wout.ctypes.data
    h = ctypes.c_void_p()
    rep = TessRefineReport()
    _check(_lib.tess_refine(lat.handle, ctypes.byref(d), ctypes.byref(h), ctypes.byref(rep),
                            _stream_handle(stream)), "tess_refine")
    fine = _Owned(h, tuple(int(x) * int(r) for x in lat.dims))
    return (fine, rep.as_dict(), wout) if want_weights else (fine, rep.as_dict())


def mlp_loss_grad(params, rff_B, q, target, want_pred: bool = False, stream=None):
    """(loss, grad[, pred]) of the network for device tensors q, target (n x 3)."""
    import numpy as np
    import torch
    p = np.ascontiguousarray(params, dtype=np.float32).reshape(-1)
    b = np.ascontiguousarray(rff_B, dtype=np.float32).reshape(-1)
    if p.size != MLP_PARAMS or b.size != 3 * MLP_FREQS:
        raise ValueError("params / rff_B have the wrong size")
    n = q.shape[0]
    for t in (q, target):
        if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and t.numel() == 3 * n):
            raise ValueError("q and target must be contiguous CUDA float32 (n, 3)")
    grad = np.empty(MLP_PARAMS, dtype=np.float32)
    pred = torch.empty((n, 3), dtype=torch.float32, device=q.device) if want_pred else None
    loss = ctypes.c_double()
    _check(_lib.tess_mlp_loss_grad(p.ctypes.data, b.ctypes.data, q.data_ptr(), target.data_ptr(),
                                   int(n), ctypes.byref(loss), grad.ctypes.data,
                                   pred.data_ptr() if pred is not None else None,
                                   _stream_handle(stream)), "tess_mlp_loss_grad")
    return (loss.value, grad, pred) if want_pred else (loss.value, grad)


def mlp_forward(params, rff_B, q, stream=None):
    """The network's predictions (n, 3) for q (contiguous CUDA float32 (n, 3)),
    by the fused inference kernel tess_refine uses."""
    import numpy as np
    import torch
    p = np.ascontiguousarray(params, dtype=np.float32).reshape(-1)
    b = np.ascontiguousarray(rff_B, dtype=np.float32).reshape(-1)
    if p.size != MLP_PARAMS or b.size != 3 * MLP_FREQS:
        raise ValueError("params / rff_B have the wrong size")
    n = q.shape[0]
    if not (q.is_cuda and q.dtype == torch.float32 and q.is_contiguous() and q.numel() == 3 * n):
        raise ValueError("q must be a contiguous CUDA float32 (n, 3) tensor")
    pred = torch.empty((n, 3), dtype=torch.float32, device=q.device)
    _check(_lib.tess_mlp_forward(p.ctypes.data, b.ctypes.data, q.data_ptr(), int(n), pred.data_ptr(),
                                 _stream_handle(stream)), "tess_mlp_forward")
    return pred


def mlp_adam(params, m, v, grad, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
             eps: float = 1e-8, stream=None):
    """One Adam update by the library's kernel; returns new (params, m, v) as FP32 arrays."""
    import numpy as np
    arrs = [np.array(a, dtype=np.float32).reshape(-1) for a in (params, m, v, grad)]
    if any(a.size != MLP_PARAMS for a in arrs):
        raise ValueError("params, m, v and grad need MLP_PARAMS entries each")
    p, mm, vv, g = arrs
    _check(_lib.tess_mlp_adam(p.ctypes.data, mm.ctypes.data, vv.ctypes.data, g.ctypes.data, int(step),
                              float(lr), float(beta1), float(beta2), float(eps), _stream_handle(stream)),
           "tess_mlp_adam")
    return p, mm, vv

"""Seeded synthetic inputs for the tessellation projector.

This module only *makes inputs*: Zel'dovich particle lattices, view
descriptions and random rotations.  It holds none of the projection's
arithmetic and is imported by the oracle tests, the GPU tests and the
benchmark alike, so both sides of every parity check see byte-identical
FP32 positions.

Field recipe (the paper's simulations are not available; these stand in for
them):

* Lagrangian lattice q = (i, j, k) * L / N, tracer id = i + N (j + N k)
  (the id <-> lattice map of the data-storage section, Eq. ``Eqn:ID``).
* Gaussian random potential phi with integer modes 1 <= |k| <= kmax,
  amplitude |k|^-1 (power P(k) ~ k^-2), complex normal coefficients drawn
  from ``numpy.random.default_rng(seed)`` over the canonical half space in
  lexicographic (kx, ky, kz) order; the other half is the complex conjugate.
  The draw order depends only on kmax, so the same analytic field can be
  sampled on lattices of any size N > 2 kmax.
* Displacement psi = -grad phi, i.e. psi_hat(k) = -2 pi i k phi_hat(k),
  scaled so that the rms of |psi| over the torus is 0.02 (computed exactly
  from the coefficients by Parseval).
* Positions x = q + D psi(q), wrapped into [0, L), computed in FP64 and
  rounded once to FP32.  The FP32 arrays are the input for every consumer.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

FIELD_SEED = 12083206
VIEW_SEED = 1
MLP_INIT_SEED = 2
MINIBATCH_SEED = 3
RMS_PSI = 0.02


# --------------------------------------------------------------------------
# workload configurations (the five synthetic workloads)
# --------------------------------------------------------------------------
@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    n: int            # particles per axis
    kmax: int         # highest mode |k|
    growth: Tuple[float, ...]   # displacement amplitudes D (one per snapshot)
    width: int
    height: int
    n_views: int = 1  # 1: z-projection with wrap; >1: seeded random rotations
    camera: Optional[Tuple[float, float, float]] = None  # perspective camera (looking along +z)

    @property
    def tets(self) -> int:
        return 6 * self.n ** 3


TINY = Workload("tiny_32^3_to_256^2", 32, 8, (3.0,), 256, 256)
MID = Workload("mid_128^3_to_1024^2", 128, 32, (5.0,), 1024, 1024)
STRESS = Workload("stress_256^3_to_2048^2", 256, 64, (8.0,), 2048, 2048)
STRESS_4K = Workload("stress_256^3_to_4096^2", 256, 64, (8.0,), 4096, 4096)
BATCHED = Workload("batched_128^3_8x64_to_512^2", 128, 32,
                   tuple(float(d) for d in range(1, 9)), 512, 512, n_views=64)
LEARNED = Workload("learned_64^3_D5_to_2048^2", 64, 16, (5.0,), 2048, 2048)
LEARNED_REF = Workload("learned_ref_256^3_D5_to_2048^2", 256, 16, (5.0,), 2048, 2048)
# resampling: the mid field into 128 depth slabs of 128^2 (a 128^3 grid)
RESAMPLE = Workload("resample_128^3_to_128^3", 128, 32, (5.0,), 128, 128)

# perspective: the mid field seen by a camera inside the volume, 90 degrees wide
PERSPECTIVE = Workload("perspective_128^3_inside_to_1024^2", 128, 32, (5.0,), 1024, 1024,
                       camera=(0.5, 0.5, 0.05))

ALL = {w.name: w for w in (TINY, MID, STRESS, STRESS_4K, BATCHED, LEARNED, LEARNED_REF, RESAMPLE,
                           PERSPECTIVE)}


# --------------------------------------------------------------------------
# Gaussian random field
# --------------------------------------------------------------------------
def half_space_modes(kmax: int) -> np.ndarray:
    """Integer modes with 1 <= |k| <= kmax in the canonical half space.

    Half space: kz > 0, or kz == 0 and ky > 0, or kz == ky == 0 and kx > 0.
    Returned in lexicographic (kx, ky, kz) order, shape (M, 3), int64.
    """
    r = np.arange(-kmax, kmax + 1)
    kx, ky, kz = np.meshgrid(r, r, r, indexing="ij")
    kx, ky, kz = kx.ravel(), ky.ravel(), kz.ravel()
    k2 = kx * kx + ky * ky + kz * kz
    half = (kz > 0) | ((kz == 0) & (ky > 0)) | ((kz == 0) & (ky == 0) & (kx > 0))
    keep = half & (k2 >= 1) & (k2 <= kmax * kmax)
    return np.stack([kx[keep], ky[keep], kz[keep]], axis=1).astype(np.int64)


def psi_coefficients(kmax: int, seed: int = FIELD_SEED) -> Tuple[np.ndarray, np.ndarray]:
    """Fourier coefficients of the displacement on the half space.

    Returns (modes (M,3) int64, psi_hat (M,3) complex128), normalised so the
    rms of |psi| over the unit torus is ``RMS_PSI``.  psi(q) =
    sum_half 2 Re(psi_hat_k exp(2 pi i k.q)).
    """
    modes = half_space_modes(kmax)
    rng = np.random.default_rng(seed)
    draws = rng.standard_normal((modes.shape[0], 2))
    c = (draws[:, 0] + 1j * draws[:, 1]) / math.sqrt(2.0)
    kn = np.sqrt((modes.astype(np.float64) ** 2).sum(axis=1))
    phi_hat = c / kn
    psi_hat = (-2j * math.pi) * modes.astype(np.float64) * phi_hat[:, None]
    # mean |psi|^2 = sum over all modes (both halves) of |psi_hat|^2
    ms = 2.0 * float((np.abs(psi_hat) ** 2).sum())
    psi_hat *= RMS_PSI / math.sqrt(ms)
    return modes, psi_hat


def displacement_grid(n: int, kmax: int, seed: int = FIELD_SEED) -> np.ndarray:
    """psi sampled at the lattice q = (i, j, k)/n of the unit torus.

    Exact for a band-limited field with kmax < n/2 (inverse DFT).  Returns
    (3, n, n, n) float64 indexed [component, k, j, i] (z slowest), so that a
    C-order ravel of one component is in tracer-id order.
    """
    if 2 * kmax >= n:
        raise ValueError("lattice too coarse for the field: need n > 2*kmax")
    modes, psi_hat = psi_coefficients(kmax, seed)
    out = np.empty((3, n, n, n), dtype=np.float64)
    iz = modes[:, 2] % n
    iy = modes[:, 1] % n
    ix = modes[:, 0] % n
    jz, jy, jx = (-modes[:, 2]) % n, (-modes[:, 1]) % n, (-modes[:, 0]) % n
    for comp in range(3):
        spec = np.zeros((n, n, n), dtype=np.complex128)
        spec[iz, iy, ix] = psi_hat[:, comp]
        spec[jz, jy, jx] = np.conj(psi_hat[:, comp])
        out[comp] = np.fft.ifftn(spec).real * (n ** 3)
        del spec
    return out


def displacement_at(points: np.ndarray, kmax: int, seed: int = FIELD_SEED) -> np.ndarray:
    """psi at arbitrary points of the unit torus by direct summation.

    points: (P, 3) float64 in units of the box.  Returns (P, 3) float64.
    Slow (P x M); meant for small point sets and for checking the grid path.
    """
    modes, psi_hat = psi_coefficients(kmax, seed)
    pts = np.asarray(points, dtype=np.float64)
    out = np.zeros((pts.shape[0], 3), dtype=np.float64)
    step = 4096
    kf = modes.astype(np.float64)
    for s in range(0, pts.shape[0], step):
        ph = np.exp(2j * math.pi * (pts[s:s + step] @ kf.T))   # (p, M)
        out[s:s + step] = 2.0 * (ph @ psi_hat).real
    return out


def lattice_q(n: int, box: float = 1.0) -> np.ndarray:
    """Lagrangian coordinates in tracer-id order, shape (n^3, 3) float64."""
    r = np.arange(n, dtype=np.float64) * (box / n)
    qz, qy, qx = np.meshgrid(r, r, r, indexing="ij")
    return np.stack([qx.ravel(), qy.ravel(), qz.ravel()], axis=1)


def wrap_to_f32(x64: np.ndarray, box: float) -> np.ndarray:
    """Wrap FP64 coordinates into [0, box) and round once to FP32."""
    w = np.mod(x64, box)
    f = w.astype(np.float32)
    f[f >= np.float32(box)] -= np.float32(box)
    f[f < 0] = 0.0
    return f


def zeldovich(n: int, kmax: int, growth: float, seed: int = FIELD_SEED,
              box: float = 1.0, psi: np.ndarray | None = None
              ) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """FP32 SoA positions (x, y, z) of the Zel'dovich lattice, tracer-id order."""
    if psi is None:
        psi = displacement_grid(n, kmax, seed)
    r = np.arange(n, dtype=np.float64) * (box / n)
    out = []
    for comp in range(3):
        shape = [1, 1, 1]
        shape[2 - comp] = n          # axis 2 is i (x), axis 1 j (y), axis 0 k (z)
        q = r.reshape(shape)
        x64 = q + growth * box * psi[comp]
        out.append(np.ascontiguousarray(wrap_to_f32(x64, box).ravel()))
    return out[0], out[1], out[2]


def undisplaced(n: int, box: float = 1.0) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    q = lattice_q(n, box)
    return tuple(np.ascontiguousarray(q[:, c].astype(np.float32)) for c in range(3))


def random_lattice(n: int, amp: float, seed: int, box: float = 1.0
                   ) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Lattice with i.i.d. uniform jitter of +-amp (in box units) per coordinate."""
    rng = np.random.default_rng(seed)
    q = lattice_q(n, box)
    x = q + rng.uniform(-amp, amp, size=q.shape) * box
    return tuple(np.ascontiguousarray(wrap_to_f32(x[:, c], box)) for c in range(3))


# --------------------------------------------------------------------------
# views
# --------------------------------------------------------------------------
def quaternion_rotation(qv: Sequence[float]) -> np.ndarray:
    """Rotation matrix of a (not necessarily unit) quaternion (w, x, y, z)."""
    w, x, y, z = (float(t) for t in qv)
    s = math.sqrt(w * w + x * x + y * y + z * z)
    w, x, y, z = w / s, x / s, y / s, z / s
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ], dtype=np.float64)


def random_rotations(count: int, seed: int = VIEW_SEED) -> np.ndarray:
    """Haar-uniform rotations from normalised Gaussian quaternions (Shoemake)."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((count, 4))
    return np.stack([quaternion_rotation(row) for row in g])


def z_view(width: int, height: int | None = None, box: float = 1.0) -> Dict:
    """Orthographic projection along z over the whole periodic box, wrapped."""
    height = width if height is None else height
    return dict(rot=np.eye(3).ravel().tolist(), center=[box / 2] * 3,
                extent=[box, box], width=int(width), height=int(height), wrap=1)


def perspective_view(rot: np.ndarray, camera, width: int, height: int | None = None,
                     extent=(1.0, 1.0)) -> Dict:
    """Perspective view: a camera at ``camera`` with axes = rows of ``rot``
    (screen u, screen v, view direction); ``extent`` is the window on the plane
    at unit distance along the view direction."""
    height = width if height is None else height
    return dict(rot=np.asarray(rot, dtype=np.float64).ravel().tolist(),
                center=[float(c) for c in camera], extent=[float(extent[0]), float(extent[1])],
                width=int(width), height=int(height), wrap=0, projection="perspective")


def rotated_view(rot: np.ndarray, width: int, height: int | None = None,
                 side: float = 2.0, center=(0.5, 0.5, 0.5)) -> Dict:
    """Orthographic view with rows of ``rot`` = (screen u, screen v, depth)."""
    height = width if height is None else height
    return dict(rot=np.asarray(rot, dtype=np.float64).ravel().tolist(),
                center=[float(c) for c in center], extent=[side, side],
                width=int(width), height=int(height), wrap=0)


def slab_views(width: int, slabs: int, box: float = 1.0) -> List[Dict]:
    """z-views of `slabs` equal depth slabs over the box, t = z - box/2 in
    [-box/2, box/2), plus one slab below and one above (cubes are unwrapped
    from their corner 0, so some reach past the box in z)."""
    cuts = np.linspace(-0.5 * box, 0.5 * box, slabs + 1)
    edges = [(-1.5 * box, cuts[0])] + list(zip(cuts[:-1], cuts[1:])) + [(cuts[-1], 1.5 * box)]
    return [dict(z_view(width, width, box), slab=(float(a), float(b))) for a, b in edges]


def workload_views(w: Workload) -> List[Dict]:
    if w.camera is not None:
        return [perspective_view(np.eye(3), w.camera, w.width, w.height, extent=(2.0, 2.0))]
    if w.n_views == 1:
        return [z_view(w.width, w.height)]
    return [rotated_view(r, w.width, w.height) for r in random_rotations(w.n_views)]


# --------------------------------------------------------------------------
# refinement network inputs (random draws only)
# --------------------------------------------------------------------------
NET_WIDTH, NET_FREQ, NET_DEPTH = 128, 64, 4


def rff_frequencies(sigma: float, seed: int) -> np.ndarray:
    """(64, 3) N(0, sigma^2) draws rounded to integers, float32."""
    rng = np.random.default_rng(seed)
    return np.rint(rng.normal(0.0, sigma, size=(NET_FREQ, 3))).astype(np.float32)


def network_params(seed: int, out_scale: float = 1.0) -> np.ndarray:
    """Flat FP32 parameters W1, b1, ..., W4, b4, W5, b5 (rows = outputs),
    uniform in +-1/sqrt(fan_in); the output layer's scaled by out_scale."""
    rng = np.random.default_rng(seed)
    parts = []
    dims = [(NET_WIDTH, 2 * NET_FREQ)] + [(NET_WIDTH, NET_WIDTH)] * (NET_DEPTH - 1) + [(3, NET_WIDTH)]
    for i, (o, n) in enumerate(dims):
        k = 1.0 / math.sqrt(n) * (out_scale if i == NET_DEPTH else 1.0)
        parts.append(rng.uniform(-k, k, size=o * n))
        parts.append(rng.uniform(-k, k, size=o))
    return np.concatenate(parts).astype(np.float32)

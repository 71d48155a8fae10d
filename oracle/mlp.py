"""FP64 CPU oracle of the refinement network (test infrastructure only).

The network maps a Lagrangian coordinate q (unit torus) to the displacement
s(q) = x(q) - q of the lattice, to place the vertices of subdivided
tetrahedra.  Layers, in order:

  g  = [sin(2 pi B q), cos(2 pi B q)]     random Fourier features, B (64, 3) integer
  h1 = GELU(W1 g  + b1)                    128 -> 128
  h2 = GELU(W2 h1 + b2)
  h3 = GELU(W3 h2 + b3)
  h4 = GELU(W4 h3 + b4)
  s' = W5 h4 + b5                          128 -> 3
  L  = mean over samples of |s' - s|^2

GELU is the exact one, x * Phi(x).  The backward pass is written out by hand
layer by layer, and Adam (Kingma & Ba) updates the parameters.  Only the test
suite and the benchmark's CPU leg use this module; the GPU library has its own
kernels and shares nothing with it.

Precision.  Everything is FP64.  The network's products are specified with
bf16 operands and wide accumulation, so ``forward(..., operands="bf16")``
rounds exactly the operands of the products to bf16 (the features, the five
weight matrices and the hidden activations that feed the next product) and
still accumulates in FP64; the biases stay as given.

Placement of the refined lattice (r-fold sub-lattice of an N^3 lattice):
fine tracer (I, J, K) has the Lagrangian point q = (I, J, K) / (r N); the
coarse tracers (all of I, J, K multiples of r) keep their positions; the
others get
  raw:    x = (q + s(q)) L, wrapped into [0, L);
  hybrid: x = (q + s(q)) L + sum_m lambda_m e_m, wrapped, where lambda are
          q's barycentric coordinates in the table tetrahedron of its coarse
          cube that contains it and e_m = x_m - (q_m + s(q_m)) L (periodic
          image in (-L/2, L/2]) the network's residual at that tetrahedron's
          corners m.
"""
from __future__ import annotations

import math
from typing import Dict, List, Tuple

import numpy as np
from scipy.special import erf

WIDTH = 128
N_FREQ = 64
DEPTH = 4
NAMES = ["W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4", "W5", "b5"]


def rff_matrix(sigma: float, seed: int) -> np.ndarray:
    """B (64, 3): N(0, sigma^2) draws rounded to integers (exactly periodic features)."""
    rng = np.random.default_rng(seed)
    return np.rint(rng.normal(0.0, sigma, size=(N_FREQ, 3)))


def init_params(seed: int) -> Dict[str, np.ndarray]:
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights and biases (FP64)."""
    rng = np.random.default_rng(seed)
    p = {}
    dims = [(WIDTH, 2 * N_FREQ)] + [(WIDTH, WIDTH)] * (DEPTH - 1) + [(3, WIDTH)]
    for i, (o, n) in enumerate(dims, start=1):
        k = 1.0 / math.sqrt(n)
        p[f"W{i}"] = rng.uniform(-k, k, size=(o, n))
        p[f"b{i}"] = rng.uniform(-k, k, size=(o,))
    return p


def bf16_round(a) -> np.ndarray:
    """Nearest bf16 value of every entry (ties to even), returned as FP64.

    The entry is held as FP32 first (the precision the network's kernels
    compute in), then its FP32 bit pattern is cut to the upper 16 bits with
    round-half-to-even on the 16 dropped bits."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def features(q: np.ndarray, B: np.ndarray) -> np.ndarray:
    a = 2.0 * math.pi * (q @ B.T)            # (N, 64)
    return np.concatenate([np.sin(a), np.cos(a)], axis=1)


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    cdf = 0.5 * (1.0 + erf(x / math.sqrt(2.0)))
    pdf = np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)
    return cdf + x * pdf


def forward(p: Dict[str, np.ndarray], q: np.ndarray, B: np.ndarray, operands: str = "fp64"):
    """Returns the prediction (N, 3) and the cache for backward.

    operands="bf16": the hidden products take bf16-rounded operands (see the
    module header); the cache then holds the rounded activations."""
    rnd = bf16_round if operands == "bf16" else (lambda a: a)
    g = rnd(features(q, B))
    hs, zs = [g], []
    h = g
    for i in range(1, DEPTH + 1):
        z = h @ rnd(p[f"W{i}"]).T + p[f"b{i}"]
        zs.append(z)
        h = rnd(gelu(z))
        hs.append(h)
    out = h @ rnd(p["W5"]).T + p["b5"]
    return out, (hs, zs)


def loss(pred: np.ndarray, target: np.ndarray) -> float:
    return float(((pred - target) ** 2).sum(axis=1).mean())


def backward(p, cache, pred, target) -> Dict[str, np.ndarray]:
    hs, zs = cache
    n = pred.shape[0]
    d = 2.0 * (pred - target) / n           # dL/dpred
    g = {"W5": d.T @ hs[DEPTH], "b5": d.sum(axis=0)}
    dh = d @ p["W5"]
    for i in range(DEPTH, 0, -1):
        dz = dh * gelu_grad(zs[i - 1])
        g[f"W{i}"] = dz.T @ hs[i - 1]
        g[f"b{i}"] = dz.sum(axis=0)
        dh = dz @ p[f"W{i}"]
    return g


def loss_and_grad(p, q, target, B) -> Tuple[float, Dict[str, np.ndarray]]:
    pred, cache = forward(p, q, B)
    return loss(pred, target), backward(p, cache, pred, target)


def adam_step(p, g, m, v, t: int, lr: float, b1: float = 0.9, b2: float = 0.999,
              eps: float = 1e-8):
    """One Adam update (bias-corrected), in place; t counts from 1."""
    for k in NAMES:
        m[k] = b1 * m[k] + (1 - b1) * g[k]
        v[k] = b2 * v[k] + (1 - b2) * g[k] * g[k]
        mh = m[k] / (1 - b1 ** t)
        vh = v[k] / (1 - b2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)


def cosine_lr(step: int, steps: int, lr0: float = 1e-3, lr1: float = 1e-5) -> float:
    """Cosine decay from lr0 to lr1 over `steps` steps."""
    c = 0.5 * (1 + math.cos(math.pi * min(step, steps) / max(steps, 1)))
    return lr1 + (lr0 - lr1) * c


def minimal_image(d: np.ndarray, box: float = 1.0) -> np.ndarray:
    """Displacement in (-box/2, box/2]."""
    return d - box * np.ceil(d / box - 0.5)


def flatten(p) -> np.ndarray:
    return np.concatenate([p[k].ravel() for k in NAMES])


# ------------------------------------------------------------ placement
# the data-storage section's table: cube corner n = a + 2b + 4c at offset (a, b, c)
TET_TABLE = ((1, 0, 2, 4), (3, 1, 2, 4), (3, 5, 1, 4), (3, 6, 5, 4), (3, 2, 6, 4), (3, 7, 5, 6))


def corner_offset(n: int) -> np.ndarray:
    return np.array([n & 1, (n >> 1) & 1, (n >> 2) & 1], dtype=np.float64)


def fine_points(dims, r: int) -> np.ndarray:
    """Lagrangian points (as FP32) of the r-fold sub-lattice, tracer-id order."""
    f = [int(d) * r for d in dims]
    ids = np.arange(f[0] * f[1] * f[2], dtype=np.int64)
    idx = (ids % f[0], (ids // f[0]) % f[1], ids // (f[0] * f[1]))
    return np.stack([(idx[a].astype(np.float64) / f[a]).astype(np.float32) for a in range(3)], axis=1)


def barycentric_in_table(p: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """For points p (P, 3) of the unit cube: index of a table tetrahedron that
    contains each point and the barycentric coordinates (P, 4) there."""
    P = p.shape[0]
    tet = np.full(P, -1, dtype=np.int64)
    lam = np.zeros((P, 4))
    for t, corners in enumerate(TET_TABLE):
        V = np.stack([corner_offset(c) for c in corners])      # (4, 3)
        M = (V[1:] - V[0]).T                                     # columns: edge vectors
        sol = np.linalg.solve(M, (p - V[0]).T).T                 # (P, 3)
        l = np.concatenate([1.0 - sol.sum(axis=1, keepdims=True), sol], axis=1)
        inside = (l >= -1e-12).all(axis=1) & (tet < 0)
        tet[inside] = t
        lam[inside] = l[inside]
    return tet, lam


def wrap_f32(x: np.ndarray, box: float) -> np.ndarray:
    w = (x - box * np.floor(x / box)).astype(np.float32)
    w[w >= np.float32(box)] -= np.float32(box)
    w[w < 0] = 0.0
    return w


def place(coarse_xyz, dims, r: int, s_fine: np.ndarray, s_coarse=None, box: float = 1.0) -> np.ndarray:
    """Fine positions (P, 3) FP32: raw placement, or hybrid when s_coarse (the
    network at the coarse tracers, tracer-id order) is given."""
    q = fine_points(dims, r).astype(np.float64)
    f = [int(d) * r for d in dims]
    ids = np.arange(f[0] * f[1] * f[2], dtype=np.int64)
    I, J, K = ids % f[0], (ids // f[0]) % f[1], ids // (f[0] * f[1])
    x = (q + s_fine) * box
    cx = np.stack([np.asarray(c, dtype=np.float64) for c in coarse_xyz], axis=1)   # (N^3, 3)
    if s_coarse is not None:
        qc = fine_points(dims, 1).astype(np.float64)
        res = minimal_image(cx - (qc + s_coarse) * box, box)
        frac = np.stack([(I % r) / r, (J % r) / r, (K % r) / r], axis=1).astype(np.float64)
        tet, lam = barycentric_in_table(frac)
        for m in range(4):
            corner = np.array([TET_TABLE[t][m] for t in tet])
            ci = (I // r + (corner & 1)) % dims[0]
            cj = (J // r + ((corner >> 1) & 1)) % dims[1]
            ck = (K // r + ((corner >> 2) & 1)) % dims[2]
            cid = ci + dims[0] * (cj + dims[1] * ck)
            x = x + lam[:, m:m + 1] * res[cid]
    out = wrap_f32(x, box)
    coarse = (I % r == 0) & (J % r == 0) & (K % r == 0)
    cid = (I // r) + dims[0] * ((J // r) + dims[1] * (K // r))
    out[coarse] = cx[cid[coarse]].astype(np.float32)
    return out

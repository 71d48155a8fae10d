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


def features(q: np.ndarray, B: np.ndarray) -> np.ndarray:
    a = 2.0 * math.pi * (q @ B.T)            # (N, 64)
    return np.concatenate([np.sin(a), np.cos(a)], axis=1)


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    cdf = 0.5 * (1.0 + erf(x / math.sqrt(2.0)))
    pdf = np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)
    return cdf + x * pdf


def forward(p: Dict[str, np.ndarray], q: np.ndarray, B: np.ndarray):
    """Returns the prediction (N, 3) and the cache for backward."""
    g = features(q, B)
    hs, zs = [g], []
    h = g
    for i in range(1, DEPTH + 1):
        z = h @ p[f"W{i}"].T + p[f"b{i}"]
        zs.append(z)
        h = gelu(z)
        hs.append(h)
    out = h @ p["W5"].T + p["b5"]
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

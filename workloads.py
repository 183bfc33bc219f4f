"""Seeded synthetic inputs for PINS solves.

This module only draws problem data (point clouds, histograms, marginals,
dense cost matrices built from points or grids).  It contains none of the
solver's arithmetic, so both the FP64 CPU oracle and the HIP path can consume
the very same arrays.

Every generator is keyed by ``np.random.SeedSequence([ROOT, config, instance,
side])`` so that any single instance can be regenerated on its own.

Families (stand-ins for the paper's workloads; none of them reproduces items
of MNIST or DOTmark):

* ``points_instance``  -- two independent point clouds in [0,1]^d and
  marginals ``(U(0,1)+0.01)`` normalised (plain single-instance case,
  100x100 in the plane), or Dirichlet(1)+floor marginals (batched case).
* ``blob_histogram``   -- 28x28 (or s x s) mixture of 1..3 Gaussian blobs,
  sigma in [1.5, 4] px, plus a 1e-6 floor, normalised (image-histogram case).
* ``grid_histogram``   -- s x s white noise / 5-component Gaussian mixture /
  Cauchy-density bumps, normalised (large-grid case).
* ``assignment_instance`` -- c_ij ~ U[0,1], a = b = 1/n (Section 5.1
  synthetic random assignment family).
"""
from __future__ import annotations

import math

import numpy as np

ROOT_SEED = 250203749

# config ids used in the seed sequence
CFG_POINTS = 1
CFG_BLOBS = 2
CFG_GRID = 3
CFG_BATCH = 4
CFG_SERVE = 5
CFG_ASSIGN = 6
CFG_MISC = 7


def rng(config: int, instance: int, side: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([ROOT_SEED, config, instance, side]))


def _normalise(v: np.ndarray) -> np.ndarray:
    v = np.asarray(v, dtype=np.float64)
    return v / v.sum()


# ----------------------------------------------------------------------------
# dense cost construction (problem input for the dense API)
# ----------------------------------------------------------------------------

def sqeuclid_dense(x: np.ndarray, y: np.ndarray, normalise: bool = True) -> np.ndarray:
    """Dense squared-Euclidean cost ||x_i - y_j||^2, optionally divided by its max."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    diff = x[:, None, :] - y[None, :, :]
    C = np.einsum("ijk,ijk->ij", diff, diff)
    if normalise:
        C = C / C.max()
    return np.ascontiguousarray(C)


def grid_coords(s: int) -> np.ndarray:
    """Pixel (row, col) coordinates of an s x s grid, pixel index = row*s + col."""
    r, c = np.divmod(np.arange(s * s), s)
    return np.stack([r, c], axis=1).astype(np.float64)


def grid_dense(s: int, normalise: bool = True) -> np.ndarray:
    """Dense squared grid distance between pixels; max is 2(s-1)^2."""
    p = grid_coords(s)
    C = sqeuclid_dense(p, p, normalise=False)
    if normalise:
        C = C / (2.0 * (s - 1) ** 2)
    return C


# ----------------------------------------------------------------------------
# families
# ----------------------------------------------------------------------------

def points_instance(instance: int, m: int = 100, n: int = 100, d: int = 2,
                    config: int = CFG_POINTS, marginals: str = "uniform+0.01"):
    """Two independent point clouds and positive marginals.

    marginals: "uniform+0.01" -> (U(0,1)+0.01)/sum;  "dirichlet" -> Dirichlet(1)+1e-8, renormalised.
    Returns dict(x, y, a, b).
    """
    gx = rng(config, instance, 0)
    gy = rng(config, instance, 1)
    x = gx.uniform(0.0, 1.0, size=(m, d))
    y = gy.uniform(0.0, 1.0, size=(n, d))
    ga = rng(config, instance, 2)
    gb = rng(config, instance, 3)
    if marginals == "uniform+0.01":
        a = _normalise(ga.uniform(0.0, 1.0, m) + 0.01)
        b = _normalise(gb.uniform(0.0, 1.0, n) + 0.01)
    elif marginals == "dirichlet":
        a = _normalise(ga.dirichlet(np.ones(m)) + 1e-8)
        b = _normalise(gb.dirichlet(np.ones(n)) + 1e-8)
    else:
        raise ValueError(marginals)
    return dict(x=x, y=y, a=a, b=b)


def blob_histogram(instance: int, side: int, s: int = 28, floor: float = 1e-6,
                   config: int = CFG_BLOBS) -> np.ndarray:
    """Mixture of 1..3 equal-weight Gaussian blobs on an s x s grid, + floor, normalised."""
    g = rng(config, instance, side)
    nb = int(g.integers(1, 4))
    p = grid_coords(s)
    h = np.zeros(s * s)
    for _ in range(nb):
        mu = g.uniform(0.0, s - 1.0, size=2)
        sig = g.uniform(1.5, 4.0)
        d2 = ((p - mu) ** 2).sum(axis=1)
        h += np.exp(-d2 / (2.0 * sig * sig))
    h = h / h.sum() + floor
    return _normalise(h)


def blob_pair(instance: int, s: int = 28):
    return dict(a=blob_histogram(instance, 0, s), b=blob_histogram(instance, 1, s), s=s)


GRID_CLASSES = ("white", "gmm", "cauchy")


def grid_histogram(cls: str, instance: int, side: int, s: int = 64,
                   config: int = CFG_GRID) -> np.ndarray:
    """s x s histogram of one of three classes, normalised."""
    g = rng(config, instance * 8 + GRID_CLASSES.index(cls), side)
    p = grid_coords(s)
    if cls == "white":
        h = g.uniform(0.0, 1.0, s * s)
        h = np.maximum(h, 1e-12)
    elif cls == "gmm":
        w = g.dirichlet(np.ones(5))
        h = np.zeros(s * s)
        for k in range(5):
            mu = g.uniform(0.0, s - 1.0, size=2)
            sig = g.uniform(3.0, 9.0) * s / 64.0
            d2 = ((p - mu) ** 2).sum(axis=1)
            h += w[k] * np.exp(-d2 / (2.0 * sig * sig)) / (2 * math.pi * sig * sig)
        h = h / h.sum() + 1e-8
    elif cls == "cauchy":
        nb = int(g.integers(1, 6))
        w = g.dirichlet(np.ones(nb))
        h = np.zeros(s * s)
        for k in range(nb):
            mu = g.uniform(0.0, s - 1.0, size=2)
            gam = g.uniform(2.0, 8.0) * s / 64.0
            d2 = ((p - mu) ** 2).sum(axis=1)
            h += w[k] * (1.0 + d2 / (gam * gam)) ** (-1.5) / (gam * gam)
        h = h / h.sum() + 1e-8
    else:
        raise ValueError(cls)
    return _normalise(h)


def grid_pair(cls: str, instance: int, s: int = 64):
    return dict(a=grid_histogram(cls, instance, 0, s), b=grid_histogram(cls, instance, 1, s), s=s)


def batch_instance(instance: int, lo: int = 64, hi: int = 2048):
    """Uneven-size point-cloud instance of the batched family: m, n log-uniform, d in {2, 8, 32}."""
    g = rng(CFG_BATCH, instance, 9)
    m = int(round(math.exp(g.uniform(math.log(lo), math.log(hi)))))
    n = int(round(math.exp(g.uniform(math.log(lo), math.log(hi)))))
    d = (2, 8, 32)[instance % 3]
    inst = points_instance(instance, m=m, n=n, d=d, config=CFG_BATCH, marginals="dirichlet")
    inst["d"] = d
    return inst


def assignment_instance(instance: int, n: int):
    """Random assignment: c_ij ~ U[0,1], a = b = 1/n."""
    g = rng(CFG_ASSIGN, instance, n)
    C = g.uniform(0.0, 1.0, size=(n, n))
    a = np.full(n, 1.0 / n)
    return dict(C=C, a=a, b=a.copy())


def serve_requests(count: int, rate: float, instance0: int = 0):
    """Poisson arrival stream of mixed grid requests: 60% s=32, 30% s=64, 10% s=128.

    Returns a list of dicts (t_arrival, s, a, b) with histograms 50/50 Gaussian mixture / white noise.
    """
    g = rng(CFG_SERVE, instance0, 0)
    t = 0.0
    out = []
    for r in range(count):
        t += g.exponential(1.0 / rate)
        u = g.uniform()
        s = 32 if u < 0.6 else (64 if u < 0.9 else 128)
        cls = "gmm" if g.uniform() < 0.5 else "white"
        a = grid_histogram(cls, instance0 * 100000 + r, 0, s, config=CFG_SERVE)
        b = grid_histogram(cls, instance0 * 100000 + r, 1, s, config=CFG_SERVE)
        out.append(dict(t=t, s=s, cls=cls, a=a, b=b))
    return out

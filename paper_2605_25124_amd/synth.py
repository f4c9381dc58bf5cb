"""Seeded synthetic inputs shared by the GPU path, the FP64 oracle and the bench.

This module only draws random numbers; it holds none of the Gini MDS
arithmetic, so both sides can take their inputs from it without sharing any
computation.  Every generator uses ``numpy.random.Generator(PCG64(seed))``
with ``seed = 260525124 + k`` for workload ``k`` and a second stream
(``seed + 10**6``) for the initial configuration, so that any subset of the
workloads can be regenerated bit-for-bit on any machine.

Workloads (the paper's datasets are not available, these stand in for their
shapes and value distributions):

* ``workload_small``   : 200 x 10 iid N(0,1) in FP64 with 5 % of rows scaled by
  10 (the outlier contamination of the UCI experiments, Section V-A), nu=2,
  p=2, 100 iterations.
* ``workload_gmm``     : 2000 x 16 three-component Gaussian mixture
  (means ~ N(0, 4I), unit covariance) plus 10 % uniform outliers in
  [-20, 20]^16, nu in {1.5, 2, 3}, p=2, 500 iterations.
* ``workload_images``  : 10000 x 784 image-like rows (28 x 28 grids with 1-3
  Gaussian blobs, the brightest 20 % of pixels quantised to uint8, plus
  N(0, 32^2) noise clipped to [0, 255]), heavy ties at 0 and 255; a
  stand-in for the shape of the MNIST experiment (Section V-B), nu=2, p=2,
  300 iterations.
* ``workload_sweep``   : 16 Gaussian-mixture problems, n ~ U{100..3000},
  m ~ U{4..64}, 5 % outliers, each at 8 values of nu in [1.1, 4]
  (128 instances, the nu-sweep of Algorithm 1), p=2, 200 iterations.
* ``workload_heavy``   : 50000 x 64 iid Student-t(3) (heavy-tailed, as in the
  simulations of Section V-C), nu=2, p=3, 100 iterations.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

SEED_BASE = 260525124
Z_STREAM = 10**6


def rng_for(k: int, stream: int = 0) -> np.random.Generator:
    """Generator for workload ``k``; ``stream=1`` is the initial-configuration stream."""
    return np.random.Generator(np.random.PCG64(SEED_BASE + k + stream * Z_STREAM))


@dataclass
class Problem:
    """One MDS problem: data X (n x m), the nu values, latent p, initial Z0 per nu."""
    X: np.ndarray
    nus: List[float]
    p: int
    iters: int
    Z0: List[np.ndarray] = field(default_factory=list)
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.X.shape[0])

    @property
    def m(self) -> int:
        return int(self.X.shape[1])


def initial_config(g: np.random.Generator, n: int, p: int, dtype=np.float32) -> np.ndarray:
    """Z0 iid N(0, 0.1^2) (variance 1e-2), shape n x p."""
    return (0.1 * g.standard_normal((n, p))).astype(dtype)


def gaussian_mixture(g: np.random.Generator, n: int, m: int, n_comp: int = 3,
                     outlier_frac: float = 0.1, box: float = 20.0) -> np.ndarray:
    """Rows from an equal-weight Gaussian mixture (means ~ N(0, 4I), unit
    covariance) plus ``outlier_frac`` of rows uniform in [-box, box]^m, shuffled."""
    n_out = int(round(outlier_frac * n))
    n_in = n - n_out
    means = 2.0 * g.standard_normal((n_comp, m))
    lab = g.integers(0, n_comp, size=n_in)
    inl = means[lab] + g.standard_normal((n_in, m))
    out = g.uniform(-box, box, size=(n_out, m))
    X = np.concatenate([inl, out], axis=0)
    return X[g.permutation(n)]


def workload_small() -> Problem:
    g = rng_for(1)
    n, m = 200, 10
    X = g.standard_normal((n, m))
    rows = g.choice(n, size=n // 20, replace=False)
    X[rows] *= 10.0
    gz = rng_for(1, 1)
    return Problem(X=X, nus=[2.0], p=2, iters=100,
                   Z0=[initial_config(gz, n, 2, np.float64)], name="small n=200 m=10")


def workload_gmm() -> Problem:
    g = rng_for(2)
    X = gaussian_mixture(g, 2000, 16, 3, 0.1).astype(np.float32)
    gz = rng_for(2, 1)
    nus = [1.5, 2.0, 3.0]
    return Problem(X=X, nus=nus, p=2, iters=500,
                   Z0=[initial_config(gz, 2000, 2) for _ in nus], name="gmm n=2000 m=16")


def image_rows(g: np.random.Generator, n: int) -> np.ndarray:
    """n image-like rows of 28 x 28 = 784 pixels (see module docstring)."""
    side = 28
    yy, xx = np.meshgrid(np.arange(side, dtype=np.float64), np.arange(side, dtype=np.float64),
                         indexing="ij")
    yy = yy.reshape(-1)
    xx = xx.reshape(-1)
    nb = g.integers(1, 4, size=n)                       # 1..3 blobs
    cy = g.uniform(4.0, 24.0, size=(n, 3))
    cx = g.uniform(4.0, 24.0, size=(n, 3))
    sb = g.uniform(1.5, 3.5, size=(n, 3))
    amp = g.uniform(0.6, 1.0, size=(n, 3))
    inten = np.zeros((n, side * side))
    for b in range(3):
        on = (b < nb).astype(np.float64)[:, None]
        d2 = (yy[None, :] - cy[:, b:b + 1]) ** 2 + (xx[None, :] - cx[:, b:b + 1]) ** 2
        inten += on * amp[:, b:b + 1] * np.exp(-d2 / (2.0 * sb[:, b:b + 1] ** 2))
    keep = int(round(0.2 * side * side))
    order = np.argsort(-inten, axis=1, kind="stable")[:, :keep]
    img = np.zeros_like(inten)
    mx = inten.max(axis=1, keepdims=True)
    vals = np.take_along_axis(inten, order, axis=1) / mx * 255.0
    np.put_along_axis(img, order, np.rint(vals), axis=1)
    img = img + 32.0 * g.standard_normal(img.shape)
    return np.clip(img, 0.0, 255.0).astype(np.float32)


def workload_images(n: int = 10000) -> Problem:
    g = rng_for(3)
    X = image_rows(g, n)
    gz = rng_for(3, 1)
    return Problem(X=X, nus=[2.0], p=2, iters=300,
                   Z0=[initial_config(gz, n, 2)], name=f"images n={n} m=784")


def workload_sweep() -> List[Problem]:
    g = rng_for(4)
    gz = rng_for(4, 1)
    nus = [float(v) for v in np.linspace(1.1, 4.0, 8)]
    probs = []
    for b in range(16):
        n = int(g.integers(100, 3001))
        m = int(g.integers(4, 65))
        X = gaussian_mixture(g, n, m, 3, 0.05).astype(np.float32)
        probs.append(Problem(X=X, nus=nus, p=2, iters=200,
                             Z0=[initial_config(gz, n, 2) for _ in nus],
                             name=f"sweep[{b}] n={n} m={m}"))
    return probs


def workload_heavy(n: int = 50000) -> Problem:
    g = rng_for(5)
    X = g.standard_t(3.0, size=(n, 64)).astype(np.float32)
    gz = rng_for(5, 1)
    return Problem(X=X, nus=[2.0], p=3, iters=100,
                   Z0=[initial_config(gz, n, 3)], name=f"heavy n={n} m=64")


def subsample(n_full: int, k: int, seed: int) -> np.ndarray:
    """Sorted seeded sample of k distinct row indices out of n_full."""
    g = np.random.Generator(np.random.PCG64(seed))
    return np.sort(g.choice(n_full, size=min(k, n_full), replace=False))


# ---------------------------------------------------------------- edge cases
def rows_with_ties(g: np.random.Generator, rows: int, d: int, levels: Optional[int] = 3) -> np.ndarray:
    """FP32 rows whose entries come from a few integer levels (many exact ties)."""
    if levels is None:
        return g.standard_normal((rows, d)).astype(np.float32)
    return g.integers(-levels, levels + 1, size=(rows, d)).astype(np.float32)


def signed_zero_rows(g: np.random.Generator, rows: int, d: int) -> np.ndarray:
    """FP32 rows mixing +0.0, -0.0 and a few non-zero values (IEEE -0 == +0)."""
    a = g.integers(0, 4, size=(rows, d))
    out = np.where(a == 0, 0.0, np.where(a == 1, -0.0, g.standard_normal((rows, d))))
    return out.astype(np.float32)

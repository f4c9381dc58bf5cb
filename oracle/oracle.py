"""ctypes wrapper around the FP64 CPU oracle (``gini_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test-suite, the package smoke check and the
benchmark's CPU-baseline leg are the only callers.  The product path never
imports this module, and this module imports nothing from the product.

``build()`` compiles ``gini_oracle.c`` with plain ``gcc -O2`` (no fast-math,
no FMA contraction, single thread) into ``liboracle.so`` next to it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "gini_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

EXACT = 0
MATCH32 = 1
LATENT_GINI = 0
LATENT_EUCLID = 1

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle shared library (always, when ``force``)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
               "-o", tmp, SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        L = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        i32 = ctypes.c_int
        f64 = ctypes.c_double
        L.orc_rank2_count.argtypes = [P, i32, P]
        L.orc_rank2_sort.argtypes = [P, i32, P]
        L.orc_rank2.argtypes = [P, i32, P]
        L.orc_rank2_rows.argtypes = [P, i64, i32, i64, P, i64]
        L.orc_gini_dist.argtypes = [P, i32, f64]
        L.orc_gini_dist.restype = f64
        L.orc_gini_dist_grad.argtypes = [P, i32, f64, P]
        L.orc_gini_dist_grad.restype = f64
        L.orc_gini_asym.argtypes = [P, i32, f64]
        L.orc_gini_asym.restype = f64
        L.orc_dissim.argtypes = [P, i64, i32, i64, i32, P, i32, P, i64, i64]
        L.orc_dissim_pairs.argtypes = [P, i32, i64, i32, P, P, i64, P, i32, P]
        L.orc_stress.argtypes = [P, i64, i64, P, i32, i64, f64, i32, i32, P, i64]
        L.orc_stress.restype = f64
        L.orc_delta_sumsq.argtypes = [P, i64, i64]
        L.orc_delta_sumsq.restype = f64
        L.orc_grad_rows.argtypes = [P, i64, P, i64, i64, P, i32, i64, f64, i32, i32, P, i64]
        L.orc_grad_rows.restype = f64
        L.orc_step_size.argtypes = [i64, i32, f64, i32]
        L.orc_step_size.restype = f64
        L.orc_solve.argtypes = [P, i64, i64, P, i32, i64, f64, i32, i32, i32, f64, P]
        L.orc_sammon.argtypes = [P, i64, i64, P, i32, i64, f64, i32, i32, P, i64]
        L.orc_sammon.restype = f64
        L.orc_sammon_step.argtypes = [P, i64, i64, i32, f64, i32]
        L.orc_sammon_step.restype = f64
        L.orc_solve_sammon.argtypes = [P, i64, i64, P, i32, i64, f64, i32, i32, i32, f64, P]
        L.orc_dissim_scale.argtypes = [P, i64, i32, i64, i32, f64, P, i64]
        L.orc_grad_scale_rows.argtypes = [P, i64, P, i64, i64, P, i32, i64, f64, i32, i32, i32, f64, P, i64]
        _lib = L
    return _lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def rank2(v, method: str = "auto") -> np.ndarray:
    """Doubled midranks t = 2R of one vector."""
    v = _f64(v).reshape(-1)
    t = np.empty(v.shape[0], dtype=np.int32)
    fn = {"auto": lib().orc_rank2, "count": lib().orc_rank2_count, "sort": lib().orc_rank2_sort}[method]
    fn(_ptr(v), int(v.shape[0]), _ptr(t))
    return t


def rank2_rows(V) -> np.ndarray:
    """Doubled midranks of every row of a 2-D array."""
    V = _f64(V)
    rows, d = V.shape
    t = np.empty((rows, d), dtype=np.int32)
    lib().orc_rank2_rows(_ptr(V), rows, d, d, _ptr(t), d)
    return t


def gini_dist(z, nu: float) -> float:
    z = _f64(z).reshape(-1)
    return float(lib().orc_gini_dist(_ptr(z), int(z.shape[0]), float(nu)))


def gini_dist_grad(z, nu: float):
    z = _f64(z).reshape(-1)
    g = np.empty_like(z)
    v = lib().orc_gini_dist_grad(_ptr(z), int(z.shape[0]), float(nu), _ptr(g))
    return float(v), g


def gini_asym(z, nu: float) -> float:
    z = _f64(z).reshape(-1)
    return float(lib().orc_gini_asym(_ptr(z), int(z.shape[0]), float(nu)))


def dissim(X, nus, mode: int = MATCH32) -> np.ndarray:
    """Full symmetric dissimilarity matrices, shape (len(nus), n, n)."""
    X = _f64(X)
    n, m = X.shape
    nus_a = _f64(list(nus))
    out = np.empty((len(nus_a), n, n), dtype=np.float64)
    lib().orc_dissim(_ptr(X), n, m, m, mode, _ptr(nus_a), len(nus_a), _ptr(out), n, n * n)
    return out


def dissim_pairs(X, pi, pj, nus, mode: int = MATCH32) -> np.ndarray:
    """Distances for explicit pairs, shape (npairs, len(nus))."""
    X = _f64(X)
    n, m = X.shape
    pi = np.ascontiguousarray(pi, dtype=np.int64)
    pj = np.ascontiguousarray(pj, dtype=np.int64)
    nus_a = _f64(list(nus))
    out = np.empty((pi.shape[0], len(nus_a)), dtype=np.float64)
    lib().orc_dissim_pairs(_ptr(X), m, m, mode, _ptr(pi), _ptr(pj), pi.shape[0], _ptr(nus_a),
                           len(nus_a), _ptr(out))
    return out


def stress(Delta, Z, nu: float, latent: int = LATENT_GINI, mode: int = MATCH32, grad: bool = True):
    """(sigma, G) with sigma = sum_{i<j} (delta_ij - Delta_ij)^2 and G its gradient."""
    D = _f64(Delta)
    Z = _f64(Z)
    n, p = Z.shape
    G = np.empty((n, p), dtype=np.float64) if grad else None
    s = lib().orc_stress(_ptr(D), n, D.shape[1], _ptr(Z), p, p, float(nu), latent, mode,
                         _ptr(G) if grad else None, p)
    return float(s), G


def delta_sumsq(Delta) -> float:
    """sum_{i<j} Delta_ij^2, the Kruskal-stress normaliser."""
    D = _f64(Delta)
    return float(lib().orc_delta_sumsq(_ptr(D), D.shape[0], D.shape[1]))


def kruskal(Delta, Z, nu: float, latent: int = LATENT_GINI, mode: int = MATCH32) -> float:
    """Kruskal stress sqrt(sigma / sum_{i<j} Delta_ij^2) of Z against Delta."""
    s, _ = stress(Delta, Z, nu, latent, mode, grad=False)
    den = delta_sumsq(Delta)
    return float(np.sqrt(s / den)) if den > 0 else 0.0


def sammon(Delta, Z, nu: float, latent: int = LATENT_GINI, mode: int = MATCH32, grad: bool = True):
    """(sigma, G): Sammon's stress (1/S) sum_{i<j} (delta_ij - Delta_ij)^2 / Delta_ij, S = sum Delta_ij."""
    D = _f64(Delta)
    Z = _f64(Z)
    n, p = Z.shape
    G = np.empty((n, p), dtype=np.float64) if grad else None
    s = lib().orc_sammon(_ptr(D), n, D.shape[1], _ptr(Z), p, p, float(nu), latent, mode,
                         _ptr(G) if grad else None, p)
    return float(s), G


def sammon_step(Delta, p: int, nu: float, latent: int = LATENT_GINI) -> float:
    D = _f64(Delta)
    return float(lib().orc_sammon_step(_ptr(D), D.shape[0], D.shape[1], p, float(nu), latent))


def solve_sammon(Delta, Z0, nu: float, iters: int, latent: int = LATENT_GINI, mode: int = MATCH32,
                 eta: float = 0.0):
    """Fixed-step descent on the Sammon stress; returns (Z_T, sigma history)."""
    D = _f64(Delta)
    Z = _f64(Z0).copy()
    n, p = Z.shape
    hist = np.empty(iters, dtype=np.float64)
    lib().orc_solve_sammon(_ptr(D), n, D.shape[1], _ptr(Z), p, p, float(nu), latent, mode, iters,
                           float(eta), _ptr(hist))
    return Z, hist


def select_nu(X, nus, Z0, iters: int, folds: int = 1, latent: int = LATENT_GINI, mode: int = MATCH32):
    """Algorithm 1: for each nu and each fold (rows [f n / K, (f+1) n / K)),
    the fold's dissimilarities, `iters` descent steps from the fold's rows of
    Z0, and the Kruskal stress of the result with the Euclidean latent
    distance; nu* minimises the mean over the folds.  Returns
    (best index, ks_mean[n_nu], ks_fold[n_nu, folds], final Z per nu)."""
    X = np.asarray(X)
    Z0 = np.asarray(Z0)
    n = X.shape[0]
    ks = np.zeros((len(nus), folds))
    Zs = np.zeros((len(nus),) + Z0.shape)
    for k, nu in enumerate(nus):
        for f in range(folds):
            a, b = f * n // folds, (f + 1) * n // folds
            D = dissim(X[a:b], [nu], mode)[0]
            Z, _ = solve(D, Z0[a:b], nu, iters, latent, mode)
            Zs[k, a:b] = Z
            ks[k, f] = kruskal(D, Z, nu, LATENT_EUCLID, mode)
    mean = ks.mean(axis=1)
    return int(np.argmin(mean)), mean, ks, Zs


def alternate_nu(X, nus, Z0, iters: int, rounds: int, init: int, latent: int = LATENT_GINI,
                 mode: int = MATCH32):
    """Algorithm 2's alternation: each round a Sammon fit at the current nu
    (orc_sammon_step's step, warm start), then the Kruskal stress of the fit
    against every nu with the Euclidean latent distance, and a move to the
    argmin.  Returns (best index, nu index per round, ks[rounds, n_nu], Z)."""
    Ds = dissim(np.asarray(X), list(nus), mode)
    Z = np.asarray(Z0, dtype=np.float64).copy()
    p = Z.shape[1]
    cur = int(init)
    hist = np.zeros(rounds, dtype=np.int64)
    ks = np.zeros((rounds, len(nus)))
    for t in range(rounds):
        eta = sammon_step(Ds[cur], p, nus[cur], latent)
        Z, _ = solve_sammon(Ds[cur], Z, nus[cur], iters, latent, mode, eta)
        hist[t] = cur
        for k, nu in enumerate(nus):
            ks[t, k] = kruskal(Ds[k], Z, nu, LATENT_EUCLID, mode)
        cur = int(np.argmin(ks[t]))
    return cur, hist, ks, Z


def classical_mds(Delta, p: int):
    """Section IV-A: B = -1/2 H D^2 H, its p largest eigenpairs (LAPACK's
    symmetric eigensolver as the library step), Z = V_p sqrt(max(lam, 0)).
    Returns (Z, eigenvalues in decreasing order)."""
    D = _f64(Delta)
    n = D.shape[0]
    D2 = D * D
    np.fill_diagonal(D2, 0.0)
    H = np.eye(n) - np.ones((n, n)) / n
    B = -0.5 * H @ D2 @ H
    lam, V = np.linalg.eigh(0.5 * (B + B.T))
    order = np.argsort(lam)[::-1][:p]
    lam = lam[order]
    return V[:, order] * np.sqrt(np.maximum(lam, 0.0)), lam


def standardize(X):
    """Section V-C preprocessing: columns to zero median, unit population variance."""
    X = np.asarray(X, dtype=np.float64)
    sd = X.std(axis=0)
    sd = np.where(sd > 0, sd, 1.0)
    return (X - np.median(X, axis=0)) / sd


def dissim_scale(X, nu: float, mode: int = MATCH32) -> np.ndarray:
    """S_ij = sum_c |z_c g_c| (g the rank-frozen gradient of the distance): the
    sum of the absolute values of the terms whose sum is Delta_ij, the scale
    of its rounding error.  Full n x n matrix."""
    X = _f64(X)
    n, m = X.shape
    S = np.empty((n, n), dtype=np.float64)
    lib().orc_dissim_scale(_ptr(X), n, m, m, mode, float(nu), _ptr(S), n)
    return S


def grad_scale_rows(Drows, rows, Z, nu: float, latent: int = LATENT_GINI, mode: int = MATCH32,
                    loss: int = 0, S: float = 0.0) -> np.ndarray:
    """B[q, c] = sum_{j != rows[q]} |term_j| over the terms whose sum is the
    gradient entry G[rows[q], c]: |2 r a_c| for the raw stress (loss 0), that
    over S Delta_ij for Sammon's stress (loss 1, S its normaliser)."""
    D = _f64(Drows)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    Z = _f64(Z)
    n, p = Z.shape
    B = np.empty((rows.shape[0], p), dtype=np.float64)
    lib().orc_grad_scale_rows(_ptr(D), D.shape[1], _ptr(rows), rows.shape[0], n, _ptr(Z), p, p, float(nu),
                              latent, mode, int(loss), float(S), _ptr(B), p)
    return B


def grad_scale(Delta, Z, nu: float, latent: int = LATENT_GINI, mode: int = MATCH32, loss: int = 0,
               S: float = 0.0) -> np.ndarray:
    """grad_scale_rows over every point (Delta n x n)."""
    n = np.asarray(Z).shape[0]
    return grad_scale_rows(Delta, np.arange(n), Z, nu, latent, mode, loss, S)


def grad_rows(Drows, rows, Z, nu: float, latent: int = LATENT_GINI, mode: int = MATCH32):
    """Gradient rows G[rows] from the corresponding rows of Delta; also returns
    the partial sum over the selected rows of sum_{j>i} r_ij^2."""
    D = _f64(Drows)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    Z = _f64(Z)
    n, p = Z.shape
    G = np.empty((rows.shape[0], p), dtype=np.float64)
    part = lib().orc_grad_rows(_ptr(D), D.shape[1], _ptr(rows), rows.shape[0], n, _ptr(Z), p, p,
                               float(nu), latent, mode, _ptr(G), p)
    return G, float(part)


def step_size(n: int, p: int, nu: float, latent: int = LATENT_GINI) -> float:
    return float(lib().orc_step_size(n, p, float(nu), latent))


def solve(Delta, Z0, nu: float, iters: int, latent: int = LATENT_GINI, mode: int = MATCH32,
          eta: float = 0.0):
    """Fixed-step gradient descent; returns (Z_T, sigma history)."""
    D = _f64(Delta)
    Z = _f64(Z0).copy()
    n, p = Z.shape
    hist = np.empty(iters, dtype=np.float64)
    lib().orc_solve(_ptr(D), n, D.shape[1], _ptr(Z), p, p, float(nu), latent, mode, iters,
                    float(eta), _ptr(hist))
    return Z, hist

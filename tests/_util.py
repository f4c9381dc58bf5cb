"""Helpers shared by the GPU parity tests (comparison only; no method arithmetic)."""
import numpy as np


def f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


def dissim_scale(orc, X32, pairs, nu):
    """S_ij = sum_c |z_c a_c|: the absolute-value sum behind Delta_ij (a_c the
    oracle's rank-frozen derivative), the natural scale of its rounding error."""
    S = np.empty(len(pairs))
    for q, (i, j) in enumerate(pairs):
        z = (X32[i].astype(np.float32) - X32[j].astype(np.float32)).astype(np.float64)
        _, a = orc.gini_dist_grad(z, nu)
        S[q] = float(np.sum(np.abs(z * a)))
    return S


def assert_dissim_close(D_gpu, D_ref, S, rtol=1e-5, what=""):
    err = np.abs(D_gpu.astype(np.float64) - D_ref)
    bound = rtol * S + 1e-30
    bad = err > bound
    if bad.any():
        k = int(np.argmax(err / bound))
        raise AssertionError(f"{what}: {int(bad.sum())} entries off; worst err {err.flat[k]:.3e} "
                             f"vs bound {bound.flat[k]:.3e} (ref {D_ref.flat[k]:.6e})")


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def assert_grad_close(G_gpu, G_ref, B, rtol=1e-4, extra=0.0, what=""):
    """Gradient parity entry by entry: |G_gpu - G_ref| <= rtol * B + extra, with
    B the oracle's sum of the absolute values of the terms whose sum is each
    entry (oracle.grad_scale / grad_scale_rows), and the relative 2-norm within
    rtol as well.  `extra` covers rounding that is not the gradient's (a step
    recovered from two iterates).  Returns the worst |error| / B."""
    G_gpu = np.asarray(G_gpu, dtype=np.float64)
    G_ref = np.asarray(G_ref, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    err = np.abs(G_gpu - G_ref)
    bound = rtol * B + extra + 1e-30
    bad = err > bound
    if bad.any():
        k = int(np.argmax(err / bound))
        raise AssertionError(f"{what}: {int(bad.sum())} gradient entries off; worst at {np.unravel_index(k, err.shape)}: "
                             f"err {err.flat[k]:.3e} vs bound {bound.flat[k]:.3e} (ref {G_ref.flat[k]:.6e}, "
                             f"scale {B.flat[k]:.3e})")
    r = rel(G_gpu, G_ref)
    assert r <= rtol, (what, r)
    return float(np.max(err / (B + 1e-300))) if err.size else 0.0


def step_rounding(Z0, Z1, eta, G_ref):
    """What rounding adds to a gradient recovered as (Z0 - Z1) / eta from one
    FP32 descent step Z1 = fl32(Z0 - eta32 G): half an ulp of Z1 over eta, and
    the roundings of eta to FP32 and of eta32 G (each relative 2^-24 of G)."""
    Z0 = np.abs(np.asarray(Z0, dtype=np.float64))
    Z1 = np.abs(np.asarray(Z1, dtype=np.float64))
    return 2.0 ** -24 * (np.maximum(Z0, Z1) / eta + 2.0 * np.abs(np.asarray(G_ref, dtype=np.float64))) * 1.01

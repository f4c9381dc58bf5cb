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

"""Python binding of ``libginimds.so`` (argument marshalling only).

Every function here has the name of the C entry point it calls and does
nothing but check tensors, pass their device pointers, sizes and the current
torch stream, and raise on a non-OK status.  All the arithmetic happens in the
HIP kernels behind the C ABI (``include/ginimds.h``).  There is no fallback:
if the library is missing, importing this module fails.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Iterable, List, Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libginimds.so")

GINI_OK = 0
LATENT_GINI = 0
LATENT_EUCLID = 1
LOSS_RAW = 0
LOSS_SAMMON = 1
SOLVE_PERSISTENT = 1
SOLVE_PLAIN = 2
SOLVE_BATCHED = 4
SOLVE_AUTOTUNE = 8
SOLVE_CHECK_FINITE = 16
SOLVE_SPLIT = 32
SOLVE_CALLER_ORDER = 64

_STATUS = {0: "GINI_OK", 1: "GINI_EINVAL", 2: "GINI_ENOMEM", 3: "GINI_EDEVICE", 4: "GINI_ENOTFINITE",
           5: "GINI_EUNSUPPORTED"}


class GiniError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS.get(status, status)}: {message}")
        self.status = status
        self.message = message


class _Instance(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("p", ctypes.c_int32), ("loss", ctypes.c_int32),
                ("Delta", ctypes.c_void_p), ("ldd", ctypes.c_int64), ("Z", ctypes.c_void_p),
                ("ldz", ctypes.c_int64), ("nu", ctypes.c_double), ("latent", ctypes.c_int),
                ("eta", ctypes.c_float), ("sigma_hist", ctypes.c_void_p),
                ("delta_sumsq", ctypes.c_void_p), ("ks_hist", ctypes.c_void_p),
                ("delta_sum", ctypes.c_void_p)]


class _SelectOpts(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("p", ctypes.c_int32), ("latent", ctypes.c_int),
                ("folds", ctypes.c_int32), ("flags", ctypes.c_int32), ("tile", ctypes.c_int32)]


class _AlternateOpts(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("p", ctypes.c_int32), ("latent", ctypes.c_int),
                ("rounds", ctypes.c_int32), ("init", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("tile", ctypes.c_int32)]


class _Profile(ctypes.Structure):
    _fields_ = [("tile_launches", ctypes.c_int64), ("tile_ms", ctypes.c_double),
                ("reduce_launches", ctypes.c_int64), ("reduce_ms", ctypes.c_double),
                ("persistent_launches", ctypes.c_int64), ("persistent_ms", ctypes.c_double),
                ("dissim_launches", ctypes.c_int64), ("dissim_ms", ctypes.c_double)]


class _Opts(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("flags", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("grid", ctypes.c_int32)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2605_25124_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P, i64, i32, f64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    L.gini_create.argtypes = [ctypes.POINTER(P), ctypes.c_int]
    L.gini_destroy.argtypes = [P]
    L.gini_destroy.restype = None
    L.gini_last_error.argtypes = [P]
    L.gini_last_error.restype = ctypes.c_char_p
    L.gini_status_string.argtypes = [ctypes.c_int]
    L.gini_status_string.restype = ctypes.c_char_p
    L.gini_version.restype = ctypes.c_int
    L.gini_weight_table.argtypes = [i32, f64, P]
    L.gini_weight_table.restype = ctypes.c_int
    L.gini_rank.argtypes = [P, P, i64, i32, i64, P, i64, P]
    L.gini_dissim.argtypes = [P, P, i64, i32, i64, P, i32, P, i64, i64, P]
    L.gini_sumsq.argtypes = [P, P, i64, i64, i32, i64, P, P]
    L.gini_sum.argtypes = [P, P, i64, i64, i32, i64, P, P]
    L.gini_sammon_fwd.argtypes = [P, P, i64, i64, P, P, i32, i64, f64, ctypes.c_int, P, P]
    L.gini_sammon_bwd.argtypes = [P, P, i64, i64, P, P, i32, i64, f64, ctypes.c_int, P, P, i64, P, P]
    L.gini_sammon_step.argtypes = [P, P, i64, i64, i32, f64, ctypes.c_int, ctypes.POINTER(f64), P]
    L.gini_stress_fwd.argtypes = [P, P, i64, i64, P, i32, i64, f64, ctypes.c_int, P, P]
    L.gini_stress_bwd.argtypes = [P, P, i64, i64, P, i32, i64, f64, ctypes.c_int, P, P, i64, P, P]
    L.gini_stress_bwd_static.argtypes = [P, P, i64, i64, P, i32, i64, f64, ctypes.c_int, P, P, i64, P, P]
    L.gini_mds_solve.argtypes = [P, ctypes.POINTER(_Instance), i32, ctypes.POINTER(_Opts), P]
    L.gini_autotune.argtypes = [P, ctypes.POINTER(_Instance), i32, i32, ctypes.POINTER(_Opts), P]
    L.gini_select_nu.argtypes = [P, P, i64, i32, i64, P, i32, P, i64, ctypes.POINTER(_SelectOpts), P, i64, i64,
                                 P, P, P, P]
    L.gini_alternate_nu.argtypes = [P, P, i64, i32, i64, P, i32, P, i64, ctypes.POINTER(_AlternateOpts), P, i64,
                                    P, P, P, P]
    L.gini_classical_mds.argtypes = [P, P, i64, i64, i32, i32, f64, P, i64, P, P, P]
    L.gini_standardize.argtypes = [P, P, i64, i32, i64, P, i64, P, P]
    L.gini_profile_enable.argtypes = [P, ctypes.c_int]
    L.gini_profile_read.argtypes = [P, ctypes.POINTER(_Profile)]
    for fn in ("gini_create", "gini_rank", "gini_dissim", "gini_sumsq", "gini_sum", "gini_sammon_fwd",
               "gini_sammon_bwd", "gini_sammon_step", "gini_stress_fwd", "gini_stress_bwd", "gini_stress_bwd_static",
               "gini_mds_solve", "gini_autotune", "gini_select_nu", "gini_alternate_nu", "gini_classical_mds",
               "gini_standardize", "gini_profile_enable",
               "gini_profile_read"):
        getattr(L, fn).restype = ctypes.c_int
    return L


_lib = _load()
_ctxs = {}


def version() -> int:
    return int(_lib.gini_version())


class Context:
    """Owns one ``gini_ctx`` bound to a device."""

    def __init__(self, device: int = 0):
        h = ctypes.c_void_p()
        st = _lib.gini_create(ctypes.byref(h), int(device))
        if st != GINI_OK:
            raise GiniError(st, "gini_create failed")
        self.handle = h
        self.device = int(device)

    def check(self, st: int):
        if st != GINI_OK:
            raise GiniError(st, _lib.gini_last_error(self.handle).decode())

    def close(self):
        if self.handle:
            _lib.gini_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def context(device: int) -> Context:
    c = _ctxs.get(device)
    if c is None:
        c = Context(device)
        _ctxs[device] = c
    return c


def _dev_index(t: torch.Tensor) -> int:
    if not t.is_cuda:
        raise ValueError("tensors must live on the GPU (no CPU path exists)")
    return t.device.index if t.device.index is not None else torch.cuda.current_device()


def _mat(t: torch.Tensor, name: str, dtype=torch.float32) -> int:
    """Leading dimension of a row-major matrix whose rows do not overlap
    (unit column stride, row stride >= the row length); anything else -- an
    expanded or transposed view -- is rejected rather than read as dense."""
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if t.dim() != 2:
        raise ValueError(f"{name} must be 2-D")
    if t.shape[1] > 1 and t.stride(1) != 1:
        raise ValueError(f"{name} must have unit column stride")
    if t.shape[0] > 1 and int(t.stride(0)) < int(t.shape[1]):
        raise ValueError(f"{name} has row stride {t.stride(0)} < row length {t.shape[1]} (overlapping rows)")
    return int(t.stride(0)) if t.shape[0] > 1 else int(t.shape[1])


def _stream(dev: int) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _ptr(t: Optional[torch.Tensor]) -> Optional[ctypes.c_void_p]:
    return None if t is None else ctypes.c_void_p(t.data_ptr())


# ---------------------------------------------------------------- entry points
def gini_weight_table(d: int, nu: float):
    """Host FP32 table W[t-2], t = 2..2d, of the generalised Gini weights (no GPU)."""
    import numpy as np
    out = np.empty(max(2 * int(d) - 1, 1), dtype=np.float32)
    st = _lib.gini_weight_table(int(d), float(nu), ctypes.c_void_p(out.ctypes.data))
    if st != GINI_OK:
        raise GiniError(st, "gini_weight_table: invalid arguments")
    return out


def gini_rank(V: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Doubled midranks of every row of V (rows x d, FP32): int32 rows x d."""
    dev = _dev_index(V)
    ldv = _mat(V, "V")
    rows, d = V.shape
    if out is None:
        out = torch.empty((rows, d), dtype=torch.int32, device=V.device)
    ldr = _mat(out, "out", torch.int32)
    c = context(dev)
    c.check(_lib.gini_rank(c.handle, _ptr(V), rows, d, ldv, _ptr(out), ldr, _stream(dev)))
    return out


def padded_ld(n: int) -> int:
    """Leading dimension for an n x n dissimilarity matrix: rows start on 256
    bytes, so a tile row never straddles a cache line shared with the next
    tile (with only 16-byte alignment half the rows of an n = 10000 matrix
    would cost one extra 128-byte line per tile row)."""
    return (n + 63) // 64 * 64


def gini_dissim(X: torch.Tensor, nus: Sequence[float], out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Generalised Gini pseudo-distances of all pairs of rows of X for each nu.

    Returns a (len(nus), n, n) view (rows padded to a multiple of 64 floats)."""
    dev = _dev_index(X)
    ldx = _mat(X, "X")
    n, m = X.shape
    nus_h = (ctypes.c_double * len(nus))(*[float(v) for v in nus])
    if out is None:
        ld = padded_ld(n)
        buf = torch.empty((len(nus), n, ld), dtype=torch.float32, device=X.device)
        out = buf[:, :, :n]
    if out.dim() != 3 or out.shape[0] != len(nus) or out.shape[1] != n or out.shape[2] != n:
        raise ValueError("out must have shape (len(nus), n, n)")
    if out.dtype != torch.float32 or (n > 1 and out.stride(2) != 1):
        raise ValueError("out must be FP32 with unit column stride")
    if n > 1 and int(out.stride(1)) < n:
        raise ValueError(f"out has row stride {out.stride(1)} < n = {n} (overlapping rows)")
    if len(nus) > 1 and int(out.stride(0)) < n * int(out.stride(1)):
        raise ValueError("the matrices of out overlap")
    ldd = int(out.stride(1)) if n > 1 else 1
    stride_nu = int(out.stride(0))
    c = context(dev)
    c.check(_lib.gini_dissim(c.handle, _ptr(X), n, m, ldx, nus_h, len(nus), _ptr(out), ldd, stride_nu,
                             _stream(dev)))
    return out


def _sum_call(fn, Delta: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """A gini_sumsq-shaped call: (k, 2) device (hi, lo) pairs for an n x n
    matrix (k = 1) or a (k, n, n) stack."""
    dev = _dev_index(Delta)
    D3 = Delta.unsqueeze(0) if Delta.dim() == 2 else Delta
    if D3.dim() != 3 or D3.shape[1] != D3.shape[2]:
        raise ValueError("Delta must be n x n or k x n x n")
    if D3.dtype != torch.float32 or (D3.shape[1] > 1 and D3.stride(2) != 1):
        raise ValueError("Delta must be FP32 with unit column stride")
    k, n = int(D3.shape[0]), int(D3.shape[1])
    if n > 1 and int(D3.stride(1)) < n:
        raise ValueError(f"Delta has row stride {D3.stride(1)} < n = {n} (overlapping rows)")
    if k > 1 and int(D3.stride(0)) < n * int(D3.stride(1)):
        raise ValueError("the matrices of a Delta stack overlap")
    ldd = int(D3.stride(1)) if n > 1 else 1
    if out is None:
        out = torch.empty((k, 2), dtype=torch.float32, device=Delta.device)
    if out.dtype != torch.float32 or not out.is_contiguous() or out.numel() != 2 * k:
        raise ValueError("out must be a contiguous FP32 tensor of 2*k elements")
    c = context(dev)
    c.check(fn(c.handle, _ptr(D3), n, ldd, k, int(D3.stride(0)), _ptr(out), _stream(dev)))
    return out


def gini_sumsq(Delta: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """sum_{i<j} Delta_ij^2 (Kruskal normaliser) of an n x n matrix or a (k, n, n)
    stack: a (k, 2) device tensor of (hi, lo) pairs."""
    return _sum_call(_lib.gini_sumsq, Delta, out)


def gini_sum(Delta: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """sum_{i<j} Delta_ij (Sammon normaliser), shaped as gini_sumsq."""
    return _sum_call(_lib.gini_sum, Delta, out)


def _check_pair(Delta: torch.Tensor, Z: torch.Tensor):
    if Delta.dim() != 2 or Delta.shape[0] != Delta.shape[1]:
        raise ValueError("Delta must be n x n")
    if Z.dim() != 2 or Z.shape[0] != Delta.shape[0]:
        raise ValueError("Z must be n x p with the n of Delta")


def gini_stress_fwd(Delta: torch.Tensor, Z: torch.Tensor, nu: float, latent: int = LATENT_GINI,
                    out_sigma: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Raw stress; returns the device pair (hi, lo) with sigma = hi + lo."""
    dev = _dev_index(Delta)
    _check_pair(Delta, Z)
    ldd = _mat(Delta, "Delta")
    ldz = _mat(Z, "Z")
    n, p = Z.shape
    if out_sigma is None:
        out_sigma = torch.empty(2, dtype=torch.float32, device=Delta.device)
    c = context(dev)
    c.check(_lib.gini_stress_fwd(c.handle, _ptr(Delta), n, ldd, _ptr(Z), p, ldz, float(nu), int(latent),
                                 _ptr(out_sigma), _stream(dev)))
    return out_sigma


def gini_stress_bwd(Delta: torch.Tensor, Z: torch.Tensor, nu: float, latent: int = LATENT_GINI,
                    grad_out: Optional[torch.Tensor] = None, gradZ: Optional[torch.Tensor] = None,
                    out_sigma: Optional[torch.Tensor] = None, want_sigma: bool = True):
    """Gradient of the raw stress (and the stress) in one pass: (gradZ, sigma pair or None)."""
    dev = _dev_index(Delta)
    _check_pair(Delta, Z)
    ldd = _mat(Delta, "Delta")
    ldz = _mat(Z, "Z")
    n, p = Z.shape
    if gradZ is None:
        gradZ = torch.empty((n, p), dtype=torch.float32, device=Delta.device)
    ldg = _mat(gradZ, "gradZ")
    if out_sigma is None and want_sigma:
        out_sigma = torch.empty(2, dtype=torch.float32, device=Delta.device)
    if grad_out is not None and (grad_out.dtype != torch.float32 or grad_out.numel() != 1):
        raise ValueError("grad_out must be a one-element FP32 tensor")
    c = context(dev)
    c.check(_lib.gini_stress_bwd(c.handle, _ptr(Delta), n, ldd, _ptr(Z), p, ldz, float(nu), int(latent),
                                 _ptr(grad_out), _ptr(gradZ), ldg, _ptr(out_sigma), _stream(dev)))
    return gradZ, out_sigma


def gini_stress_bwd_static(Delta: torch.Tensor, Z: torch.Tensor, nu: float, latent: int = LATENT_GINI,
                           grad_out: Optional[torch.Tensor] = None, gradZ: Optional[torch.Tensor] = None,
                           out_sigma: Optional[torch.Tensor] = None):
    """gini_stress_bwd through the entry point that allocates no device memory
    (its scratch is a static device array per GPU): (gradZ, sigma pair).  With
    gradZ and out_sigma passed in, nothing is allocated on this call at all."""
    dev = _dev_index(Delta)
    _check_pair(Delta, Z)
    ldd = _mat(Delta, "Delta")
    ldz = _mat(Z, "Z")
    n, p = Z.shape
    if gradZ is None:
        gradZ = torch.empty((n, p), dtype=torch.float32, device=Delta.device)
    ldg = _mat(gradZ, "gradZ")
    if out_sigma is None:
        out_sigma = torch.empty(2, dtype=torch.float32, device=Delta.device)
    if grad_out is not None and (grad_out.dtype != torch.float32 or grad_out.numel() != 1):
        raise ValueError("grad_out must be a one-element FP32 tensor")
    c = context(dev)
    c.check(_lib.gini_stress_bwd_static(c.handle, _ptr(Delta), n, ldd, _ptr(Z), p, ldz, float(nu), int(latent),
                                        _ptr(grad_out), _ptr(gradZ), ldg, _ptr(out_sigma), _stream(dev)))
    return gradZ, out_sigma


def _dsum(t: Optional[torch.Tensor], Delta: torch.Tensor) -> torch.Tensor:
    if t is None:
        return gini_sum(Delta)[0]
    if t.dtype != torch.float32 or t.numel() < 2 or not t.is_contiguous():
        raise ValueError("delta_sum must be a contiguous FP32 (hi, lo) pair")
    return t


def gini_sammon_fwd(Delta: torch.Tensor, Z: torch.Tensor, nu: float, latent: int = LATENT_GINI,
                    delta_sum: Optional[torch.Tensor] = None, out_sigma: Optional[torch.Tensor] = None):
    """Sammon stress (hi, lo); delta_sum from gini_sum (computed when omitted)."""
    dev = _dev_index(Delta)
    _check_pair(Delta, Z)
    ldd = _mat(Delta, "Delta")
    ldz = _mat(Z, "Z")
    n, p = Z.shape
    ds = _dsum(delta_sum, Delta)
    if out_sigma is None:
        out_sigma = torch.empty(2, dtype=torch.float32, device=Delta.device)
    c = context(dev)
    c.check(_lib.gini_sammon_fwd(c.handle, _ptr(Delta), n, ldd, _ptr(ds), _ptr(Z), p, ldz, float(nu), int(latent),
                                 _ptr(out_sigma), _stream(dev)))
    return out_sigma


def gini_sammon_bwd(Delta: torch.Tensor, Z: torch.Tensor, nu: float, latent: int = LATENT_GINI,
                    delta_sum: Optional[torch.Tensor] = None, grad_out: Optional[torch.Tensor] = None,
                    gradZ: Optional[torch.Tensor] = None, out_sigma: Optional[torch.Tensor] = None):
    """Gradient of the Sammon stress and the stress in one pass: (gradZ, sigma pair)."""
    dev = _dev_index(Delta)
    _check_pair(Delta, Z)
    ldd = _mat(Delta, "Delta")
    ldz = _mat(Z, "Z")
    n, p = Z.shape
    ds = _dsum(delta_sum, Delta)
    if gradZ is None:
        gradZ = torch.empty((n, p), dtype=torch.float32, device=Delta.device)
    ldg = _mat(gradZ, "gradZ")
    if out_sigma is None:
        out_sigma = torch.empty(2, dtype=torch.float32, device=Delta.device)
    if grad_out is not None and (grad_out.dtype != torch.float32 or grad_out.numel() != 1):
        raise ValueError("grad_out must be a one-element FP32 tensor")
    c = context(dev)
    c.check(_lib.gini_sammon_bwd(c.handle, _ptr(Delta), n, ldd, _ptr(ds), _ptr(Z), p, ldz, float(nu), int(latent),
                                 _ptr(grad_out), _ptr(gradZ), ldg, _ptr(out_sigma), _stream(dev)))
    return gradZ, out_sigma


def gini_sammon_step(Delta: torch.Tensor, p: int, nu: float, latent: int = LATENT_GINI) -> float:
    """A descent step under which the Sammon stress does not increase."""
    dev = _dev_index(Delta)
    ldd = _mat(Delta, "Delta")
    eta = ctypes.c_double(0.0)
    c = context(dev)
    c.check(_lib.gini_sammon_step(c.handle, _ptr(Delta), int(Delta.shape[0]), ldd, int(p), float(nu), int(latent),
                                  ctypes.byref(eta), _stream(dev)))
    return float(eta.value)


@dataclass
class Instance:
    """One descent problem for gini_mds_solve (Z is updated in place)."""
    Delta: torch.Tensor
    Z: torch.Tensor
    nu: float
    latent: int = LATENT_GINI
    eta: float = 0.0
    sigma_hist: Optional[torch.Tensor] = None
    delta_sumsq: Optional[torch.Tensor] = None   # (hi, lo) from gini_sumsq; needed by ks_hist
    ks_hist: Optional[torch.Tensor] = None       # per-iteration Kruskal stress
    loss: int = LOSS_RAW
    delta_sum: Optional[torch.Tensor] = None     # (hi, lo) from gini_sum; needed by LOSS_SAMMON


def _hist_ptr(t: Optional[torch.Tensor], name: str):
    if t is None:
        return None
    if t.dtype != torch.float32 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous FP32 tensor")
    return t.data_ptr()


def _instances(insts: Sequence[Instance]):
    arr = (_Instance * len(insts))()
    dev = None
    for k, I in enumerate(insts):
        d = _dev_index(I.Delta)
        if dev is None:
            dev = d
        elif d != dev or _dev_index(I.Z) != dev:
            raise ValueError("all instances must live on one device")
        _check_pair(I.Delta, I.Z)
        a = arr[k]
        a.n, a.p = int(I.Z.shape[0]), int(I.Z.shape[1])
        a.loss = int(I.loss)
        if I.delta_sum is not None and I.delta_sum.numel() < 2:
            raise ValueError("delta_sum must hold (hi, lo)")
        a.delta_sum = _hist_ptr(I.delta_sum, "delta_sum")
        a.Delta, a.ldd = I.Delta.data_ptr(), _mat(I.Delta, "Delta")
        a.Z, a.ldz = I.Z.data_ptr(), _mat(I.Z, "Z")
        a.nu, a.latent, a.eta = float(I.nu), int(I.latent), float(I.eta)
        a.sigma_hist = _hist_ptr(I.sigma_hist, "sigma_hist")
        a.ks_hist = _hist_ptr(I.ks_hist, "ks_hist")
        if I.delta_sumsq is not None and I.delta_sumsq.numel() < 2:
            raise ValueError("delta_sumsq must hold (hi, lo)")
        a.delta_sumsq = _hist_ptr(I.delta_sumsq, "delta_sumsq")
    return arr, dev


def gini_mds_solve(insts: Sequence[Instance], iters: int, flags: int = SOLVE_PERSISTENT, tile: int = 0,
                   grid: int = 0) -> None:
    """Fixed-step gradient descent on every instance, on the current stream
    (the persistent mode and CHECK_FINITE synchronise it; the others only
    enqueue)."""
    for I in insts:
        for h, name in ((I.sigma_hist, "sigma_hist"), (I.ks_hist, "ks_hist")):
            if h is not None and h.numel() < iters:
                raise ValueError(f"{name} shorter than iters")
    arr, dev = _instances(insts)
    opts = _Opts(int(iters), int(flags), int(tile), int(grid))
    c = context(dev)
    c.check(_lib.gini_mds_solve(c.handle, arr, len(insts), ctypes.byref(opts), _stream(dev)))


def gini_autotune(insts: Sequence[Instance], probe_iters: int = 3) -> dict:
    """Measure candidate (mode, tile, grid) choices; returns the fastest."""
    arr, dev = _instances(insts)
    best = _Opts(0, 0, 0, 0)
    c = context(dev)
    c.check(_lib.gini_autotune(c.handle, arr, len(insts), int(probe_iters), ctypes.byref(best), _stream(dev)))
    return {"flags": int(best.flags), "tile": int(best.tile), "grid": int(best.grid)}


def gini_select_nu(X: torch.Tensor, nus: Sequence[float], Z0: torch.Tensor, iters: int, folds: int = 1,
                   latent: int = LATENT_GINI, flags: int = SOLVE_BATCHED, tile: int = 0,
                   Z_out: Optional[torch.Tensor] = None):
    """Algorithm 1: fit every nu on every fold, score each fit by its Kruskal
    stress with the Euclidean latent distance, return nu* = argmin of the
    fold mean.  Returns (best index, ks_mean[n_nu], ks_fold[n_nu, folds],
    Z_out[n_nu, n, p]); synchronises the stream."""
    import numpy as np
    dev = _dev_index(X)
    if _dev_index(Z0) != dev:
        raise ValueError("X and Z0 must live on one device")
    ldx = _mat(X, "X")
    ldz0 = _mat(Z0, "Z0")
    n, m = X.shape
    if Z0.shape[0] != n:
        raise ValueError("Z0 must have the rows of X")
    p = int(Z0.shape[1])
    k = len(nus)
    if Z_out is None:
        Z_out = torch.empty((k, n, p), dtype=torch.float32, device=X.device)
    if Z_out.dim() != 3 or tuple(Z_out.shape) != (k, n, p) or Z_out.dtype != torch.float32:
        raise ValueError("Z_out must be an FP32 tensor of shape (len(nus), n, p)")
    if p > 1 and Z_out.stride(2) != 1:
        raise ValueError("Z_out must have unit column stride")
    if n > 1 and int(Z_out.stride(1)) < p:
        raise ValueError("Z_out has overlapping rows")
    if k > 1 and int(Z_out.stride(0)) < n * int(Z_out.stride(1)):
        raise ValueError("the configurations of Z_out overlap")
    ldzo = int(Z_out.stride(1)) if n > 1 else p
    nus_h = (ctypes.c_double * k)(*[float(v) for v in nus])
    ks_mean = np.zeros(k, dtype=np.float64)
    ks_fold = np.zeros((k, int(folds)), dtype=np.float64)
    best = ctypes.c_int32(-1)
    opts = _SelectOpts(int(iters), p, int(latent), int(folds), int(flags), int(tile))
    c = context(dev)
    c.check(_lib.gini_select_nu(c.handle, _ptr(X), n, m, ldx, nus_h, k, _ptr(Z0), ldz0, ctypes.byref(opts),
                                _ptr(Z_out), ldzo, int(Z_out.stride(0)), ctypes.c_void_p(ks_mean.ctypes.data),
                                ctypes.c_void_p(ks_fold.ctypes.data), ctypes.byref(best), _stream(dev)))
    return int(best.value), ks_mean, ks_fold, Z_out


def gini_alternate_nu(X: torch.Tensor, nus: Sequence[float], Z0: torch.Tensor, iters: int, rounds: int = 3,
                      init: Optional[int] = None, latent: int = LATENT_GINI, flags: int = SOLVE_BATCHED,
                      tile: int = 0, Z_out: Optional[torch.Tensor] = None):
    """Algorithm 2's alternation: Sammon fit at the current nu, then move to the
    nu whose dissimilarities the fit matches best (Kruskal stress, Euclidean
    latent distance).  init defaults to the index of nu = 2 (else 0).  Returns
    (best index, nu index fitted per round, ks[rounds, n_nu], Z_out)."""
    import numpy as np
    dev = _dev_index(X)
    if _dev_index(Z0) != dev:
        raise ValueError("X and Z0 must live on one device")
    ldx = _mat(X, "X")
    ldz0 = _mat(Z0, "Z0")
    n, m = X.shape
    if Z0.shape[0] != n:
        raise ValueError("Z0 must have the rows of X")
    p = int(Z0.shape[1])
    k = len(nus)
    if init is None:
        init = [float(v) for v in nus].index(2.0) if 2.0 in [float(v) for v in nus] else 0
    if Z_out is None:
        Z_out = torch.empty((n, p), dtype=torch.float32, device=X.device)
    ldzo = _mat(Z_out, "Z_out")
    nus_h = (ctypes.c_double * k)(*[float(v) for v in nus])
    hist = np.zeros(int(rounds), dtype=np.int32)
    ks = np.zeros((int(rounds), k), dtype=np.float64)
    best = ctypes.c_int32(-1)
    opts = _AlternateOpts(int(iters), p, int(latent), int(rounds), int(init), int(flags), int(tile))
    c = context(dev)
    c.check(_lib.gini_alternate_nu(c.handle, _ptr(X), n, m, ldx, nus_h, k, _ptr(Z0), ldz0, ctypes.byref(opts),
                                   _ptr(Z_out), ldzo, ctypes.c_void_p(hist.ctypes.data),
                                   ctypes.c_void_p(ks.ctypes.data), ctypes.byref(best), _stream(dev)))
    return int(best.value), hist, ks, Z_out


def gini_classical_mds(Delta: torch.Tensor, p: int, max_iters: int = 300, tol: float = 1e-7,
                       Z: Optional[torch.Tensor] = None):
    """Classical MDS of Delta: (Z[n, p], eigenvalues[p], iterations used)."""
    import numpy as np
    dev = _dev_index(Delta)
    if Delta.dim() != 2 or Delta.shape[0] != Delta.shape[1]:
        raise ValueError("Delta must be n x n")
    ldd = _mat(Delta, "Delta")
    n = int(Delta.shape[0])
    if Z is None:
        Z = torch.empty((n, int(p)), dtype=torch.float32, device=Delta.device)
    ldz = _mat(Z, "Z")
    ev = np.zeros(int(p), dtype=np.float64)
    it = ctypes.c_int32(0)
    c = context(dev)
    c.check(_lib.gini_classical_mds(c.handle, _ptr(Delta), n, ldd, int(p), int(max_iters), float(tol), _ptr(Z), ldz,
                                    ctypes.c_void_p(ev.ctypes.data), ctypes.byref(it), _stream(dev)))
    return Z, ev, int(it.value)


def gini_standardize(X: torch.Tensor, out: Optional[torch.Tensor] = None, stats: bool = False):
    """Columns centred to zero median and scaled to unit (population) variance.
    Returns Y, or (Y, (m, 2) tensor of (median, sd)) with stats=True."""
    dev = _dev_index(X)
    ldx = _mat(X, "X")
    n, m = X.shape
    if out is None:
        out = torch.empty((n, m), dtype=torch.float32, device=X.device)
    ldy = _mat(out, "out")
    st = torch.empty((m, 2), dtype=torch.float32, device=X.device) if stats else None
    c = context(dev)
    c.check(_lib.gini_standardize(c.handle, _ptr(X), n, m, ldx, _ptr(out), ldy, _ptr(st), _stream(dev)))
    return (out, st) if stats else out


def gini_profile_enable(device: int = 0, enable: bool = True) -> None:
    """Start or stop per-launch kernel timing on the device's context (clears totals)."""
    c = context(device)
    c.check(_lib.gini_profile_enable(c.handle, 1 if enable else 0))


def gini_profile_read(device: int = 0) -> dict:
    """Totals of the kernel timings recorded since the last read."""
    c = context(device)
    out = _Profile()
    c.check(_lib.gini_profile_read(c.handle, ctypes.byref(out)))
    return {f: getattr(out, f) for f, _ in _Profile._fields_}


class GiniStress(torch.autograd.Function):
    """sigma(Z) = sum_{i<j} (delta(Z_i - Z_j) - Delta_ij)^2 with a hand-written
    backward: the forward makes ONE pass over Delta that yields both the stress
    and its gradient (latent ranks held fixed); the backward scales the saved
    gradient by the incoming one."""

    @staticmethod
    def forward(ctx, Delta, Z, nu, latent=LATENT_GINI):
        if Z.requires_grad:
            G, sig = gini_stress_bwd(Delta, Z.detach(), nu, latent)
            ctx.save_for_backward(G)
        else:
            sig = gini_stress_fwd(Delta, Z, nu, latent)
            ctx.save_for_backward(None)
        return sig[0] + sig[1]

    @staticmethod
    def backward(ctx, grad_out):
        (G,) = ctx.saved_tensors
        if G is None:
            return None, None, None, None
        return None, G * grad_out, None, None


def stress(Delta: torch.Tensor, Z: torch.Tensor, nu: float, latent: int = LATENT_GINI) -> torch.Tensor:
    return GiniStress.apply(Delta, Z, nu, latent)


class GiniSammon(torch.autograd.Function):
    """Sammon stress of Z against Delta with a hand-written backward (one pass
    over Delta for the stress and its gradient, latent ranks held fixed)."""

    @staticmethod
    def forward(ctx, Delta, Z, nu, latent=LATENT_GINI, delta_sum=None):
        if Z.requires_grad:
            G, sig = gini_sammon_bwd(Delta, Z.detach(), nu, latent, delta_sum)
            ctx.save_for_backward(G)
        else:
            sig = gini_sammon_fwd(Delta, Z, nu, latent, delta_sum)
            ctx.save_for_backward(None)
        return sig[0] + sig[1]

    @staticmethod
    def backward(ctx, grad_out):
        (G,) = ctx.saved_tensors
        if G is None:
            return None, None, None, None, None
        return None, G * grad_out, None, None, None

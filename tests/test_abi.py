"""Host-side checks of the C ABI: every declared symbol is exported, argument
validation fails before any GPU work, and the host weight table agrees with
the oracle.  None of these tests launches a kernel."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ginimds.h")
LIB = os.path.join(ROOT, "paper_2605_25124_amd", "libginimds.so")

EINVAL, EUNSUPPORTED = 1, 5


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gini_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libginimds.so is not built (run python -m paper_2605_25124_amd.build)")
    return ctypes.CDLL(LIB)


@pytest.fixture(scope="module")
def gm():
    from paper_2605_25124_amd import ginimds
    return ginimds


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert {"gini_create", "gini_destroy", "gini_last_error", "gini_rank", "gini_dissim", "gini_stress_fwd",
            "gini_stress_bwd", "gini_mds_solve", "gini_autotune", "gini_weight_table"} <= set(names)
    for n in names:
        assert hasattr(lib, n), n


def test_status_strings_and_version(gm):
    L = gm._lib
    assert L.gini_status_string(1) == b"GINI_EINVAL"
    assert L.gini_status_string(5) == b"GINI_EUNSUPPORTED"
    assert gm.version() >= 10000


def _ctx(gm):
    h = ctypes.c_void_p()
    assert gm._lib.gini_create(ctypes.byref(h), 0) == 0
    return h


def _err(gm, h):
    return gm._lib.gini_last_error(h).decode()


def test_create_rejects_negative_device(gm):
    h = ctypes.c_void_p()
    assert gm._lib.gini_create(ctypes.byref(h), -1) == EINVAL
    assert gm._lib.gini_create(None, 0) == EINVAL


def test_dissim_validation(gm):
    L, h = gm._lib, _ctx(gm)
    X = ctypes.c_void_p(0x1000)
    D = ctypes.c_void_p(0x2000)
    nu = (ctypes.c_double * 2)(2.0, 3.0)
    bad_nu = (ctypes.c_double * 1)(1.0)
    nan_nu = (ctypes.c_double * 1)(float("nan"))
    cases = [
        ((h, X, 0, 4, 4, nu, 1, D, 4, 0, None), "n = 0"),
        ((h, X, 10, 0, 4, nu, 1, D, 10, 0, None), "m = 0"),
        ((h, X, 10, 5000, 5000, nu, 1, D, 10, 0, None), "m = 5000"),
        ((h, X, 10, 4, 3, nu, 1, D, 10, 0, None), "ldx"),
        ((h, X, 10, 4, 4, nu, 1, D, 9, 0, None), "ldd"),
        ((h, X, 10, 4, 4, bad_nu, 1, D, 10, 0, None), "nu[0]"),
        ((h, X, 10, 4, 4, nan_nu, 1, D, 10, 0, None), "nu[0]"),
        ((h, X, 10, 4, 4, nu, 2, D, 10, 50, None), "stride_nu"),
        ((h, X, 10, 4, 4, nu, 0, D, 10, 0, None), "n_nu"),
        ((h, None, 10, 4, 4, nu, 1, D, 10, 0, None), "non-null"),
    ]
    for args, frag in cases:
        assert L.gini_dissim(*args) == EINVAL, frag
        assert frag.split()[0] in _err(gm, h), (frag, _err(gm, h))
    L.gini_destroy(h)


def test_stress_validation(gm):
    L, h = gm._lib, _ctx(gm)
    D, Z, G, S = (ctypes.c_void_p(a) for a in (0x1000, 0x2000, 0x3000, 0x4000))
    f = L.gini_stress_fwd
    assert f(h, D, 1, 1, Z, 2, 2, 2.0, 0, S, None) == EINVAL          # n < 2
    assert f(h, D, 10, 9, Z, 2, 2, 2.0, 0, S, None) == EINVAL         # ldd < n
    assert f(h, D, 10, 10, Z, 1, 1, 2.0, 0, S, None) == EINVAL        # Gini with p = 1
    assert "p >= 2" in _err(gm, h)
    assert f(h, D, 10, 10, Z, 9, 9, 2.0, 1, S, None) == EINVAL        # p > 8
    assert f(h, D, 10, 10, Z, 2, 2, 0.5, 0, S, None) == EINVAL        # nu <= 1
    assert f(h, D, 10, 10, Z, 2, 2, float("inf"), 0, S, None) == EINVAL
    assert f(h, D, 10, 10, Z, 3, 2, 2.0, 0, S, None) == EINVAL        # ldz < p
    assert f(h, D, 10, 10, Z, 2, 2, 2.0, 7, S, None) == EINVAL        # bad latent
    assert f(h, D, 10, 10, Z, 2, 2, 2.0, 0, None, None) == EINVAL     # no output
    b = L.gini_stress_bwd
    assert b(h, D, 10, 10, Z, 2, 2, 2.0, 0, None, None, 2, S, None) == EINVAL   # gradZ null
    assert b(h, D, 10, 10, Z, 2, 2, 2.0, 0, None, G, 1, S, None) == EINVAL      # ldg < p
    L.gini_destroy(h)


def test_rank_validation(gm):
    L, h = gm._lib, _ctx(gm)
    V, T = ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000)
    assert L.gini_rank(h, V, 4, 0, 4, T, 4, None) == EINVAL
    assert L.gini_rank(h, V, 4, 5, 4, T, 5, None) == EINVAL
    assert L.gini_rank(h, V, 4, 5, 5, T, 4, None) == EINVAL
    assert L.gini_rank(h, V, -1, 5, 5, T, 5, None) == EINVAL
    assert L.gini_rank(h, None, 0, 5, 5, None, 5, None) == 0       # empty input is a no-op
    L.gini_destroy(h)


def test_solve_validation(gm):
    L, h = gm._lib, _ctx(gm)
    Inst = gm._Instance
    Opts = gm._Opts

    def inst(n=10, p=2, Z=0x2000, latent=0, nu=2.0, hist=None, res=0):
        a = Inst()
        a.n, a.p, a.loss = n, p, res
        a.Delta, a.ldd, a.Z, a.ldz = 0x1000, n, Z, p
        a.nu, a.latent, a.eta, a.sigma_hist = nu, latent, 0.0, hist
        return a

    def run(insts, opts):
        arr = (Inst * len(insts))(*insts)
        return L.gini_mds_solve(h, arr, len(insts), ctypes.byref(opts), None)

    ok = Opts(10, gm.SOLVE_PERSISTENT, 0, 0)
    assert run([inst(n=1)], ok) == EINVAL
    assert run([inst(p=1)], ok) == EINVAL
    assert run([inst(nu=1.0)], ok) == EINVAL
    assert run([inst(res=3)], ok) == EINVAL
    assert run([inst(Z=0x2000), inst(Z=0x2000)], ok) == EINVAL
    assert "share Z" in _err(gm, h)
    assert run([inst(Z=0x2000, hist=0x5000), inst(Z=0x3000, hist=0x5000)], ok) == EINVAL
    assert run([inst(Z=0x2000, p=2), inst(Z=0x3000, p=3)], ok) == EUNSUPPORTED
    sam = inst(res=1)                                       # Sammon loss
    assert run([sam], ok) == EINVAL and "delta_sum" in _err(gm, h)
    sam.delta_sum = 0x8000
    assert run([sam], ok) == EINVAL and "eta" in _err(gm, h)
    sam.eta = 0.5
    sam.ks_hist, sam.delta_sumsq = 0x6000, 0x7000
    assert run([sam], ok) == EINVAL and "raw stress" in _err(gm, h)
    sam.ks_hist = None
    raw = inst(Z=0x3000)
    assert run([sam, raw], ok) == EUNSUPPORTED and "loss" in _err(gm, h)
    k = inst()
    k.ks_hist = 0x6000                                    # Kruskal history without its normaliser
    assert run([k], ok) == EINVAL
    assert "delta_sumsq" in _err(gm, h)
    k1, k2 = inst(Z=0x2000), inst(Z=0x3000)
    k1.ks_hist = k2.ks_hist = 0x6000
    k1.delta_sumsq = k2.delta_sumsq = 0x7000
    assert run([k1, k2], ok) == EINVAL
    assert "share ks_hist" in _err(gm, h)
    assert run([inst()], Opts(-1, gm.SOLVE_PERSISTENT, 0, 0)) == EINVAL
    assert run([inst()], Opts(5, gm.SOLVE_PERSISTENT | gm.SOLVE_PLAIN, 0, 0)) == EINVAL
    assert run([inst()], Opts(5, gm.SOLVE_PERSISTENT, 100, 0)) == EINVAL
    assert run([inst()], Opts(5, 1 << 10, 0, 0)) == EINVAL
    assert run([inst()], Opts(5, gm.SOLVE_SPLIT, 0, 0)) == EINVAL and "SPLIT" in _err(gm, h)
    assert run([inst()], Opts(5, gm.SOLVE_BATCHED, 0, 512)) == EINVAL and "reduction" in _err(gm, h)
    assert run([inst()], Opts(5, gm.SOLVE_PERSISTENT | gm.SOLVE_SPLIT, 0, 0)) == EINVAL
    assert L.gini_mds_solve(h, None, 1, ctypes.byref(ok), None) == EINVAL
    L.gini_destroy(h)


def test_sumsq_validation(gm):
    L, h = gm._lib, _ctx(gm)
    D = ctypes.c_void_p(0x1000)
    out = ctypes.c_void_p(0x2000)
    cases = [((h, D, 0, 4, 1, 0, out, None), "n = 0"),
             ((h, D, 10, 9, 1, 0, out, None), "ldd"),
             ((h, None, 10, 10, 1, 0, out, None), "non-null"),
             ((h, D, 10, 10, 1, 0, None, None), "non-null"),
             ((h, D, 10, 10, 0, 100, out, None), "n_mat"),
             ((h, D, 10, 10, 70000, 100, out, None), "n_mat"),
             ((h, D, 10, 10, 2, 99, out, None), "stride")]
    for args, msg in cases:
        assert L.gini_sumsq(*args) == EINVAL, msg
        assert msg in _err(gm, h), (msg, _err(gm, h))
    assert L.gini_sumsq(None, D, 10, 10, 1, 0, out, None) == EINVAL
    L.gini_destroy(h)


def test_sammon_entry_validation(gm):
    L, h = gm._lib, _ctx(gm)
    D, Z, G, o, ds = (ctypes.c_void_p(v) for v in (0x1000, 0x2000, 0x3000, 0x4000, 0x5000))
    assert L.gini_sammon_fwd(h, D, 10, 10, None, Z, 2, 2, 2.0, 0, o, None) == EINVAL
    assert "delta_sum" in _err(gm, h)
    assert L.gini_sammon_bwd(h, D, 10, 10, None, Z, 2, 2, 2.0, 0, None, G, 2, o, None) == EINVAL
    assert L.gini_sammon_fwd(h, D, 1, 10, ds, Z, 2, 2, 2.0, 0, o, None) == EINVAL      # n < 2
    assert L.gini_sammon_fwd(h, D, 10, 10, ds, Z, 1, 2, 2.0, 0, o, None) == EINVAL     # Gini latent, p = 1
    eta = ctypes.c_double()
    assert L.gini_sammon_step(h, D, 1, 1, 2, 2.0, 0, ctypes.byref(eta), None) == EINVAL
    assert L.gini_sammon_step(h, D, 10, 9, 2, 2.0, 0, ctypes.byref(eta), None) == EINVAL
    assert L.gini_sammon_step(h, D, 10, 10, 2, 0.9, 0, ctypes.byref(eta), None) == EINVAL
    assert L.gini_sammon_step(h, D, 10, 10, 2, 2.0, 0, None, None) == EINVAL
    assert L.gini_sum(h, D, 0, 4, 1, 0, o, None) == EINVAL
    assert L.gini_sum(h, D, 10, 9, 1, 0, o, None) == EINVAL
    L.gini_destroy(h)


def test_alternate_validation(gm):
    L, h = gm._lib, _ctx(gm)
    X, Z0, Zo = ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000), ctypes.c_void_p(0x3000)
    nu = (ctypes.c_double * 2)(2.0, 3.0)
    hist = (ctypes.c_int32 * 3)()
    best = ctypes.c_int32()

    def run(n=100, opts=None, Zout=Zo, nus=nu):
        o = opts or gm._AlternateOpts(10, 2, 0, 3, 0, gm.SOLVE_BATCHED, 0)
        return L.gini_alternate_nu(h, X, n, 4, 4, nus, 2, Z0, 2, ctypes.byref(o), Zout, 2, hist, None,
                                   ctypes.byref(best), None)

    assert run(n=1) == EINVAL
    assert run(opts=gm._AlternateOpts(0, 2, 0, 3, 0, gm.SOLVE_BATCHED, 0)) == EINVAL and "iters" in _err(gm, h)
    assert run(opts=gm._AlternateOpts(10, 2, 0, 0, 0, gm.SOLVE_BATCHED, 0)) == EINVAL and "rounds" in _err(gm, h)
    assert run(opts=gm._AlternateOpts(10, 2, 0, 3, 2, gm.SOLVE_BATCHED, 0)) == EINVAL and "init" in _err(gm, h)
    assert run(opts=gm._AlternateOpts(10, 1, 0, 3, 0, gm.SOLVE_BATCHED, 0)) == EINVAL
    assert run(Zout=None) == EINVAL
    assert run(nus=(ctypes.c_double * 2)(2.0, 1.0)) == EINVAL
    L.gini_destroy(h)


def test_classical_mds_validation(gm):
    L, h = gm._lib, _ctx(gm)
    D, Z = ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000)
    assert L.gini_classical_mds(h, D, 1, 1, 1, 10, 1e-7, Z, 1, None, None, None) == EINVAL
    assert L.gini_classical_mds(h, D, 10, 9, 2, 10, 1e-7, Z, 2, None, None, None) == EINVAL
    assert L.gini_classical_mds(h, D, 10, 10, 0, 10, 1e-7, Z, 2, None, None, None) == EINVAL
    assert L.gini_classical_mds(h, D, 10, 10, 9, 10, 1e-7, Z, 9, None, None, None) == EINVAL   # p > 8
    assert L.gini_classical_mds(h, D, 3, 3, 3, 10, 1e-7, Z, 3, None, None, None) == EINVAL     # p > n - 1
    assert L.gini_classical_mds(h, D, 10, 10, 2, 0, 1e-7, Z, 2, None, None, None) == EINVAL
    assert L.gini_classical_mds(h, D, 10, 10, 2, 10, -1.0, Z, 2, None, None, None) == EINVAL
    assert L.gini_classical_mds(h, D, 10, 10, 2, 10, 1e-7, Z, 1, None, None, None) == EINVAL
    assert L.gini_classical_mds(h, None, 10, 10, 2, 10, 1e-7, Z, 2, None, None, None) == EINVAL
    L.gini_destroy(h)


def test_standardize_validation(gm):
    L, h = gm._lib, _ctx(gm)
    X, Y = ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000)
    assert L.gini_standardize(h, X, 0, 3, 3, Y, 3, None, None) == EINVAL
    assert L.gini_standardize(h, X, 10, 0, 3, Y, 3, None, None) == EINVAL
    assert L.gini_standardize(h, X, 10, 4, 3, Y, 4, None, None) == EINVAL
    assert L.gini_standardize(h, X, 10, 4, 4, Y, 3, None, None) == EINVAL
    assert L.gini_standardize(h, X, 10, 4, 4, X, 5, None, None) == EINVAL and "in place" in _err(gm, h)
    assert L.gini_standardize(h, None, 10, 4, 4, Y, 4, None, None) == EINVAL
    L.gini_destroy(h)


def test_select_validation(gm):
    L, h = gm._lib, _ctx(gm)
    X, Z0, Zo = ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000), ctypes.c_void_p(0x3000)
    nu = (ctypes.c_double * 2)(2.0, 3.0)
    bad = (ctypes.c_double * 2)(2.0, 0.5)
    km = (ctypes.c_double * 2)()
    best = ctypes.c_int32()

    def run(n=100, m=4, nus=nu, n_nu=2, opts=None, Zout=Zo, stride=1000, ldz0=2):
        o = opts or gm._SelectOpts(10, 2, 0, 2, gm.SOLVE_BATCHED, 0)
        return L.gini_select_nu(h, X, n, m, m, nus, n_nu, Z0, ldz0, ctypes.byref(o), Zout, 2, stride, km, None,
                                ctypes.byref(best), None)

    assert run(nus=bad) == EINVAL and "nu[1]" in _err(gm, h)
    assert run(opts=gm._SelectOpts(10, 2, 0, 60, gm.SOLVE_BATCHED, 0)) == EINVAL and "fold" in _err(gm, h)
    assert run(opts=gm._SelectOpts(0, 2, 0, 2, gm.SOLVE_BATCHED, 0)) == EINVAL and "iters" in _err(gm, h)
    assert run(opts=gm._SelectOpts(10, 1, 0, 2, gm.SOLVE_BATCHED, 0)) == EINVAL           # Gini latent, p = 1
    assert run(opts=gm._SelectOpts(10, 2, 0, 2, gm.SOLVE_BATCHED | gm.SOLVE_PLAIN, 0)) == EINVAL
    assert run(m=0) == EINVAL
    assert run(n_nu=0) == EINVAL
    assert run(Zout=None) == EINVAL
    assert run(stride=10) == EINVAL and "stride_z" in _err(gm, h)
    assert run(ldz0=1) == EINVAL
    L.gini_destroy(h)


@pytest.mark.parametrize("d", [1, 2, 3, 10, 64, 784])
@pytest.mark.parametrize("nu", [1.1, 1.5, 2.0, 3.7])
def test_weight_table_matches_oracle_gradient(gm, orc, d, nu):
    """(d/2) W[t] is the rank-frozen derivative of the oracle's distance with
    respect to a coordinate of doubled midrank t."""
    W = gm.gini_weight_table(d, nu)
    assert W.shape == (2 * d - 1,)
    assert np.array_equal(W[::-1], -W)                      # exact antisymmetry
    z = np.arange(d, dtype=np.float64) * 0.37 - 1.0        # tie-free: t = 2, 4, ..., 2d
    _, a = orc.gini_dist_grad(z, nu)
    t = orc.rank2(z)
    np.testing.assert_allclose(0.5 * d * W[t - 2].astype(np.float64), a, rtol=2e-7, atol=1e-7)
    # ties: a constant vector takes the middle entry, which is 0
    assert W[d - 1] == 0.0


def test_weight_table_rejects_bad_arguments(gm):
    with pytest.raises(gm.GiniError):
        gm.gini_weight_table(0, 2.0)
    with pytest.raises(gm.GiniError):
        gm.gini_weight_table(4, 1.0)
    with pytest.raises(gm.GiniError):
        gm.gini_weight_table(4, math.nan)


def test_binding_refuses_cpu_tensors(gm):
    import torch
    with pytest.raises(ValueError):
        gm.gini_rank(torch.zeros(3, 4))
    with pytest.raises(ValueError):
        gm.gini_dissim(torch.zeros(3, 4), [2.0])


def test_binding_rejects_overlapping_rows(gm):
    """An expanded or transposed view is not a row-major matrix with rows of
    their own: the binding refuses it instead of reading it as dense."""
    import torch
    with pytest.raises(ValueError):
        gm._mat(torch.zeros(1, 3).expand(5, 3), "Z")
    with pytest.raises(ValueError):
        gm._mat(torch.zeros(4, 3).t(), "Z")
    assert gm._mat(torch.zeros(5, 3), "Z") == 3
    assert gm._mat(torch.zeros(5, 8)[:, :3], "Z") == 8
    assert gm._mat(torch.zeros(1, 3), "Z") == 3

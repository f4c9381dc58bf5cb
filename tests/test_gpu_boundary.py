"""The boundary's checks that need a GPU: arrays that are not device memory
of the context's GPU are refused before any kernel runs, and the refusal
leaves nothing behind for the next call."""
import ctypes

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def gm():
    from paper_2605_25124_amd import ginimds
    return ginimds


def _fwd(gm, D, zptr, n, p, out):
    c = gm.context(0)
    st = gm._lib.gini_stress_fwd(c.handle, ctypes.c_void_p(D.data_ptr()), n, int(D.stride(0)), zptr, p, p, 2.0, 0,
                                 ctypes.c_void_p(out.data_ptr()), gm._stream(0))
    return st, gm._lib.gini_last_error(c.handle).decode()


def test_host_arrays_are_refused(gm):
    g = np.random.Generator(np.random.PCG64(2))
    n, p = 200, 2
    X = torch.from_numpy(g.standard_normal((n, 5)).astype(np.float32)).to(DEV)
    D = gm.gini_dissim(X, [2.0])[0]
    out = torch.zeros(2, device=DEV)
    Zh = torch.from_numpy((0.3 * g.standard_normal((n, p))).astype(np.float32)).pin_memory()
    st, msg = _fwd(gm, D, ctypes.c_void_p(Zh.data_ptr()), n, p, out)
    assert st == 1 and "host memory" in msg, (st, msg)
    Zn = np.ascontiguousarray(Zh.numpy())                   # plain host memory HIP does not know
    st, msg = _fwd(gm, D, ctypes.c_void_p(Zn.ctypes.data), n, p, out)
    assert st == 1 and "Z" in msg, (st, msg)
    # a valid call right after the refusals runs normally
    Zd = Zh.to(DEV)
    st, msg = _fwd(gm, D, ctypes.c_void_p(Zd.data_ptr()), n, p, out)
    assert st == 0, msg
    ref = gm.gini_stress_fwd(D, Zd, 2.0, 0)
    assert torch.equal(out, ref)


def test_rank_of_host_rows_refused(gm):
    V = np.zeros((3, 300), dtype=np.float32)
    out = torch.zeros((3, 300), dtype=torch.int32, device=DEV)
    c = gm.context(0)
    st = gm._lib.gini_rank(c.handle, ctypes.c_void_p(V.ctypes.data), 3, 300, 300, ctypes.c_void_p(out.data_ptr()),
                           300, gm._stream(0))
    assert st == 1

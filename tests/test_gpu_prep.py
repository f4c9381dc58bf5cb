"""GPU parity of gini_standardize (zero median, unit population variance per
column) against the oracle; the median is an exact order statistic."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def gm():
    from paper_2605_25124_amd import ginimds
    return ginimds


def _data(n, m, seed):
    g = np.random.Generator(np.random.PCG64(seed))
    X = g.standard_t(3, size=(n, m)).astype(np.float32)
    if m > 2:
        X[:, 1] = np.round(X[:, 1])                       # heavy ties
        X[:, 2] = 4.25                                   # a constant column
    return X


@pytest.mark.parametrize("n,m", [(1, 3), (2, 3), (7, 5), (100, 16), (1001, 64), (50000, 3)])
def test_standardize_parity(gm, orc, n, m):
    X = _data(n, m, n + m)
    Y, st = gm.gini_standardize(torch.from_numpy(X).to(DEV), stats=True)
    Yn = Y.cpu().numpy().astype(np.float64)
    ref = orc.standardize(X)
    med = np.median(X.astype(np.float64), axis=0)
    np.testing.assert_allclose(st[:, 0].cpu().numpy(), med, rtol=1e-7, atol=1e-7)
    scale = np.maximum(np.abs(ref).max(axis=0), 1.0)
    assert np.all(np.abs(Yn - ref) <= 1e-5 * scale)


def test_standardize_strided_and_in_place(gm, orc):
    X = _data(300, 9, 5)
    big = torch.zeros((300, 12), device=DEV)
    big[:, :9] = torch.from_numpy(X).to(DEV)
    view = big[:, :9]
    Y = gm.gini_standardize(view)
    gm.gini_standardize(view, out=view)                    # in place, same leading dimension
    assert torch.equal(view, Y)
    assert torch.all(big[:, 9:] == 0)
    ref = orc.standardize(X)
    assert np.abs(Y.cpu().numpy() - ref).max() <= 1e-5 * max(np.abs(ref).max(), 1.0)

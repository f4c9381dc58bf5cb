"""GPU parity of gini_select_nu (Algorithm 1: every nu on every fold, Kruskal
stress of each fit with the Euclidean latent distance, nu* = argmin of the
fold mean) against the FP64 oracle's Algorithm 1."""
import numpy as np
import pytest
import torch

from paper_2605_25124_amd import synth

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def gm():
    from paper_2605_25124_amd import ginimds
    return ginimds


def test_select_one_dimensional_data_fitted_exactly(gm):
    """Two-coordinate rows embed in one Euclidean dimension at every nu; one
    Guttman step from a correctly ordered start reaches the embedding."""
    g = np.random.Generator(np.random.PCG64(71))
    X = g.standard_normal((300, 2)).astype(np.float32)
    Z0 = (0.5 * (X[:, :1] - X[:, 1:])).astype(np.float32)
    best, mean, ks, Z = gm.gini_select_nu(torch.from_numpy(X).to(DEV), [1.5, 2.0, 3.0],
                                          torch.from_numpy(Z0).to(DEV), 1, folds=3,
                                          latent=gm.LATENT_EUCLID)
    assert ks.shape == (3, 3)
    assert np.all(ks < 1e-5), ks


@pytest.mark.parametrize("folds", [1, 2])
def test_select_matches_oracle(gm, orc, folds):
    w = synth.workload_small()
    X = w.X.astype(np.float32)
    Z0 = w.Z0[0].astype(np.float32)
    nus = [1.5, 2.0, 3.0]
    iters = 50
    best, mean, ks, Z = gm.gini_select_nu(torch.from_numpy(X).to(DEV), nus, torch.from_numpy(Z0).to(DEV),
                                          iters, folds=folds)
    rbest, rmean, rks, rZ = orc.select_nu(X, nus, Z0, iters, folds=folds, mode=orc.MATCH32)
    np.testing.assert_allclose(ks, rks, rtol=1e-3)
    assert best == rbest
    Zg = Z.cpu().numpy().astype(np.float64)
    for k in range(len(nus)):
        assert np.linalg.norm(Zg[k] - rZ[k]) <= 1e-3 * np.linalg.norm(rZ[k]), k


def test_select_modes_agree(gm):
    w = synth.workload_gmm()
    X = torch.from_numpy(w.X[:900]).to(DEV)
    Z0 = torch.from_numpy(w.Z0[0][:900]).to(DEV)
    nus = [1.2, 1.5, 2.0, 2.5, 3.0, 4.0]
    out = [gm.gini_select_nu(X, nus, Z0, 10, folds=3, flags=f, tile=64)
           for f in (gm.SOLVE_BATCHED, gm.SOLVE_PERSISTENT, gm.SOLVE_PLAIN, gm.SOLVE_BATCHED | gm.SOLVE_SPLIT)]
    for b, mean, ks, Z in out[1:]:
        assert b == out[0][0]
        assert np.array_equal(ks, out[0][2])
        assert torch.equal(Z, out[0][3])

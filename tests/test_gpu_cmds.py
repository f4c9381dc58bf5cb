"""GPU parity of gini_classical_mds (Section IV-A) against the FP64 oracle's
classical MDS; the columns of the result are determined up to sign."""
import numpy as np
import pytest
import torch
from scipy.spatial.distance import pdist, squareform

from paper_2605_25124_amd import synth

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def gm():
    from paper_2605_25124_amd import ginimds
    return ginimds


def _match_signs(Z, ref):
    out = Z.copy()
    for k in range(Z.shape[1]):
        if np.dot(out[:, k], ref[:, k]) < 0:
            out[:, k] = -out[:, k]
    return out


@pytest.mark.parametrize("n,p", [(60, 3), (500, 2), (2001, 3)])
def test_euclidean_distances_recovered(gm, n, p):
    g = np.random.Generator(np.random.PCG64(n))
    Y = g.standard_normal((n, p)) * np.array([3.0, 1.5, 0.5][:p])
    D = torch.from_numpy(squareform(pdist(Y)).astype(np.float32)).to(DEV)
    Z, lam, it = gm.gini_classical_mds(D, p)
    Zn = Z.cpu().numpy().astype(np.float64)
    Dn = D.cpu().numpy().astype(np.float64)
    err = np.abs(squareform(pdist(Zn)) - Dn).max()
    assert err <= 1e-4 * Dn.max(), (err, it)
    sv = np.linalg.svd(Y - Y.mean(axis=0), compute_uv=False)
    np.testing.assert_allclose(lam, sv ** 2, rtol=1e-4)


@pytest.mark.parametrize("nu", [1.5, 2.0, 3.0])
def test_gini_dissimilarities_match_oracle(gm, orc, nu):
    w = synth.workload_gmm()
    X = w.X[:700]
    D = gm.gini_dissim(torch.from_numpy(X).to(DEV), [nu])[0]
    Z, lam, it = gm.gini_classical_mds(D, 2, max_iters=1000, tol=1e-9)
    Zr, lr = orc.classical_mds(D.cpu().numpy(), 2)
    np.testing.assert_allclose(lam, lr, rtol=1e-4)
    Zn = _match_signs(Z.cpu().numpy().astype(np.float64), Zr)
    assert np.linalg.norm(Zn - Zr) <= 1e-3 * np.linalg.norm(Zr), it


def test_rank_one_and_repeatable(gm):
    """Two-coordinate rows give a one-dimensional embedding (B of rank one):
    the second eigenvalue is 0 and the run repeats bitwise."""
    g = np.random.Generator(np.random.PCG64(3))
    X = torch.from_numpy(g.standard_normal((300, 2)).astype(np.float32)).to(DEV)
    D = gm.gini_dissim(X, [2.0])[0]
    Z1, l1, _ = gm.gini_classical_mds(D, 2)
    Z2, l2, _ = gm.gini_classical_mds(D, 2)
    assert torch.equal(Z1, Z2) and np.array_equal(l1, l2)
    assert abs(l1[1]) <= 1e-5 * l1[0]
    y = 0.5 * (X[:, 0] - X[:, 1]).double().cpu().numpy()
    z = Z1[:, 0].double().cpu().numpy()
    z = z if np.dot(z, y - y.mean()) > 0 else -z
    np.testing.assert_allclose(z, y - y.mean(), atol=1e-4 * np.abs(y).max())

"""GPU parity of the rank and dissimilarity kernels against the FP64 oracle."""
import numpy as np
import pytest
import torch

from paper_2605_25124_amd import synth
from tests._util import assert_dissim_close, dissim_scale, f32

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def gm():
    from paper_2605_25124_amd import ginimds
    return ginimds


def _rows(kind, rows, d, seed):
    g = np.random.Generator(np.random.PCG64(seed))
    if kind == "gauss":
        return g.standard_normal((rows, d)).astype(np.float32)
    if kind == "ties":
        return synth.rows_with_ties(g, rows, d, 2)
    if kind == "const":
        return np.full((rows, d), 1.25, dtype=np.float32)
    return synth.signed_zero_rows(g, rows, d)


@pytest.mark.parametrize("d", [1, 2, 3, 4, 10, 16, 63, 64, 65, 255, 256, 257, 784, 1000, 4095, 4096, 4097, 8193,
                               40000])
@pytest.mark.parametrize("kind", ["gauss", "ties", "const", "zeros"])
def test_rank_bit_exact(gm, orc, d, kind):
    rows = 37 if d < 1000 else (5 if d < 10000 else 2)
    V = _rows(kind, rows, d, 1000 + d)
    t = gm.gini_rank(torch.from_numpy(V).to(DEV)).cpu().numpy()
    ref = orc.rank2_rows(V)
    assert np.array_equal(t, ref)


def test_rank_rows_in_batches(gm, orc):
    """Long rows are ranked through sorted chunks in a bounded scratch: more
    rows than one batch holds (2^24 words) are processed batch by batch."""
    rows, d = 3400, 5000
    V = _rows("ties", rows, d, 77)
    t = gm.gini_rank(torch.from_numpy(V).to(DEV)).cpu().numpy()
    assert np.array_equal(t, orc.rank2_rows(V))


def test_rank_strided_and_empty(gm, orc):
    V = _rows("ties", 20, 50, 7)
    big = torch.zeros((20, 64), device=DEV)
    big[:, :50] = torch.from_numpy(V).to(DEV)
    out = torch.full((20, 70), -1, dtype=torch.int32, device=DEV)
    gm.gini_rank(big[:, :50], out[:, :50])
    o = out.cpu().numpy()
    assert np.array_equal(o[:, :50], orc.rank2_rows(V))
    assert np.all(o[:, 50:] == -1)                        # nothing written past d
    e = gm.gini_rank(torch.zeros((0, 5), device=DEV))
    assert e.shape == (0, 5)


def _check_full(gm, orc, X32, nus, what):
    n = X32.shape[0]
    D = gm.gini_dissim(torch.from_numpy(X32).to(DEV), nus)
    torch.cuda.synchronize()
    Dg = D.cpu().numpy()
    ref = orc.dissim(X32, nus, orc.MATCH32)
    iu = np.triu_indices(n, 1)
    pairs = list(zip(iu[0], iu[1]))
    for k, nu in enumerate(nus):
        assert np.array_equal(Dg[k], Dg[k].T), what
        assert np.all(np.diag(Dg[k]) == 0.0), what
        S = dissim_scale(orc, X32, pairs, nu)
        assert_dissim_close(Dg[k][iu], ref[k][iu], S, what=f"{what} nu={nu}")


def test_dissim_small_workload(gm, orc):
    w = synth.workload_small()
    _check_full(gm, orc, f32(w.X), [2.0], "n=200 m=10")


def test_dissim_gmm_subsample(gm, orc):
    w = synth.workload_gmm()
    idx = synth.subsample(w.n, 150, 11)
    _check_full(gm, orc, f32(w.X[idx]), [1.5, 2.0, 3.0], "gmm m=16")


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5, 9, 12, 13, 24, 30, 33, 47, 64])
def test_dissim_lane_path_sizes(gm, orc, m):
    g = np.random.Generator(np.random.PCG64(m))
    X = g.standard_normal((45, m)).astype(np.float32)
    _check_full(gm, orc, X, list(np.linspace(1.1, 4.0, 8)), f"lane m={m}")


@pytest.mark.parametrize("m", [5, 16, 64])
def test_dissim_lane_path_ties(gm, orc, m):
    g = np.random.Generator(np.random.PCG64(50 + m))
    X = synth.rows_with_ties(g, 40, m, 2)
    _check_full(gm, orc, X, [1.5, 2.0, 3.7], f"lane ties m={m}")


@pytest.mark.parametrize("m", [65, 100, 128, 129, 256, 300, 512, 513, 784, 1024, 1500, 2048, 3000, 4096])
def test_dissim_group_path_sizes(gm, orc, m):
    g = np.random.Generator(np.random.PCG64(m))
    n = 19 if m > 1024 else 35
    X = g.standard_normal((n, m)).astype(np.float32)
    X[3] = X[5]                                       # an all-tied (zero) difference
    X[7, : m // 3] = X[8, : m // 3]                  # a long run of zero differences
    _check_full(gm, orc, X, [2.0, 3.7], f"group m={m}")


def test_dissim_images_ties(gm, orc):
    X = synth.image_rows(synth.rng_for(3), 40)
    _check_full(gm, orc, X, [2.0, 3.7], "images m=784")


def test_dissim_many_nu_chunks(gm, orc):
    g = np.random.Generator(np.random.PCG64(99))
    X = g.standard_normal((20, 12)).astype(np.float32)
    nus = list(np.linspace(1.05, 6.0, 19))
    _check_full(gm, orc, X, nus, "19 nu")
    Xg = g.standard_normal((12, 200)).astype(np.float32)
    _check_full(gm, orc, Xg, nus, "19 nu group")


@pytest.mark.parametrize("n", [1, 2, 3, 31, 32, 33, 65])
def test_dissim_ragged_n(gm, orc, n):
    g = np.random.Generator(np.random.PCG64(n))
    X = g.standard_normal((n, 7)).astype(np.float32)
    D = gm.gini_dissim(torch.from_numpy(X).to(DEV), [2.0]).cpu().numpy()[0]
    assert D.shape == (n, n)
    ref = orc.dissim(X, [2.0], orc.MATCH32)[0]
    assert np.all(np.diag(D) == 0.0)
    assert np.array_equal(D, D.T)
    np.testing.assert_allclose(D, ref, rtol=2e-6, atol=1e-6)


def test_dissim_padded_output_untouched(gm, orc):
    g = np.random.Generator(np.random.PCG64(5))
    X = g.standard_normal((30, 8)).astype(np.float32)
    buf = torch.full((2, 30, 37), 7.0, device=DEV)
    out = buf[:, :, :30]
    gm.gini_dissim(torch.from_numpy(X).to(DEV), [2.0, 3.0], out=out)
    b = buf.cpu().numpy()
    assert np.all(b[:, :, 30:] == 7.0)
    ref = orc.dissim(X, [2.0, 3.0], orc.MATCH32)
    np.testing.assert_allclose(b[:, :, :30], ref, rtol=2e-6, atol=1e-6)


def test_dissim_worked_example(gm):
    X = torch.tensor([[10.0, 1200.0], [10.0, 12.0]], device=DEV)
    D = gm.gini_dissim(X, [2.0]).cpu().numpy()[0]
    assert D[0, 1] == 594.0 and D[1, 0] == 594.0

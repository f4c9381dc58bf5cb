"""Stress reductions with more than sixteen stress slices: every instance's
scratch holds all of its slices, so an instance queued in front of another in
a batched solve leaves the other's partial sums alone.  Slices pass sixteen
from n ~ 16400 at tile 64 and n ~ 24000 at tile 128."""
import numpy as np
import pytest
import torch

from tests._util import assert_grad_close, step_rounding

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def gm():
    from paper_2605_25124_amd import ginimds
    return ginimds


def _data(gm, n, seed, p=2):
    g = np.random.Generator(np.random.PCG64(seed))
    X = g.standard_normal((n, 8)).astype(np.float32)
    Z = (0.1 * g.standard_normal((n, p))).astype(np.float32)
    D = gm.gini_dissim(torch.from_numpy(X).to(DEV), [2.0])[0]
    return D, Z


def _slices(n, tile):
    nb = -(-n // tile)
    units = 2 if tile == 128 else (1 if tile == 64 else 4)
    cnt = nb * (nb + 1) // 2 * units * 4
    return min(32, max(1, -(-cnt // (1024 * 8))))


def _solve(gm, insts, flags, tile):
    out = []
    for D, Z0, latent in insts:
        out.append((D, torch.from_numpy(Z0).to(DEV), torch.zeros(1, device=DEV), latent))
    gm.gini_mds_solve([gm.Instance(D, Z, 2.0, latent, 0.0, h) for D, Z, h, latent in out], 1, flags, tile)
    return [(Z.cpu(), h.cpu()) for _, Z, h, _ in out]


@pytest.mark.parametrize("tile,n_big", [(64, 17000), (128, 30000)])
def test_batched_in_front_of_another_instance(gm, orc, tile, n_big):
    """One descent step of [big, small] in one batched launch equals each one
    run alone, bitwise; the big instance's stress and sampled gradient rows
    match the oracle (Euclidean latent: the stress over every row is cheap for
    the oracle)."""
    assert _slices(n_big, tile) > 16
    Db, Zb = _data(gm, n_big, 7)
    Ds, Zs = _data(gm, 700, 8)
    for latent in (1, 0):
        pair = _solve(gm, [(Db, Zb, latent), (Ds, Zs, latent)], gm.SOLVE_BATCHED, tile)
        alone_b = _solve(gm, [(Db, Zb, latent)], gm.SOLVE_BATCHED, tile)[0]
        alone_s = _solve(gm, [(Ds, Zs, latent)], gm.SOLVE_PLAIN, tile)[0]
        assert torch.equal(pair[0][0], alone_b[0]) and torch.equal(pair[0][1], alone_b[1]), latent
        assert torch.equal(pair[1][0], alone_s[0]) and torch.equal(pair[1][1], alone_s[1]), latent
    # the big instance (Euclidean latent) against the oracle: the stress over
    # all rows in blocks, and the gradient on sampled rows, from the step
    Z1, h = _solve(gm, [(Db, Zb, 1)], gm.SOLVE_BATCHED, tile)[0]
    total = 0.0
    for a in range(0, n_big, 2000):
        rows = np.arange(a, min(a + 2000, n_big))
        Dr = Db[a:a + len(rows)].cpu().numpy()
        _, part = orc.grad_rows(Dr, rows, Zb, 2.0, 1, orc.MATCH32)
        total += part
    assert abs(float(h[0]) - total) <= 1e-4 * total, (float(h[0]), total)
    rows = np.array([0, 1, tile - 1, tile, n_big // 2, n_big - 2, n_big - 1])
    Dr = Db.index_select(0, torch.from_numpy(rows).to(DEV)).cpu().numpy()
    G_ref, _ = orc.grad_rows(Dr, rows, Zb, 2.0, 1, orc.MATCH32)
    B = orc.grad_scale_rows(Dr, rows, Zb, 2.0, 1, orc.MATCH32)
    eta = orc.step_size(n_big, 2, 2.0, 1)
    Z0n, Z1n = Zb[rows].astype(np.float64), Z1.numpy()[rows].astype(np.float64)
    assert_grad_close((Z0n - Z1n) / eta, G_ref, B, 1e-4, step_rounding(Z0n, Z1n, eta, G_ref), "big instance")


def test_single_evaluation_many_slices(gm, orc):
    """gini_stress_fwd / gini_stress_bwd at n = 30000 (28 slices at tile 128):
    the two stresses agree bitwise, repeated calls are bitwise equal, and
    sampled gradient rows (Gini latent, p = 3) match the oracle."""
    n = 30000
    D, Z = _data(gm, n, 9, p=3)
    Zt = torch.from_numpy(Z).to(DEV)
    G1, s1 = gm.gini_stress_bwd(D, Zt, 2.0, 0)
    G2, s2 = gm.gini_stress_bwd(D, Zt, 2.0, 0)
    sf = gm.gini_stress_fwd(D, Zt, 2.0, 0)
    assert torch.equal(G1, G2) and torch.equal(s1, s2) and torch.equal(s1, sf)
    rows = np.array([0, 5, 127, 128, 12345, n - 2, n - 1])
    Dr = D.index_select(0, torch.from_numpy(rows).to(DEV)).cpu().numpy()
    G_ref, _ = orc.grad_rows(Dr, rows, Z, 2.0, 0, orc.MATCH32)
    B = orc.grad_scale_rows(Dr, rows, Z, 2.0, 0, orc.MATCH32)
    assert_grad_close(G1.cpu().numpy()[rows], G_ref, B, 1e-4, what="n=30000 p=3 rows")

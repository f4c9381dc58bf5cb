"""The entry point that allocates nothing (gini_stress_bwd_static): its
results equal gini_stress_bwd's bitwise, on two calls in a row, the second
with a smaller problem, so nothing the static scratch kept from the first
call leaks into the second; a problem larger than the static array is
refused before anything runs."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def gm():
    from paper_2605_25124_amd import ginimds
    return ginimds


def _problem(gm, n, p, seed, nu):
    g = np.random.Generator(np.random.PCG64(seed))
    X = torch.from_numpy(g.standard_normal((n, 7)).astype(np.float32)).to(DEV)
    Z = torch.from_numpy((0.5 * g.standard_normal((n, p))).astype(np.float32)).to(DEV)
    return gm.gini_dissim(X, [nu])[0], Z


@pytest.mark.parametrize("first,second", [((2000, 3, 0, 1.5), (700, 2, 0, 2.0)),
                                          ((4097, 2, 1, 2.0), (65, 2, 0, 3.0))])
def test_static_entry_matches_the_allocating_one(gm, first, second):
    for n, p, latent, nu in (first, second):
        D, Z = _problem(gm, n, p, 100 + n, nu)
        go = torch.tensor([0.75], device=DEV)
        G_ref, s_ref = gm.gini_stress_bwd(D, Z, nu, latent, grad_out=go)
        G = torch.full((n, p), float("nan"), device=DEV)
        s = torch.full((2,), float("nan"), device=DEV)
        gm.gini_stress_bwd_static(D, Z, nu, latent, grad_out=go, gradZ=G, out_sigma=s)
        torch.cuda.synchronize()
        assert torch.equal(G, G_ref), (n, p, latent)
        assert torch.equal(s, s_ref), (n, p, latent)


def test_static_entry_refuses_what_does_not_fit(gm):
    n = 40000                                   # p = 3 needs about 150 MB of scratch, over the 64 MiB array
    D = torch.empty((n, n), device=DEV)
    Z = torch.zeros((n, 3), device=DEV)
    with pytest.raises(gm.GiniError) as e:
        gm.gini_stress_bwd_static(D, Z, 2.0, 0)
    assert e.value.status == 5 and "scratch" in e.value.message

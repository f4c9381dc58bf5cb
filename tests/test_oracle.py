"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these tests retypes the oracle's own formula: each checks it against a
printed value, a rank-free identity, a library routine, a closed form, a
property the paper proves, or brute force.
"""
import itertools
import json
import os

import numpy as np
import pytest
from scipy.spatial.distance import pdist, squareform
from scipy.stats import rankdata

from paper_2605_25124_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")
NUS = [1.1, 1.5, 2.0, 3.0, 3.7, 5.0]


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


# ------------------------------------------------------------------ ranks
def test_rank_worked_example(orc):
    g = _gold("worked_example.json")
    z = np.array(g["u"]) - np.array(g["v"])
    assert list(orc.rank2(z)) == [2 * r for r in g["ranks_of_u_minus_v"]]


def test_rank_zero_vector_is_midpoint(orc):
    g = _gold("rank_zero_vector.json")
    for d in g["dims"]:
        t = orc.rank2(np.zeros(d))
        assert np.all(t == d + 1)            # t = 2R = d+1


@pytest.mark.parametrize("d", [1, 2, 3, 5, 16, 63, 64, 65, 200, 784])
def test_rank_matches_scipy_average(orc, d):
    g = np.random.Generator(np.random.PCG64(11 + d))
    for levels in (None, 2, 6):
        v = g.standard_normal(d) if levels is None else g.integers(-levels, levels + 1, d).astype(float)
        ref = (2 * rankdata(v, method="average")).astype(np.int64)
        assert np.array_equal(orc.rank2(v, "sort"), ref)
        if d <= 300:
            assert np.array_equal(orc.rank2(v, "count"), ref)
        assert np.array_equal(orc.rank2(v), ref)


@pytest.mark.parametrize("d", [1, 2, 7, 64, 100])
def test_rank_invariants(orc, d):
    g = np.random.Generator(np.random.PCG64(5 * d))
    v = g.integers(-3, 4, d).astype(float)
    t = orc.rank2(v).astype(np.int64)
    assert t.sum() == d * (d + 1)                              # sum of ranks
    assert np.array_equal(orc.rank2(-v), 2 * d + 2 - t)         # R(-x) = d+1-R(x)
    assert np.all(orc.rank2(np.full(d, 3.25)) == d + 1)         # all tied


def test_rank_signed_zero_ties(orc):
    t = orc.rank2(np.array([0.0, -0.0, 1.0, -1.0]))
    assert list(t) == [5, 5, 8, 2]          # -1 < (0 == -0) < 1


# ------------------------------------------------------- the distance
def test_worked_example_distance(orc):
    g = _gold("worked_example.json")
    u, v = np.array(g["u"]), np.array(g["v"])
    assert orc.gini_dist(u - v, g["nu"]) == g["D_G"]
    assert orc.gini_dist(v - u, g["nu"]) == g["D_G"]
    assert orc.gini_asym(u - v, g["nu"]) == g["D_G"]


@pytest.mark.parametrize("d", [2, 3, 10, 64, 97])
def test_nu2_is_half_gini_mean_difference(orc, d):
    """At nu=2 the distance is (1/2) sum_{a<b} |z_a - z_b|: rank-free, tie-free or not."""
    g = np.random.Generator(np.random.PCG64(100 + d))
    for levels in (None, 3):
        z = g.standard_normal(d) if levels is None else g.integers(-levels, levels + 1, d).astype(float)
        gmd = 0.5 * sum(abs(z[a] - z[b]) for a in range(d) for b in range(a + 1, d))
        assert orc.gini_dist(z, 2.0) == pytest.approx(gmd, rel=1e-12, abs=1e-12)


@pytest.mark.parametrize("d", [2, 5, 33])
def test_nu2_is_definition2_with_library_midranks(orc, d):
    g = np.random.Generator(np.random.PCG64(7 + d))
    z = g.integers(-2, 3, d).astype(float)
    dg = float(np.sum(z * (rankdata(z, method="average") - (d + 1) / 2.0)))
    assert orc.gini_dist(z, 2.0) == pytest.approx(dg, rel=1e-12, abs=1e-12)
    assert orc.gini_asym(z, 2.0) == pytest.approx(dg, rel=1e-12, abs=1e-12)


@pytest.mark.parametrize("nu", NUS)
def test_closed_form_d2(orc, nu):
    g = np.random.Generator(np.random.PCG64(3))
    for _ in range(20):
        z = g.standard_normal(2)
        assert orc.gini_dist(z, nu) == pytest.approx(2.0 ** (1 - nu) * abs(z[0] - z[1]), rel=1e-12)
    assert orc.gini_dist([1.5, 1.5], nu) == 0.0


@pytest.mark.parametrize("nu", NUS)
def test_closed_form_d3(orc, nu):
    g = np.random.Generator(np.random.PCG64(4))
    for _ in range(20):
        z = g.standard_normal(3)
        ref = 1.5 * (2.0 / 3.0) ** (nu - 1) * (z.max() - z.min())
        assert orc.gini_dist(z, nu) == pytest.approx(ref, rel=1e-12)
    # a tie at the bottom: two coordinates share doubled rank 3, the third has 6
    z = np.array([-5.0, -5.0, -4.0])
    w3 = (1 / 6) ** (nu - 1) - (1 / 2) ** (nu - 1)
    w6 = (2 / 3) ** (nu - 1)
    ref = 1.5 * (2 * w3 * -5.0 + w6 * -4.0)
    assert orc.gini_dist(z, nu) == pytest.approx(ref, rel=1e-12, abs=1e-12)


def test_ties_can_break_nonnegativity_off_nu2(orc):
    assert orc.gini_dist([-5.0, -5.0, -4.0], 1.5) < 0.0
    assert orc.gini_dist([-5.0, -5.0, -4.0], 2.0) >= 0.0


@pytest.mark.parametrize("nu", NUS)
def test_d1_is_zero(orc, nu):
    assert orc.gini_dist([3.0], nu) == 0.0


@pytest.mark.parametrize("nu", NUS)
def test_pseudometric_properties(orc, nu):
    """Proposition 2 / 3: null, egalitarian, symmetry, homogeneity, triangle and
    non-negativity (tie-free data for nu != 2)."""
    g = np.random.Generator(np.random.PCG64(int(nu * 10)))
    d = 9
    assert orc.gini_dist(np.zeros(d), nu) == 0.0
    assert orc.gini_dist(np.full(d, -2.5), nu) == 0.0
    for _ in range(40):
        x, y, w = g.standard_normal((3, d))
        dxy = orc.gini_dist(x - y, nu)
        assert dxy == orc.gini_dist(y - x, nu)
        assert dxy >= 0.0
        lam = g.uniform(-3, 3)
        assert orc.gini_dist(lam * (x - y), nu) == pytest.approx(abs(lam) * dxy, rel=1e-12, abs=1e-14)
        assert dxy <= orc.gini_dist(x - w, nu) + orc.gini_dist(w - y, nu) + 1e-12


def test_pseudometric_with_ties_at_nu2(orc):
    g = np.random.Generator(np.random.PCG64(77))
    for _ in range(40):
        x, y, w = g.integers(-2, 3, (3, 8)).astype(float)
        dxy = orc.gini_dist(x - y, 2.0)
        assert dxy >= 0.0
        assert dxy <= orc.gini_dist(x - w, 2.0) + orc.gini_dist(w - y, 2.0) + 1e-12


@pytest.mark.parametrize("nu", [1.5, 2.0, 3.7])
def test_support_function_inequality(orc, nu):
    """With ranks frozen the distance is linear; over tie-free points it is the
    maximum of these linear pieces (the rearrangement argument of the proofs),
    so delta(z) >= a(z') . z for every z'."""
    g = np.random.Generator(np.random.PCG64(9))
    for _ in range(30):
        z, z2 = g.standard_normal((2, 6))
        dz = orc.gini_dist(z, nu)
        _, a2 = orc.gini_dist_grad(z2, nu)
        assert dz >= float(a2 @ z) - 1e-12
        # brute force over every ordering of the weights of z2
        best = max(float(np.dot(z, a2[list(perm)])) for perm in itertools.permutations(range(6)))
        assert dz == pytest.approx(best, rel=1e-12)


@pytest.mark.parametrize("nu", [1.3, 2.0, 4.2])
def test_distance_gradient_finite_difference(orc, nu):
    g = np.random.Generator(np.random.PCG64(21))
    for d in (2, 3, 7):
        z = g.standard_normal(d)
        _, a = orc.gini_dist_grad(z, nu)
        h = 1e-7
        for c in range(d):
            e = np.zeros(d)
            e[c] = h
            fd = (orc.gini_dist(z + e, nu) - orc.gini_dist(z - e, nu)) / (2 * h)
            assert fd == pytest.approx(a[c], rel=1e-6, abs=1e-8)


def test_match32_decides_on_float_bits(orc):
    X = np.array([[1.0 + 2.0 ** -30, 0.0], [1.0, 0.0]])
    D32 = orc.dissim(X, [3.0], orc.MATCH32)
    D64 = orc.dissim(X, [3.0], orc.EXACT)
    assert D32[0, 0, 1] == 0.0                      # the difference rounds to 0 in FP32
    assert D64[0, 0, 1] > 0.0


def test_dissim_matrix_structure(orc):
    g = np.random.Generator(np.random.PCG64(31))
    X = g.standard_normal((13, 6))
    D = orc.dissim(X, [1.5, 2.0], orc.EXACT)
    for k, nu in enumerate([1.5, 2.0]):
        assert np.array_equal(D[k], D[k].T)
        assert np.all(np.diag(D[k]) == 0.0)
        i, j = np.triu_indices(13, 1)
        P = orc.dissim_pairs(X, i, j, [nu], orc.EXACT)[:, 0]
        assert np.array_equal(P, D[k][i, j])
        assert D[k][0, 5] == orc.gini_dist(X[0] - X[5], nu)


# ---------------------------------------------------------- the stress
def _problem(seed, n, m, p):
    g = np.random.Generator(np.random.PCG64(seed))
    X = g.standard_normal((n, m))
    Z = 0.5 * g.standard_normal((n, p))
    return X, Z


@pytest.mark.parametrize("p", [1, 2, 3])
def test_euclid_stress_matches_pdist(orc, p):
    X, Z = _problem(1, 25, 5, p)
    D = orc.dissim(X, [2.0], orc.EXACT)[0]
    s, _ = orc.stress(D, Z, 2.0, orc.LATENT_EUCLID, orc.EXACT)
    ref = float(np.sum((pdist(Z) - squareform(D, checks=False)) ** 2))
    assert s == pytest.approx(ref, rel=1e-12)


@pytest.mark.parametrize("nu", [1.5, 2.0, 3.0])
def test_gini_p2_stress_closed_form(orc, nu):
    X, Z = _problem(2, 30, 4, 2)
    D = orc.dissim(X, [nu], orc.EXACT)[0]
    s, _ = orc.stress(D, Z, nu, orc.LATENT_GINI, orc.EXACT)
    u = Z[:, None, :] - Z[None, :, :]
    delta = 2.0 ** (1 - nu) * np.abs(u[..., 0] - u[..., 1])
    i, j = np.triu_indices(30, 1)
    ref = float(np.sum((delta[i, j] - D[i, j]) ** 2))
    assert s == pytest.approx(ref, rel=1e-12)


@pytest.mark.parametrize("latent,p,nu", [(0, 2, 2.0), (0, 3, 1.5), (0, 3, 3.7), (1, 2, 2.0), (1, 3, 3.0)])
def test_stress_gradient_finite_difference(orc, latent, p, nu):
    X, Z = _problem(3 + p, 18, 6, p)
    D = orc.dissim(X, [nu], orc.EXACT)[0]
    _, G = orc.stress(D, Z, nu, latent, orc.EXACT)
    h = 1e-7
    for i in range(0, 18, 5):
        for c in range(p):
            Zp, Zm = Z.copy(), Z.copy()
            Zp[i, c] += h
            Zm[i, c] -= h
            fd = (orc.stress(D, Zp, nu, latent, orc.EXACT, grad=False)[0]
                  - orc.stress(D, Zm, nu, latent, orc.EXACT, grad=False)[0]) / (2 * h)
            assert fd == pytest.approx(G[i, c], rel=1e-5, abs=1e-6)


@pytest.mark.parametrize("nu", [1.5, 2.0, 3.0])
def test_zero_residual_fixed_point(orc, nu):
    """m == p and Z == X: the latent Gini distances equal Delta, sigma = 0, G = 0."""
    g = np.random.Generator(np.random.PCG64(55))
    X = g.standard_normal((20, 3))
    D = orc.dissim(X, [nu], orc.EXACT)[0]
    s, G = orc.stress(D, X, nu, orc.LATENT_GINI, orc.EXACT)
    assert s == 0.0
    assert np.all(G == 0.0)


@pytest.mark.parametrize("latent", [0, 1])
def test_kruskal_stress_pins(orc, latent):
    """Kruskal stress (Section IV-B): a collapsed configuration (all latent
    distances 0) has sigma equal to the normaliser, so KS = 1 exactly; the
    zero-residual configuration has KS = 0; and KS is scale free under the
    Euclidean latent distance (Delta and Z scaled together)."""
    X, Z = _problem(31, 26, 4, 2)
    D = orc.dissim(X, [2.0], orc.EXACT)[0]
    assert orc.kruskal(D, np.zeros_like(Z), 2.0, latent, orc.EXACT) == 1.0
    g = np.random.Generator(np.random.PCG64(56))
    Y = g.standard_normal((15, 2))
    DY = orc.dissim(Y, [2.0], orc.EXACT)[0]
    assert orc.kruskal(DY, Y, 2.0, orc.LATENT_GINI, orc.EXACT) == 0.0
    if latent == 1:
        k1 = orc.kruskal(D, Z, 2.0, latent, orc.EXACT)
        k2 = orc.kruskal(3.5 * D, 3.5 * Z, 2.0, latent, orc.EXACT)
        assert k2 == pytest.approx(k1, rel=1e-13)
        assert 0.0 < k1 < 10.0


@pytest.mark.parametrize("latent,p", [(0, 2), (0, 3), (1, 2)])
def test_gradient_translation_invariance(orc, latent, p):
    X, Z = _problem(8, 40, 5, p)
    D = orc.dissim(X, [2.5], orc.EXACT)[0]
    _, G = orc.stress(D, Z, 2.5, latent, orc.EXACT)
    assert np.abs(G.sum(axis=0)).max() <= 1e-10 * np.abs(G).sum()
    if latent == 0:
        # tie-free Gini weights sum to zero over the coordinates of each point
        assert np.abs(G.sum(axis=1)).max() <= 1e-10 * np.abs(G).sum()


def test_euclid_step_is_guttman_transform(orc):
    """SMACOF (Section IV-B, unit weights): Z - grad/(2n) = B(Z) Z / n + centroid."""
    X, Z = _problem(9, 22, 5, 2)
    n = 22
    D = orc.dissim(X, [2.0], orc.EXACT)[0]
    _, G = orc.stress(D, Z, 2.0, orc.LATENT_EUCLID, orc.EXACT)
    eta = orc.step_size(n, 2, 2.0, orc.LATENT_EUCLID)
    assert eta == 1.0 / (2 * n)
    dz = squareform(pdist(Z))
    B = np.zeros((n, n))
    off = ~np.eye(n, dtype=bool)
    B[off] = -D[off] / dz[off]
    B[np.diag_indices(n)] = -B.sum(axis=1)
    guttman = B @ Z / n + Z.mean(axis=0)
    assert np.allclose(Z - eta * G, guttman, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("nu", [1.5, 2.0, 3.0])
def test_gini_p2_step_constant(orc, nu):
    n = 50
    assert orc.step_size(n, 2, nu, orc.LATENT_GINI) == pytest.approx(1.0 / (2 * n * 2 * 4.0 ** (1 - nu)), rel=1e-14)


@pytest.mark.parametrize("latent,p,nu", [(1, 2, 2.0), (1, 3, 1.5), (0, 2, 2.0), (0, 2, 3.0), (0, 2, 1.5)])
def test_monotone_stress(orc, latent, p, nu):
    from paper_2605_25124_amd import synth
    w = synth.workload_small()
    X = w.X[:80]
    D = orc.dissim(X, [nu], orc.EXACT)[0]
    Z0 = synth.initial_config(synth.rng_for(1, 1), 80, p, np.float64)
    _, hist = orc.solve(D, Z0, nu, 60, latent, orc.EXACT)
    assert hist[-1] < hist[0]
    assert np.all(np.diff(hist) <= 1e-12 * hist[0])


def test_gini_p3_nearly_monotone(orc):
    from paper_2605_25124_amd import synth
    w = synth.workload_small()
    X = w.X[:60]
    D = orc.dissim(X, [2.0], orc.EXACT)[0]
    Z0 = synth.initial_config(synth.rng_for(1, 1), 60, 3, np.float64)
    _, hist = orc.solve(D, Z0, 2.0, 60, orc.LATENT_GINI, orc.EXACT)
    assert hist[-1] < 0.9 * hist[0]
    assert np.all(np.diff(hist) <= 1e-5 * hist[0])


def test_grad_rows_matches_full_gradient(orc):
    X, Z = _problem(12, 35, 4, 3)
    D = orc.dissim(X, [2.0], orc.MATCH32)[0]
    s, G = orc.stress(D, Z, 2.0, orc.LATENT_GINI, orc.MATCH32)
    rows = np.array([0, 7, 34])
    Gr, part = orc.grad_rows(D[rows], rows, Z, 2.0, orc.LATENT_GINI, orc.MATCH32)
    assert np.allclose(Gr, G[rows], rtol=1e-12, atol=1e-12)
    allrows = np.arange(35)
    _, tot = orc.grad_rows(D, allrows, Z, 2.0, orc.LATENT_GINI, orc.MATCH32)
    assert tot == pytest.approx(s, rel=1e-12)


# ------------------------------------------------------ Algorithm 1 (nu*)
def test_select_nu_one_dimensional_data_is_fitted_exactly(orc):
    """Rows of two coordinates: at any nu the dissimilarity is a multiple of
    |y_i - y_j|, y = x_1 - x_2 (the d = 2 weights are -w, 0, +w), so the data
    embed exactly in one Euclidean dimension.  From a start in the right order
    one Guttman step (the Euclidean descent step) reaches the embedding, and
    Algorithm 1's Kruskal stress is 0 for every nu and every fold."""
    g = np.random.Generator(np.random.PCG64(71))
    X = g.standard_normal((40, 2))
    Z0 = 0.5 * (X[:, :1] - X[:, 1:])
    best, mean, ks, _ = orc.select_nu(X, [1.5, 2.0, 3.0], Z0, 1, folds=2, latent=orc.LATENT_EUCLID,
                                      mode=orc.EXACT)
    assert ks.shape == (3, 2)
    assert np.all(ks < 1e-12), ks
    # a start in the wrong order is not fitted by one step
    _, mean2, _, _ = orc.select_nu(X, [2.0], Z0[::-1].copy(), 1, folds=1, latent=orc.LATENT_EUCLID,
                                   mode=orc.EXACT)
    assert mean2[0] > 1e-3


def test_select_nu_scale_invariance_and_argmin(orc):
    """Distances are 1-homogeneous and the step size does not depend on the
    scale, so scaling X and Z0 together leaves every KS unchanged; nu* is the
    argmin of the fold means."""
    w = synth.workload_small()
    X, Z0 = w.X[:60], w.Z0[0][:60].astype(np.float64)
    nus = [1.5, 2.0, 3.0]
    best, mean, ks, Z = orc.select_nu(X, nus, Z0, 20, folds=2, mode=orc.EXACT)
    best2, mean2, ks2, Z2 = orc.select_nu(4.0 * X, nus, 4.0 * Z0, 20, folds=2, mode=orc.EXACT)
    np.testing.assert_allclose(ks2, ks, rtol=1e-9)
    np.testing.assert_allclose(Z2, 4.0 * Z, rtol=1e-9, atol=1e-12)
    assert best == best2 == int(np.argmin(ks.mean(axis=1)))
    np.testing.assert_allclose(mean, ks.mean(axis=1))
    assert np.all(np.isfinite(ks) & (ks > 0))


# ------------------------------------------------------------ Sammon stress
def test_sammon_two_points(orc):
    """One pair: S = Delta, so the Sammon stress is (delta - Delta)^2 / Delta^2."""
    D = np.array([[0.0, 2.5], [2.5, 0.0]])
    Z = np.array([[0.0, 0.0], [3.0, 4.0]])
    s, G = orc.sammon(D, Z, 2.0, orc.LATENT_EUCLID, orc.EXACT)
    assert s == pytest.approx((5.0 - 2.5) ** 2 / 2.5 ** 2, rel=1e-15)
    # d/dZ_0 of (|Z_0 - Z_1| - 2.5)^2 / 2.5^2 = 2 (5 - 2.5) / 2.5^2 * (Z_0 - Z_1) / 5
    np.testing.assert_allclose(G[0], 2 * 2.5 / 6.25 * np.array([-3.0, -4.0]) / 5.0, rtol=1e-14)
    np.testing.assert_allclose(G[1], -G[0], rtol=1e-15)


def test_sammon_uniform_dissimilarities_scale_the_raw_stress(orc):
    """All Delta_ij = c0: Sammon = raw / (c0 * S) with S = c0 * n (n - 1) / 2."""
    n, c0 = 17, 1.7
    D = np.full((n, n), c0)
    np.fill_diagonal(D, 0.0)
    Z = np.random.Generator(np.random.PCG64(5)).standard_normal((n, 2))
    for latent in (orc.LATENT_EUCLID, orc.LATENT_GINI):
        s, G = orc.sammon(D, Z, 2.5, latent, orc.EXACT)
        r, Gr = orc.stress(D, Z, 2.5, latent, orc.EXACT)
        scale = c0 * c0 * n * (n - 1) / 2
        assert s == pytest.approx(r / scale, rel=1e-13)
        np.testing.assert_allclose(G, Gr / scale, rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("latent,p,nu", [(0, 2, 2.0), (0, 3, 1.5), (1, 2, 2.0), (1, 3, 3.0)])
def test_sammon_gradient_finite_difference(orc, latent, p, nu):
    X, Z = _problem(13 + p, 16, 5, p)
    X[3] = X[7]                                         # a zero dissimilarity: no weight, no NaN
    D = orc.dissim(X, [nu], orc.EXACT)[0]
    assert D[3, 7] == 0.0
    s, G = orc.sammon(D, Z, nu, latent, orc.EXACT)
    assert np.isfinite(s) and np.all(np.isfinite(G))
    h = 1e-7
    for i in (0, 3, 7, 15):
        for c in range(p):
            Zp, Zm = Z.copy(), Z.copy()
            Zp[i, c] += h
            Zm[i, c] -= h
            fd = (orc.sammon(D, Zp, nu, latent, orc.EXACT, grad=False)[0]
                  - orc.sammon(D, Zm, nu, latent, orc.EXACT, grad=False)[0]) / (2 * h)
            assert fd == pytest.approx(G[i, c], rel=1e-5, abs=1e-8)


@pytest.mark.parametrize("latent", [0, 1])
def test_sammon_descent_never_increases(orc, latent):
    """The Gershgorin step keeps the descent inside the majorising quadratic."""
    w = synth.workload_small()
    X = w.X[:80]
    D = orc.dissim(X, [2.0], orc.EXACT)[0]
    Z, hist = orc.solve_sammon(D, w.Z0[0][:80], 2.0, 60, latent, orc.EXACT)
    assert np.all(np.diff(hist) <= 1e-12 * hist[0])
    assert hist[-1] < 0.9 * hist[0]


def test_sammon_zero_residual(orc):
    g = np.random.Generator(np.random.PCG64(57))
    X = g.standard_normal((20, 3))
    D = orc.dissim(X, [1.7], orc.EXACT)[0]
    s, G = orc.sammon(D, X, 1.7, orc.LATENT_GINI, orc.EXACT)
    assert s == 0.0 and np.all(G == 0.0)


# ------------------------------------------------ Algorithm 2 (alternation)
def test_alternation_on_one_dimensional_data(orc):
    """Two-coordinate rows: Delta_nu = (1/2)^(nu-1) |y_i - y_j| embeds in one
    dimension, the Sammon fit at nu reaches it, and the Kruskal stress of that
    fit against nu' is |2^(nu' - nu) - 1|: the alternation stays at nu."""
    g = np.random.Generator(np.random.PCG64(71))
    X = g.standard_normal((40, 2))
    Z0 = X[:, :1] - X[:, 1:]                       # right order, wrong scale
    nus = [1.5, 2.0, 3.0]
    best, hist, ks, Z = orc.alternate_nu(X, nus, Z0, 1500, 2, 2, orc.LATENT_EUCLID, orc.EXACT)
    assert list(hist) == [2, 2] and best == 2
    ref = [abs(2.0 ** (v - 3.0) - 1.0) for v in nus]
    np.testing.assert_allclose(ks[-1], ref, atol=2e-3)


def test_alternation_scale_invariance(orc):
    w = synth.workload_small()
    X, Z0 = w.X[:50], w.Z0[0][:50].astype(np.float64)
    nus = [1.5, 2.0, 3.0]
    b1, h1, k1, Z1 = orc.alternate_nu(X, nus, Z0, 30, 3, 1, orc.LATENT_GINI, orc.EXACT)
    b2, h2, k2, Z2 = orc.alternate_nu(3.0 * X, nus, 3.0 * Z0, 30, 3, 1, orc.LATENT_GINI, orc.EXACT)
    assert list(h1) == list(h2) and b1 == b2
    np.testing.assert_allclose(k2, k1, rtol=1e-9)
    np.testing.assert_allclose(Z2, 3.0 * Z1, rtol=1e-9, atol=1e-12)
    assert h1[0] == 1 and all(h1[t + 1] == int(np.argmin(k1[t])) for t in range(2))


# --------------------------------------------------------- classical MDS
def test_classical_mds_recovers_euclidean_configurations(orc):
    """Textbook: for Euclidean distances of points in R^p, classical MDS
    returns a configuration with exactly those distances, and the eigenvalues
    are the squared singular values of the centred points."""
    g = np.random.Generator(np.random.PCG64(81))
    Y = g.standard_normal((60, 3)) * np.array([3.0, 1.5, 0.5])
    D = squareform(pdist(Y))
    Z, lam = orc.classical_mds(D, 3)
    np.testing.assert_allclose(squareform(pdist(Z)), D, atol=1e-9)
    sv = np.linalg.svd(Y - Y.mean(axis=0), compute_uv=False)
    np.testing.assert_allclose(lam, sv ** 2, rtol=1e-10)
    # fewer dimensions: the leading principal axes
    Z2, lam2 = orc.classical_mds(D, 2)
    np.testing.assert_allclose(lam2, lam[:2], rtol=1e-12)
    np.testing.assert_allclose(np.abs(Z2), np.abs(Z[:, :2]), atol=1e-9)


def test_standardize_properties(orc):
    """Zero median, unit population variance, invariance under a positive
    affine map of each column, and Gini dissimilarities that change only by
    the per-column scale (differences remove the centre)."""
    g = np.random.Generator(np.random.PCG64(91))
    X = g.standard_t(3, size=(51, 6))
    Y = orc.standardize(X)
    np.testing.assert_allclose(np.median(Y, axis=0), 0.0, atol=1e-15)
    np.testing.assert_allclose(Y.var(axis=0), 1.0, rtol=1e-12)
    a, b = g.uniform(0.5, 3.0, 6), g.uniform(-5, 5, 6)
    np.testing.assert_allclose(orc.standardize(a * X + b), Y, rtol=1e-10, atol=1e-12)
    Xs = X / X.std(axis=0)
    np.testing.assert_allclose(orc.dissim(Y, [2.0], orc.EXACT), orc.dissim(Xs, [2.0], orc.EXACT), rtol=1e-12,
                               atol=1e-12)


# ------------------------------------------- rounding scales of the tolerances
@pytest.mark.parametrize("nu", [1.5, 2.0, 3.7])
def test_dissim_scale_bounds_and_homogeneity(orc, nu):
    """S_ij is a sum of absolute values of terms whose sum is Delta_ij:
    S >= |Delta| everywhere, symmetric, zero on the diagonal, and 1-homogeneous
    (ranks do not change under scaling by a positive power of two)."""
    X, _ = _problem(31, 25, 9, 2)
    S = orc.dissim_scale(X, nu, orc.EXACT)
    D = orc.dissim(X, [nu], orc.EXACT)[0]
    assert np.all(S >= np.abs(D) * (1 - 1e-12))
    assert np.array_equal(S, S.T) and np.all(np.diag(S) == 0.0)
    np.testing.assert_allclose(orc.dissim_scale(4.0 * X, nu, orc.EXACT), 4.0 * S, rtol=1e-13)
    # with ties (integer data) as well
    Xt = np.round(X)
    St = orc.dissim_scale(Xt, nu, orc.EXACT)
    if nu == 2.0:
        assert np.all(St >= np.abs(orc.dissim(Xt, [nu], orc.EXACT)[0]) * (1 - 1e-12))


def test_dissim_scale_closed_forms(orc):
    """At nu = 2 the distance is half the Gini mean difference, whose
    rank-free derivative is g_c = (#{b: z_b < z_c} - #{b: z_b > z_c}) / 2.
    z = (1, 2, 3, 4): g = (-3/2, -1/2, 1/2, 3/2), Delta = 5, S = 10.
    z = (-3, -1, 2, 5): every z_c g_c >= 0, so S = Delta = 13.5."""
    for z, s_ref, d_ref in (([1.0, 2.0, 3.0, 4.0], 10.0, 5.0), ([-3.0, -1.0, 2.0, 5.0], 13.5, 13.5)):
        X = np.array([z, [0.0, 0.0, 0.0, 0.0]])
        S = orc.dissim_scale(X, 2.0, orc.EXACT)
        D = orc.dissim(X, [2.0], orc.EXACT)[0]
        assert S[0, 1] == pytest.approx(s_ref, rel=1e-14)
        assert D[0, 1] == pytest.approx(d_ref, rel=1e-14)
    # the no-cancellation case holds at any nu: negative z exactly on the low ranks
    X = np.array([[-3.0, -1.0, 2.0, 5.0], [0.0, 0.0, 0.0, 0.0]])
    for nu in (1.3, 3.7):
        assert orc.dissim_scale(X, nu, orc.EXACT)[0, 1] == pytest.approx(
            orc.dissim(X, [nu], orc.EXACT)[0][0, 1], rel=1e-13)


@pytest.mark.parametrize("latent,p,loss", [(0, 2, 0), (0, 3, 0), (1, 2, 0), (1, 3, 0), (0, 2, 1), (1, 3, 1)])
def test_grad_scale_bounds(orc, latent, p, loss):
    """B_ic >= |G_ic| for the raw and the Sammon stress; two points (one term)
    give B == |G| exactly; rows of the full call match the row call."""
    X, Z = _problem(41 + p, 30, 6, p)
    D = orc.dissim(X, [2.5], orc.EXACT)[0]
    S = float(np.triu(D, 1).sum())
    fn = orc.stress if loss == 0 else orc.sammon
    _, G = fn(D, Z, 2.5, latent, orc.EXACT)
    B = orc.grad_scale(D, Z, 2.5, latent, orc.EXACT, loss, S)
    assert np.all(B >= np.abs(G) * (1 - 1e-12))
    rows = np.array([0, 11, 29])
    np.testing.assert_array_equal(orc.grad_scale_rows(D[rows], rows, Z, 2.5, latent, orc.EXACT, loss, S), B[rows])
    D2 = D[:2, :2].copy()
    _, G2 = fn(D2, Z[:2], 2.5, latent, orc.EXACT)
    B2 = orc.grad_scale(D2, Z[:2], 2.5, latent, orc.EXACT, loss, float(D2[0, 1]))
    np.testing.assert_allclose(B2, np.abs(G2), rtol=1e-14, atol=0)


@pytest.mark.parametrize("latent", [0, 1])
def test_grad_scale_equals_gradient_when_terms_share_a_sign(orc, latent):
    """Delta = 0 makes every residual r = delta >= 0.  At p = 2, the point with
    the largest Z_1 - Z_0 sees u_1 > u_0 against every other point, so every
    Gini term has the sign pattern (-, +); the point with the largest Z_0 has
    u_0 > 0 against every other point, so every Euclidean term of coordinate 0
    is positive.  Then B equals |G| there; elsewhere B > |G| somewhere."""
    g = np.random.Generator(np.random.PCG64(17))
    n = 40
    Z = g.standard_normal((n, 2))
    D = np.zeros((n, n))
    _, G = orc.stress(D, Z, 1.8, latent, orc.EXACT)
    B = orc.grad_scale(D, Z, 1.8, latent, orc.EXACT)
    if latent == 0:
        i = int(np.argmax(Z[:, 1] - Z[:, 0]))
        np.testing.assert_allclose(B[i], np.abs(G[i]), rtol=1e-13)
    else:
        i = int(np.argmax(Z[:, 0]))
        assert B[i, 0] == pytest.approx(abs(G[i, 0]), rel=1e-13)
    assert np.any(B > np.abs(G) * (1 + 1e-6))


def test_grad_scale_homogeneity(orc):
    """Scaling Delta and Z by 2: the raw-stress terms 2 r a scale by 2; the
    Sammon terms 2 r a / (S Delta) by 1/2."""
    X, Z = _problem(43, 24, 5, 3)
    D = orc.dissim(X, [2.0], orc.EXACT)[0]
    S = float(np.triu(D, 1).sum())
    B = orc.grad_scale(D, Z, 2.0, 0, orc.EXACT)
    np.testing.assert_allclose(orc.grad_scale(2 * D, 2 * Z, 2.0, 0, orc.EXACT), 2 * B, rtol=1e-13)
    Bs = orc.grad_scale(D, Z, 2.0, 0, orc.EXACT, 1, S)
    np.testing.assert_allclose(orc.grad_scale(2 * D, 2 * Z, 2.0, 0, orc.EXACT, 1, 2 * S), Bs / 2, rtol=1e-13)

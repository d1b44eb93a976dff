"""Pins for the oracle's convergence metrics (Sec. 4.1): closed forms built from sign
patterns, library special cases (numpy quantiles, scipy's 1-d Wasserstein distance), a
brute-force optimal-transport linear program on tiny inputs, and invariances."""
import numpy as np
import pytest
from scipy import optimize, stats

from oracle import metrics as OM
from workloads import walsh_chains


def test_rhat_closed_form_from_sign_patterns():
    deltas = [0.3, 1.7, 0.9]
    rec = walsh_chains(deltas)
    n = rec.shape[2]
    expect = max(dl * dl for dl in deltas) * n / (n - 1)
    assert OM.rhat_minus_one(rec) == pytest.approx(expect, rel=1e-12)


def test_rhat_affine_invariance_and_unscaled_eigenvalues():
    rng = np.random.default_rng(1)
    rec = rng.normal(size=(50, 4, 12)) + rng.normal(size=(1, 4, 12)) * 0.3
    r = OM.rhat_minus_one(rec)
    A = rng.normal(size=(4, 4)) + 3 * np.eye(4)
    rec2 = np.einsum("ij,tjn->tin", A, rec) + rng.normal(size=(1, 4, 1))
    assert OM.rhat_minus_one(rec2) == pytest.approx(r, rel=1e-9)
    # without the diagonal normalisation: the same eigenvalues (similar matrices)
    chains = rec.transpose(2, 0, 1)
    B = np.cov(chains.mean(1), rowvar=False)
    W = np.mean([np.cov(c, rowvar=False) for c in chains], axis=0)
    lam = np.linalg.eigvals(np.linalg.inv(W) @ B)
    assert np.max(np.abs(lam)) == pytest.approx(r, rel=1e-9)


def test_rhat_of_iid_chains_is_small():
    rng = np.random.default_rng(2)
    T, d, N = 2000, 3, 64
    rec = rng.normal(size=(T, d, N))
    r = OM.rhat_minus_one(rec)
    # B_ii ~ 1/T, W ~ I: the largest eigenvalue of ~ (1/T) Wishart_d(N - 1)/(N - 1)
    assert 0 < r < 5.0 / T


@pytest.mark.parametrize("p", [0.0, 0.025, 0.16, 0.5, 0.84, 0.975, 1.0, 0.3333])
def test_quantile_matches_numpy_linear_rule(p):
    v = np.random.default_rng(3).normal(size=1001)
    assert OM.quantile(v, p) == pytest.approx(np.quantile(v, p, method="linear"), abs=1e-14)


@pytest.mark.parametrize("alpha", [0.68, 0.95])
def test_credible_limits_of_a_uniform_grid(alpha):
    n = 1001
    rec = np.arange(n, dtype=np.float64).reshape(n, 1, 1)
    lo, hi = OM.credible_limits(rec, alpha)
    assert lo[0] == pytest.approx((n - 1) * (1 - alpha) / 2, abs=1e-9)
    assert hi[0] == pytest.approx((n - 1) * (1 + alpha) / 2, abs=1e-9)


@pytest.mark.parametrize("alpha,z", [(0.68, stats.norm.ppf(0.84)), (0.95, stats.norm.ppf(0.975))])
def test_credible_metric_gaussian_closed_form_and_shift(alpha, z):
    n = 20001
    mu, sd = np.array([1.5, -2.0]), np.array([0.7, 3.0])
    u = (np.arange(n) + 0.5) / n
    base = stats.norm.ppf(u)
    rec = (mu[None, :] + base[:, None] * sd[None, :])[:, :, None]  # (n, 2, 1)
    lo0, hi0 = mu - z * sd, mu + z * sd
    m, lo, hi = OM.credible_metric(rec, alpha, lo0, hi0)
    assert m < 2e-3
    # a shift s of every draw moves both limits by s: metric 2|s| / width, exactly
    s = 0.05
    m2, _, _ = OM.credible_metric(rec + np.array([s, 0.0])[None, :, None], alpha, lo, hi)
    assert m2 == pytest.approx(2 * s / (hi[0] - lo[0]), rel=1e-9)


def test_credible_limits_with_whitening():
    rng = np.random.default_rng(4)
    L = np.array([[2.0, 0.0], [0.8, 0.5]])
    mu = np.array([1.0, -1.0])
    z = rng.normal(size=(300, 2, 5))
    x = mu[None, :, None] + np.einsum("ij,tjn->tin", L, z)
    lo, hi = OM.credible_limits(x, 0.68, mu=mu, L=L)
    lo_z, hi_z = OM.credible_limits(z, 0.68)
    np.testing.assert_allclose(lo, lo_z, atol=1e-12)
    np.testing.assert_allclose(hi, hi_z, atol=1e-12)


def test_w1_matches_scipy_and_brute_force_transport():
    rng = np.random.default_rng(5)
    p, q = rng.normal(size=137), rng.normal(0.3, 1.4, size=211)
    assert OM.w1_1d(p, q) == pytest.approx(stats.wasserstein_distance(p, q), rel=1e-12)
    # tiny case: the optimal-transport linear program (uniform masses, |x - y| cost)
    p, q = rng.normal(size=5), rng.normal(size=7)
    n, m = len(p), len(q)
    cost = np.abs(p[:, None] - q[None, :]).ravel()
    a_eq = np.zeros((n + m, n * m))
    for i in range(n):
        a_eq[i, i * m:(i + 1) * m] = 1.0
    for j in range(m):
        a_eq[n + j, j::m] = 1.0
    b_eq = np.concatenate([np.full(n, 1.0 / n), np.full(m, 1.0 / m)])
    lp = optimize.linprog(cost, A_eq=a_eq, b_eq=b_eq, bounds=(0, None), method="highs")
    assert OM.w1_1d(p, q) == pytest.approx(lp.fun, rel=1e-9)


def test_sliced_wasserstein_closed_forms():
    rng = np.random.default_rng(6)
    d, K, seed = 4, 500, 77
    w = OM.directions(d, K, seed)
    np.testing.assert_allclose(np.linalg.norm(w, axis=1), 1.0, rtol=1e-14)
    # isotropic directions: E|w_1| = Gamma(d/2) / (sqrt(pi) Gamma((d+1)/2)); 5 sigma of the
    # mean of 500 draws (sd of |w_1| below 0.3)
    from math import gamma, pi, sqrt
    e1 = gamma(d / 2) / (sqrt(pi) * gamma((d + 1) / 2))
    assert abs(np.mean(np.abs(w[:, 0])) - e1) < 5 * 0.3 / np.sqrt(K)
    a = rng.normal(size=(40, d, 25))
    assert OM.sliced_wasserstein(a, a, K, seed) == 0.0
    # a rigid shift s u moves every projection by s (w . u): W1 = |s| |w . u|
    u = np.array([1.0, 2.0, -1.0, 0.5])
    s = 0.37
    sw = OM.sliced_wasserstein(a, a + s * u[None, :, None], K, seed)
    assert sw == pytest.approx(s * np.mean(np.abs(w @ u)), rel=1e-9)
    # homogeneity
    b = rng.normal(1.0, 2.0, size=(30, d, 20))
    assert OM.sliced_wasserstein(3 * a, 3 * b, 64, seed) == pytest.approx(
        3 * OM.sliced_wasserstein(a, b, 64, seed), rel=1e-12)

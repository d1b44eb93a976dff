"""Pins for the oracle's differential-evolution move (Sec. 2.3): the log-ratio of a symmetric
proposal in closed form on a Gaussian, partner bookkeeping, the law of gamma, a flat target
that accepts exactly the proposals inside the box, and stationarity of one iteration from
exact Gaussian draws."""
import numpy as np
import pytest
from scipy import stats

from oracle import samplers as S, target
from workloads import make_problem


def _gauss(n, seed):
    prob = make_problem("c2", with_mlp=False)
    L = np.linalg.cholesky(prob["closed_cov"])
    x = prob["gauss_mean"] + np.random.default_rng(seed).normal(size=(n, 6)) @ L.T
    lp, _ = target.log_target(prob, x)
    return prob, x, lp


def test_de_log_alpha_closed_form_and_partners():
    prob, x, lp = _gauss(64, 3)
    new, info = S.de_step(prob, dict(x=x, lp=lp), 5, 81, 0.1)
    k = np.arange(32)  # first half: partners from the original second half
    j, kk = info["partners"][k, 0], info["partners"][k, 1]
    assert np.all(j != kk) and np.all(j >= 32) and np.all(kk >= 32)
    assert np.all(info["partners"][32:] < 32)
    y = x[k] + info["gamma"][k, None] * (x[j] - x[kk])
    P = prob["gauss_prec"]
    r_y, r_x = y - prob["gauss_mean"], x[k] - prob["gauss_mean"]
    ref = -0.5 * np.einsum("ni,ij,nj->n", r_y, P, r_y) + 0.5 * np.einsum("ni,ij,nj->n", r_x, P, r_x)
    np.testing.assert_allclose(info["log_alpha"][k], ref, atol=1e-8)


def test_de_gamma_law():
    prob, x, lp = _gauss(20000, 4)
    g0 = 2.38 / np.sqrt(12.0)
    _, info = S.de_step(prob, dict(x=x, lp=lp), 2, 82, 0.0)
    assert np.all(info["gamma"] == g0)
    sig = 0.3
    _, info = S.de_step(prob, dict(x=x, lp=lp), 2, 82, sig)
    eta = info["gamma"] / g0 - 1.0
    assert stats.kstest(eta / sig, "norm").pvalue > 1e-4
    # partners uniform over the other half's ordered pairs: j and k each uniform
    j = info["partners"][:10000, 0] - 10000
    assert stats.chisquare(np.bincount(j // 100, minlength=100)).pvalue > 1e-4


def test_de_on_a_flat_target_accepts_exactly_the_proposals_inside_the_box():
    prob = make_problem("c2", with_mlp=False)
    prob = dict(prob, gauss_coef=0.0)
    rng = np.random.default_rng(5)
    x = prob["lower"] + rng.uniform(size=(400, 6)) * (prob["upper"] - prob["lower"])
    lp, _ = target.log_target(prob, x)
    new, info = S.de_step(prob, dict(x=x, lp=lp), 1, 83, 0.5)
    k = np.arange(200)
    j, kk = info["partners"][k, 0], info["partners"][k, 1]
    y = x[k] + info["gamma"][k, None] * (x[j] - x[kk])
    inside = np.all((y >= prob["lower"]) & (y <= prob["upper"]), axis=1)
    assert np.array_equal(info["accepted"][k], inside)
    assert 0 < inside.mean() < 1


def test_de_preserves_the_gaussian():
    """Exact draws in, one iteration, draws out: per-coordinate KS and variance (5 sigma)."""
    prob, x, lp = _gauss(20000, 6)
    new, info = S.de_step(prob, dict(x=x, lp=lp), 3, 84, 0.1)
    L = np.linalg.cholesky(prob["closed_cov"])
    z = np.linalg.solve(L, (new["x"] - prob["gauss_mean"]).T).T
    n = z.shape[0]
    for i in range(6):
        assert stats.kstest(z[:, i], "norm").pvalue > 1e-4
    assert np.all(np.abs(z.var(0) - 1) < 5 * np.sqrt(2.0 / n))
    assert 0.1 < info["accepted"].mean() < 0.9


def test_de_rejects_small_or_odd_ensembles():
    prob, x, lp = _gauss(3, 7)
    with pytest.raises(ValueError):
        S.de_step(prob, dict(x=x, lp=lp), 0, 1, 0.1)
    prob, x, lp = _gauss(2, 7)
    with pytest.raises(ValueError):
        S.de_step(prob, dict(x=x, lp=lp), 0, 1, 0.1)

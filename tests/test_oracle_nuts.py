"""Pins for the oracle's NUTS transition (Hoffman & Gelman 2014, efficient slice version):
the depth-1 special case equals a one-step HMC transition in the drawn direction with the
slice acceptance u <= exp(H0 - H1); the stationary distribution of a standard normal is
preserved by one transition (moments and a KS test from exact draws); the trajectory
stops on U-turns (a 1-d oscillator never needs the maximum depth at moderate step
sizes); leaves are counted and trees never exceed the maximum depth."""
import numpy as np
import pytest
from scipy import stats

from oracle import nuts as N, philox as ph, samplers as S
from workloads import make_problem


def _std_normal(n, seed, name="c2"):
    prob = make_problem(name, with_mlp=False)
    W = dict(mu=prob["gauss_mean"], L=np.linalg.cholesky(prob["closed_cov"]))
    z = np.random.default_rng(seed).normal(size=(n, prob["d"]))
    return prob, W, S.init_state(prob, W, W["mu"] + z @ W["L"].T)


@pytest.mark.parametrize("eps", [0.3, 0.9, 1.6])
def test_depth_one_is_one_step_hmc_with_slice_acceptance(eps):
    prob, W, st = _std_normal(200, 3)
    t, seed = 4, 91
    new, info = N.nuts_step(prob, W, st, t, seed, eps, max_depth=1)
    ids = np.arange(200, dtype=np.uint64)
    v = np.where(ph.uniforms2(seed, ids, t, N.STREAM_NUTS, 0, 0)[0] < 0.5, -1.0, 1.0)
    q0 = ph.normals(seed, ids, t, ph.STREAM_NORMAL, 0, prob["d"])
    # one leapfrog step of the oracle HMC, with the momentum flipped for v = -1 (a step of
    # -eps from (z, q) is a step of +eps from (z, -q) with the momentum flipped back)
    z1, q1, lp1, g1 = S.leapfrog(prob, W, st["z"], q0 * v[:, None], st["g"], eps, 1)
    h0 = -st["lp"] + 0.5 * np.sum(q0 * q0, 1)
    h1 = -lp1 + 0.5 * np.sum(q1 * q1, 1)
    log_u = np.log(ph.accept_uniform(seed, ids, t))
    take = log_u <= h0 - h1
    expect = np.where(take[:, None], z1, st["z"])
    np.testing.assert_allclose(new["z"], expect, atol=1e-12)
    assert np.all(info["n_leaves"] == 1) and np.all(info["depth"] == 1)
    np.testing.assert_allclose(info["accept_stat"], np.minimum(1.0, np.exp(h0 - h1)), rtol=1e-12)


@pytest.mark.parametrize("eps", [0.4, 1.1])
def test_one_transition_preserves_the_standard_normal(eps):
    """Exact draws in, one transition, draws out: marginal moments and KS against N(0, 1)
    per coordinate (4000 chains; 5-sigma Monte-Carlo bounds)."""
    prob, W, st = _std_normal(4000, 17, name="c1")
    new, info = N.nuts_step(prob, W, st, 2, 93, eps, max_depth=6)
    z = new["z"]
    n = z.shape[0]
    assert np.all(np.abs(z.mean(0)) < 5.0 / np.sqrt(n))
    assert np.all(np.abs(z.var(0) - 1.0) < 5.0 * np.sqrt(2.0 / n))
    for i in range(z.shape[1]):
        assert stats.kstest(z[:, i], "norm").pvalue > 1e-4
    # the chains really moved
    assert np.mean(np.any(z != st["z"], axis=1)) > 0.5


def test_trajectories_stop_on_u_turns():
    """On a standard normal a trajectory turns back after about half a period (length
    pi); at eps = 0.5 that is ~6 leapfrog steps, so no tree reaches depth 8."""
    prob, W, st = _std_normal(300, 5, name="c1")
    new, info = N.nuts_step(prob, W, st, 1, 95, 0.5, max_depth=8)
    assert info["depth"].max() < 8
    assert np.all(info["n_leaves"] <= 2 ** info["depth"] - 1)
    assert np.all(info["n_leaves"] >= info["depth"])
    assert 0.0 < info["accept_stat"].mean() <= 1.0


def test_depth_limit_and_leaf_count():
    """A tiny step never turns within the depth limit: every tree has 2^D - 1 leaves."""
    prob, W, st = _std_normal(20, 7, name="c1")
    new, info = N.nuts_step(prob, W, st, 1, 97, 1e-3, max_depth=5)
    assert np.all(info["depth"] == 5)
    assert np.all(info["n_leaves"] == 31)
    assert np.all(info["accept_stat"] > 0.999)

"""Pins for the oracle's NUTS transition (Hoffman & Gelman 2014, efficient slice version):
the depth-1 special case equals a one-step HMC transition in the drawn direction with the
slice acceptance u <= exp(H0 - H1); the stationary distribution of a standard normal is
preserved by one transition (moments and a KS test from exact draws); the trajectory
stops on U-turns (a 1-d oscillator never needs the maximum depth at moderate step
sizes); leaves are counted and trees never exceed the maximum depth; and, exactly, the
point a depth-4 tree selects follows the progressive-sampling law (uniform within each
doubling's valid leaves, replacement with probability min(1, n'/n)) by a chi-square test
whose negative control, a biased merge coin, fails."""
import numpy as np
import pytest
from scipy import stats

from oracle import nuts as N, philox as ph, samplers as S
from oracle.target import whitened
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


# ---- exact selection law of the tree (merges at every depth) ----------------------------
def _bumpy_problem():
    """1-d target: a wide Gaussian (precision 0.02) plus 4 x a 16-wide tanh network of the
    input, identity whitening.  The network's bumps make the leapfrog energy error change
    sign along a trajectory, so a slice threshold leaves valid and invalid leaves."""
    from workloads import xavier_mlp
    prob = dict(name="bumpy1", d=1, lower=np.array([-60.0]), upper=np.array([60.0]),
                gauss_coef=0.02, gauss_mean=np.zeros(1), gauss_prec=np.eye(1), twist=None,
                width=16, n_hidden=1,
                mlp_params=xavier_mlp(np.random.default_rng(0), 1, 16, 1),
                in_center=np.zeros(1), in_invscale=np.ones(1), mlp_coef=4.0, offset=0.0,
                plain=None, plain_mode=0, train_lo=None, train_hi=None)
    return prob, dict(mu=np.zeros(1), L=np.eye(1))


def _forward_trajectory(prob, W, z0, q0, eps, n_steps):
    """Kick-drift-kick leapfrog, written out here (the target's value and gradient from the
    pinned target module): the leaves of a tree whose doublings all go forward, in order,
    with their momenta and energies H - H(z0, q0)."""
    def lg(z):
        lp, g, _ = whitened(prob, W["mu"], W["L"], np.array([[z]]), with_box=False)
        return float(lp[0]), float(g[0, 0])
    lp, g = lg(z0)
    h0 = -lp + 0.5 * q0 * q0
    z, q = z0, q0
    zs, qs, dh = [], [], []
    for _ in range(n_steps):
        qh = q + 0.5 * eps * g
        z = z + eps * qh
        lp, g = lg(z)
        q = qh + 0.5 * eps * g
        zs.append(z)
        qs.append(q)
        dh.append(-lp + 0.5 * q * q - h0)
    return np.array(zs), np.array(qs), np.array(dh)


def _exact_selection(valid, depth):
    """P(final point) over [start, leaf 1 .. leaf 2^D - 1] for a tree that never stops:
    doubling j appends leaves 2^j .. 2^(j+1) - 1; its candidate is uniform over its valid
    leaves (the merge coins n2 / (n1 + n2) compose to that) and replaces the tree's with
    probability min(1, n' / n), n the valid count so far, start included."""
    p = np.zeros(len(valid) + 1)
    n = 1.0
    probs = []
    for j in range(depth):
        lo, hi = (1 << j) - 1, (1 << (j + 1)) - 1   # 0-based leaf slice of doubling j
        nj = float(valid[lo:hi].sum())
        probs.append((lo, hi, nj, min(1.0, nj / n)))
        n += nj
    for j, (lo, hi, nj, pr) in enumerate(probs):
        later = np.prod([1.0 - q[3] for q in probs[j + 1:]])
        if nj > 0:
            p[1 + lo:1 + hi] = valid[lo:hi] * (pr * later / nj)
    p[0] = np.prod([1.0 - q[3] for q in probs])
    return p


def test_exact_selection_law_closed_forms():
    # all leaves valid: doubling j replaces with probability 2^j / 2^j = 1, so the last
    # doubling's leaves are uniform
    p = _exact_selection(np.ones(7), 3)
    np.testing.assert_allclose(p, [0, 0, 0, 0, .25, .25, .25, .25], atol=1e-15)
    # only leaf 1 valid: it replaces the start with probability 1 / 1
    p = _exact_selection(np.array([1, 0, 0, 0, 0, 0, 0.]), 3)
    np.testing.assert_allclose(p, [0, 1, 0, 0, 0, 0, 0, 0], atol=1e-15)
    # leaves 1, 2, 7 valid: leaf 1 replaces the start (1/1), leaf 2 replaces it with 1/2,
    # leaf 7 with 1/3 -- each of the three ends with 1/3
    p = _exact_selection(np.array([1, 1, 0, 0, 0, 0, 1.]), 3)
    np.testing.assert_allclose(p, [0, 1 / 3, 1 / 3, 0, 0, 0, 0, 1 / 3], atol=1e-15)


@pytest.mark.parametrize("biased", [False, True])
def test_tree_selects_its_point_with_the_exact_progressive_law(monkeypatch, biased):
    """Depth-4 tree, every doubling forced forward, its replacement and merge uniforms
    redrawn on each of 12000 repetitions (the oracle's random source patched); momentum and
    slice variable stay those of the chain.  The start and chain are chosen so that the
    trajectory never turns and the slice leaves valid points [1 | 0 0 | 1 1 1 1 |
    1 1 1 1 1 0 0 0]: the last doubling replaces with probability 5/6 and its depth-3 merge
    takes the 1-valid sibling with probability 1/5.  The chosen point's frequencies match the
    law (chi-square p > 1e-4).  With a biased merge coin (u^2 in place of u, planted in the
    oracle's random source) the same check rejects (p < 1e-6)."""
    prob, W = _bumpy_problem()
    seed, t, eps, depth, chain, z0 = 5, 3, 0.8, 4, 605, -3.0
    ids = np.array([chain], dtype=np.uint64)
    q0 = float(ph.normals(seed, ids, t, ph.STREAM_NORMAL, 0, 1)[0, 0])
    log_u = float(np.log(ph.accept_uniform(seed, ids, t))[0])
    zs, qs, dh = _forward_trajectory(prob, W, z0, q0, eps, (1 << depth) - 1)
    assert np.all(qs > 0) and np.all(np.diff(np.concatenate([[z0], zs])) > 0)  # no U-turn
    valid = (log_u <= -dh).astype(float)
    np.testing.assert_array_equal(valid, [1, 0, 0, 1, 1, 1, 1, 1, 1, 1, 1, 1, 0, 0, 0])
    assert np.min(np.abs(log_u + dh)) > 1e-5          # no leaf on the threshold
    rng = np.random.default_rng(11)

    def patched(seed_, chain_, t_, sub, blk):
        if sub < 16:                     # doubling sub: forward, replacement uniform
            return 0.75, float(rng.uniform())
        u = float(rng.uniform())         # merge coin
        return (u * u if biased else u), 0.0

    monkeypatch.setattr(N, "_u", patched)
    st = S.init_state(prob, W, np.array([[z0]]))
    counts = np.zeros(len(zs) + 1)
    reps = 12000
    for _ in range(reps):
        new, info = N.nuts_step(prob, W, st, t, seed, eps, max_depth=depth, chains=ids)
        assert info["depth"][0] == depth and info["n_leaves"][0] == len(zs)
        z = new["z"][0, 0]
        k = 0 if z == z0 else 1 + int(np.argmin(np.abs(zs - z)))
        assert k == 0 or abs(zs[k - 1] - z) < 1e-12
        counts[k] += 1
    p = _exact_selection(valid, depth)
    assert abs(p.sum() - 1.0) < 1e-12
    np.testing.assert_allclose(p[8:13], 1.0 / 6.0, atol=1e-15)
    keep = p > 0
    assert counts[~keep].sum() == 0       # never an invalid leaf, never a wiped point
    chi2 = np.sum((counts[keep] - reps * p[keep]) ** 2 / (reps * p[keep]))
    pval = stats.chi2.sf(chi2, keep.sum() - 1)
    if biased:
        assert pval < 1e-6, pval
    else:
        assert pval > 1e-4, (pval, counts, reps * p)

"""Pins for the oracle's adaptation (moments, jittered Cholesky, dual averaging), the
multi-chain ESS, and the training pieces (MSE gradient, Adam, importance weights)."""
import numpy as np
import pytest

from oracle import adapt, ess, mlp, train
from workloads import ar1_chains, latin_hypercube, spd_with_condition, xavier_mlp


def test_moments_of_a_known_sample():
    # the 2^3 corners of a cube scaled per axis: mean 0, cov = diag(s^2) * 8/7
    s = np.array([1.0, 2.0, 3.0])
    pts = np.array([[i, j, k] for i in (-1, 1) for j in (-1, 1) for k in (-1, 1)]) * s
    m, c = adapt.ensemble_moments(pts)
    np.testing.assert_allclose(m, 0, atol=1e-15)
    np.testing.assert_allclose(c, np.diag(s * s) * 8 / 7, atol=1e-14)


def test_cholesky_round_trip_and_library_agreement():
    rng = np.random.default_rng(0)
    S, _, _ = spd_with_condition(rng, 27, 1e3)
    L, jit = adapt.regularised_cholesky(S)
    assert jit == 0.0
    np.testing.assert_allclose(L @ L.T, S, atol=1e-12 * np.abs(S).max())
    np.testing.assert_allclose(L, np.linalg.cholesky(S), atol=1e-12)
    assert np.all(np.triu(L, 1) == 0)


def test_singular_covariance_takes_jitter_path():
    v = np.array([1.0, 2.0, -1.0])
    S = np.outer(v, v)  # rank one
    L, jit = adapt.regularised_cholesky(S)
    assert jit > 0
    np.testing.assert_allclose(L @ L.T, S + jit * np.eye(3), atol=1e-12)


def test_nan_covariance_fails():
    with pytest.raises(np.linalg.LinAlgError):
        adapt.regularised_cholesky(np.full((2, 2), np.nan))


def test_dual_averaging_reaches_closed_form_target():
    """With a deterministic acceptance curve alpha(eps) = exp(-eps), the averaged step size
    converges to eps* = -ln(delta)."""
    for delta in (0.57, 0.8):
        da = adapt.DualAveraging(1.0, delta)
        eps = 1.0
        for _ in range(4000):
            eps = da.update(np.exp(-eps))
        assert da.final == pytest.approx(-np.log(delta), rel=0.01)


def test_fft_autocovariance_matches_brute_force():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(3, 50))
    ac = ess.autocov_fft(x)
    y = x - x.mean(1, keepdims=True)
    for t in (0, 1, 7, 49):
        ref = np.sum(y[:, :50 - t] * y[:, t:], 1) / 50
        np.testing.assert_allclose(ac[:, t], ref, atol=1e-12)


@pytest.mark.parametrize("rho", [0.0, 0.5, 0.9])
def test_ess_of_ar1_chains(rho):
    """AR(1) chains: integrated autocorrelation time tau = (1 + rho)/(1 - rho)."""
    x = ar1_chains(np.random.default_rng(int(rho * 10) + 2), rho, 32, 4000)
    e = ess.ess(x)
    ref = x.size * (1 - rho) / (1 + rho)
    assert abs(e / ref - 1) < 0.08


def test_ess_of_exactly_alternating_chains_hits_the_tau_floor():
    """x_t = (-1)^t: rho_1 = -1 makes the first pair sum 0, the truncated Geyer sum is
    empty and tau would be -1; the floor 1 / log10(M T) gives ESS = M T log10(M T)."""
    M, T = 8, 200
    x = np.tile(np.where(np.arange(T) % 2 == 0, 1.0, -1.0), (M, 1))
    assert ess.ess(x) == pytest.approx(M * T * np.log10(M * T), rel=1e-12)


def test_ess_of_constant_chains_is_flagged_frozen():
    """Chains that never move (nothing accepted): W = 0, no estimate.  Whether the chains
    sit at one value (0/0 autocorrelations) or at different values (rho_t = 1 at every
    lag, which used to give M T / (2 T - 1)), the ESS is 0 with the frozen flag."""
    M, T = 4096, 20
    same = np.full((M, T), 1.25)
    start = np.random.default_rng(11).normal(size=(M, 1))
    spread = np.repeat(start, T, axis=1)
    for x in (same, spread):
        e, flag = ess.ess_flagged(x)
        assert e == 0.0 and flag == ess.FLAG_FROZEN
        assert ess.ess(x) == 0.0
    # one parameter frozen, the others not: min_ess reports 0 and names the frozen one
    rng = np.random.default_rng(12)
    samples = np.stack([rng.normal(size=(T, 64)), np.ones((T, 64)), rng.normal(size=(T, 64))],
                       axis=2)
    m, per, flags = ess.min_ess(samples)
    assert m == 0.0 and per[1] == 0.0
    assert list(flags) == [ess.FLAG_OK, ess.FLAG_FROZEN, ess.FLAG_OK]


def test_ess_of_a_window_shorter_than_tau_is_flagged_untruncated():
    """AR(1) chains with coefficient 0.999 (tau = 1999) started from their stationary law
    and observed for 50 steps: the between-chain variance dominates var+, every pair sum the
    window holds stays positive and the Geyer sequence is cut by the window, not by the
    autocorrelation.  The estimate is flagged, and it is far below the M T draws."""
    x = ar1_chains(np.random.default_rng(13), 0.999, 32, 50)
    e, flag = ess.ess_flagged(x)
    assert flag == ess.FLAG_UNTRUNCATED
    assert e < 0.1 * x.size
    # a well-mixing window of the same size ends its Geyer sequence inside the window
    y = ar1_chains(np.random.default_rng(14), 0.3, 32, 50)
    assert ess.ess_flagged(y)[1] == ess.FLAG_OK


def test_cosine_learning_rate_closed_forms():
    """lr(s) = lr1 + (lr0 - lr1)(1 + cos(pi s / S)) / 2: lr0 at s = 0, the midpoint of the
    two rates at s = S / 2, lr1 at s = S, and a quarter of the way down at s = S / 3
    (cos(pi / 3) = 1/2)."""
    lr0, lr1, S = 1e-3, 1e-5, 600
    assert train.cosine_lr(0, S, lr0, lr1) == pytest.approx(lr0, rel=1e-15)
    assert train.cosine_lr(S // 2, S, lr0, lr1) == pytest.approx(0.5 * (lr0 + lr1), rel=1e-14)
    assert train.cosine_lr(S, S, lr0, lr1) == pytest.approx(lr1, rel=1e-12)
    assert train.cosine_lr(S // 3, S, lr0, lr1) == pytest.approx(lr1 + 0.75 * (lr0 - lr1),
                                                                 rel=1e-14)
    # monotone decreasing between the ends
    v = [train.cosine_lr(s, S, lr0, lr1) for s in range(S + 1)]
    assert all(a >= b for a, b in zip(v, v[1:]))


def test_first_adam_step_closed_form():
    rng = np.random.default_rng(2)
    p = rng.normal(size=10)
    g = rng.normal(size=10)
    opt = train.Adam(10)
    p1 = opt.step(p, g, 1e-3)
    np.testing.assert_allclose(p1, p - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_mse_gradient_matches_central_differences():
    rng = np.random.default_rng(3)
    d, w, nh = 3, 8, 2
    p = xavier_mlp(rng, d, w, nh) + rng.normal(0, 0.1, size=1)
    th = rng.uniform(-1, 1, size=(16, d))
    y = rng.normal(size=16)
    _, g = train.mse_loss_grad(p, th, y, d, w, nh)
    fd = np.zeros_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = 1e-6
        fd[i] = (train.mse_loss_grad(p + e, th, y, d, w, nh)[0]
                 - train.mse_loss_grad(p - e, th, y, d, w, nh)[0]) / 2e-6
    np.testing.assert_allclose(g, fd, rtol=1e-5, atol=1e-8)


def test_training_fits_a_smooth_function():
    rng = np.random.default_rng(4)
    d, w, nh = 2, 16, 2
    th = latin_hypercube(rng, 512, d) * 2 - 1
    y = -(th ** 2).sum(1)
    yh, mu, sig = train.standardise(y)
    perms = [rng.permutation(512) for _ in range(150)]
    p, losses = train.train(xavier_mlp(rng, d, w, nh), th, yh, perms, 64, 1e-2, 1e-4, d, w, nh)
    assert losses[-1] < 0.02 * losses[0]


def test_importance_weights_of_exact_emulator_are_uniform():
    ll = np.random.default_rng(5).normal(size=100) * 30
    w = train.importance_weights(ll, ll)
    np.testing.assert_allclose(w, 0.01, rtol=1e-12)
    assert train.kish_ess(w) == pytest.approx(100)


def test_latin_hypercube_hits_every_stratum_once():
    u = latin_hypercube(np.random.default_rng(6), 1000, 4)
    for j in range(4):
        assert np.array_equal(np.sort(np.floor(u[:, j] * 1000).astype(int)), np.arange(1000))

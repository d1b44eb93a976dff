"""Pins for the oracle's emulator MLP, target densities, plain model and whitening."""
import numpy as np
import pytest
from scipy import stats

from oracle import mlp, target
from workloads import make_problem, small_problem, mlp_nparams, xavier_mlp
from workloads.synth import _simulate_spectrum


def _fd_grad(f, x, h_rel=1e-6):
    x = np.array(x, dtype=np.float64)
    g = np.zeros_like(x)
    for i in range(x.size):
        h = h_rel * max(1.0, abs(x.flat[i]))
        e = np.zeros_like(x)
        e.flat[i] = h
        g.flat[i] = (f(x + e) - f(x - e)) / (2 * h)
    return g


@pytest.mark.parametrize("d,width,nh", [(6, 16, 1), (6, 32, 3), (12, 24, 4)])
def test_mlp_input_grad_matches_central_differences(d, width, nh):
    rng = np.random.default_rng(d * 100 + nh)
    p = xavier_mlp(rng, d, width, nh)
    p += rng.normal(0, 0.05, size=p.size)  # nonzero biases too
    th = rng.normal(size=(4, d))
    out, g = mlp.value_and_input_grad(p, th, d, width, nh)
    for c in range(4):
        fd = _fd_grad(lambda t: mlp.forward(p, t[None, :], d, width, nh)[0][0], th[c])
        np.testing.assert_allclose(g[c], fd, rtol=1e-7, atol=1e-9)


def test_mlp_identity_activation_collapses_to_affine_map():
    rng = np.random.default_rng(3)
    d, w, nh = 4, 8, 3
    p = rng.normal(size=mlp_nparams(d, w, nh))
    Ws, bs, wo, bo = mlp.unpack(p, d, w, nh)
    A = np.eye(d)
    c = np.zeros(d)
    for W, b in zip(Ws, bs):  # compose the affine maps by hand
        c = W @ c + b
        A = W @ A
    th = rng.normal(size=(5, d))
    out, _ = mlp.forward(p, th, d, w, nh, activation=lambda v: v)
    np.testing.assert_allclose(out, th @ (wo @ A) + wo @ c + bo, rtol=1e-12)


def test_mlp_zero_output_weights_gives_bias():
    rng = np.random.default_rng(4)
    d, w, nh = 3, 16, 2
    p = rng.normal(size=mlp_nparams(d, w, nh))
    Ws, bs, wo, bo = mlp.unpack(p, d, w, nh)
    p2 = mlp.pack(Ws, bs, np.zeros_like(wo), 1.25)
    out, g = mlp.value_and_input_grad(p2, rng.normal(size=(7, d)), d, w, nh)
    assert np.all(out == 1.25) and np.all(g == 0)


def test_mlp_param_grad_matches_central_differences():
    rng = np.random.default_rng(5)
    d, w, nh = 3, 6, 3
    p = rng.normal(0, 0.5, size=mlp_nparams(d, w, nh))
    th = rng.normal(size=(5, d))
    up = rng.normal(size=5)
    g, _ = mlp.param_grad(p, th, up, d, w, nh)
    fd = _fd_grad(lambda q: float(up @ mlp.forward(q, th, d, w, nh)[0]), p)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-9)


def test_gaussian_part_matches_scipy_logpdf():
    prob = make_problem("c2", with_mlp=False)
    rng = np.random.default_rng(0)
    x = prob["gauss_mean"] + rng.normal(size=(6, 6)) * 3
    lp, _ = target.log_target(prob, x)
    ref = stats.multivariate_normal(prob["gauss_mean"], prob["closed_cov"]).logpdf(x)
    # equal up to the normalising constant
    np.testing.assert_allclose(lp - ref, np.full(6, (lp - ref)[0]), atol=1e-9)


@pytest.mark.parametrize("name", ["c1", "c3", "c5"])
def test_full_target_gradient_matches_central_differences(name):
    prob = make_problem(name)
    rng = np.random.default_rng(1)
    sd = np.sqrt(np.diag(prob["closed_cov"]))
    x = prob["gauss_mean"] + rng.normal(size=(3, prob["d"])) * sd
    _, g = target.log_target(prob, x)
    for c in range(3):
        fd = _fd_grad(lambda v: target.log_target(prob, v[None, :])[0][0], x[c])
        np.testing.assert_allclose(g[c], fd, rtol=2e-6, atol=1e-7 * np.abs(g[c]).max())


def test_box_prior_is_hard():
    prob = make_problem("c2")
    x = np.stack([prob["upper"] + 1e-9, prob["upper"], prob["lower"]])
    lp, g = target.log_target(prob, x)
    assert lp[0] == -np.inf and np.isfinite(lp[1]) and np.isfinite(lp[2])
    assert np.all(np.isfinite(g))


def test_twisted_pair_has_closed_form_moments():
    """Sampling the latent construction directly reproduces the closed-form covariance the
    generator states, and the density's gradient vanishes at the mode (MLP off)."""
    prob = small_problem(d=4, twist=True, with_mlp=False)
    tw = prob["twist"]
    rng = np.random.default_rng(2)
    n = 400000
    sig_u = np.sqrt(tw["kappa"])
    sig_w = 1.0 / np.sqrt(prob["gauss_prec"][tw["v"], tw["v"]])
    xu = tw["center"] + sig_u * rng.normal(size=n)
    xv = prob["gauss_mean"][tw["v"]] + sig_w * rng.normal(size=n) - tw["beta"] * (
        (xu - tw["center"]) ** 2 - tw["kappa"])
    assert abs(np.var(xv) / prob["closed_cov"][tw["v"], tw["v"]] - 1) < 0.02
    # the Gaussian block: its closed-form covariance inverts its precision block
    gi = [i for i in range(prob["d"]) if i not in (tw["u"], tw["v"])]
    np.testing.assert_allclose(prob["closed_cov"][np.ix_(gi, gi)] @ prob["gauss_prec"][np.ix_(gi, gi)],
                               np.eye(len(gi)), atol=1e-10)
    x = np.tile(prob["gauss_mean"], (1, 1))
    x[0, tw["u"]] = tw["center"]
    x[0, tw["v"]] = prob["gauss_mean"][tw["v"]] + tw["beta"] * tw["kappa"]
    _, g = target.log_target(prob, x)
    np.testing.assert_allclose(g, 0.0, atol=1e-12)


def test_whitened_standard_normal_identity():
    """MLP off and (mu, L) = (m, chol S): log pi_z(z) = -|z|^2/2 + const, grad_z = -z, and
    p^T Sigma p = q^T q for p = L^{-T} q (Sec. 2.2)."""
    prob = make_problem("c5", with_mlp=False)
    L = np.linalg.cholesky(prob["closed_cov"])
    mu = prob["gauss_mean"]
    rng = np.random.default_rng(3)
    z = rng.normal(size=(8, prob["d"]))
    lpz, gz, x = target.whitened(prob, mu, L, z)
    const = lpz + 0.5 * np.sum(z * z, 1)
    np.testing.assert_allclose(const, const[0], atol=1e-9)
    np.testing.assert_allclose(gz, -z, atol=1e-9)
    q = rng.normal(size=prob["d"])
    p = np.linalg.solve(L.T, q)
    assert abs(p @ prob["closed_cov"] @ p - q @ q) < 1e-9 * (q @ q)


def test_plain_model_zero_chi2_at_truth_without_noise():
    """The oracle's spectrum model reproduces the independent data simulator: with the
    noise switched off the chi^2 at the true parameters is exactly zero."""
    prob = make_problem("c4")
    pl = dict(prob["plain"])
    t_star = (pl["theta_star"] - pl["center"]) * pl["invscale"]
    pl["data"] = _simulate_spectrum(t_star, pl["xgrid"], pl["a"], pl["g"], pl["p"], pl["k"],
                                    pl["gamma0"])
    v, g = target.plain_logL(pl, pl["theta_star"][None, :])
    assert abs(v[0]) < 1e-18
    np.testing.assert_allclose(g, 0.0, atol=1e-9)


def test_plain_model_gradient_matches_central_differences():
    prob = make_problem("c4")
    pl = prob["plain"]
    rng = np.random.default_rng(4)
    th = pl["theta_star"] + rng.normal(size=(2, 6)) * 0.01 / pl["invscale"]
    _, g = target.plain_logL(pl, th)
    for c in range(2):
        fd = _fd_grad(lambda v: target.plain_logL(pl, v[None, :])[0][0], th[c], 1e-7)
        np.testing.assert_allclose(g[c], fd, rtol=1e-5, atol=1e-6 * np.abs(g[c]).max())


def test_emulator_fallback_switches_at_training_box():
    prob = make_problem("c4")
    prob = dict(prob, plain_mode=1)
    inside = 0.5 * (prob["train_lo"] + prob["train_hi"])
    outside = prob["train_hi"] + 0.1 * (prob["train_hi"] - prob["train_lo"])
    lp, _ = target.log_target(prob, np.stack([inside, outside]))
    mv, _ = target.mlp_part(prob, inside[None, :])
    pv, _ = target.plain_logL(prob["plain"], outside[None, :])
    assert lp[0] == pytest.approx(mv[0], abs=1e-12)
    assert lp[1] == pytest.approx(pv[0], rel=1e-12)

"""Pins for the oracle's MH / MALA / HMC / AIES transitions: exact closed forms of log alpha
on a standard normal (whitened, MLP off), leapfrog invariants, stretch-move law, and
Gaussian moment recovery within Monte-Carlo error."""
import numpy as np
import pytest
from scipy import stats

from oracle import philox as ph, samplers as S, target
from oracle.adapt import ensemble_moments
from workloads import make_problem, small_problem


def _std_normal_setup(name="c2", n=256, seed=11, spread=1.0):
    prob = make_problem(name, with_mlp=False)
    W = dict(mu=prob["gauss_mean"], L=np.linalg.cholesky(prob["closed_cov"]))
    rng = np.random.default_rng(seed)
    z = rng.normal(size=(n, prob["d"])) * spread
    st = S.init_state(prob, W, W["mu"] + z @ W["L"].T)
    return prob, W, st


def test_mh_log_alpha_closed_form():
    prob, W, st = _std_normal_setup()
    new, info = S.mh_step(prob, W, st, 3, 77, 0.7)
    z, zp = st["z"], info["proposal"]
    ref = 0.5 * (np.sum(z * z, 1) - np.sum(zp * zp, 1))
    np.testing.assert_allclose(info["log_alpha"], ref, atol=1e-9)
    xi = ph.normals(77, np.arange(256, dtype=np.uint64), 3, ph.STREAM_NORMAL, 0, prob["d"])
    np.testing.assert_allclose(zp, z + 0.7 * xi, atol=1e-12)


@pytest.mark.parametrize("eps", [0.05, 0.4, 1.1])
def test_mala_log_alpha_closed_form(eps):
    """On N(0, I): log alpha = (eps/4)(|z|^2 - |z'|^2) exactly (Sec. 2.1 proposal)."""
    prob, W, st = _std_normal_setup()
    new, info = S.mala_step(prob, W, st, 5, 78, eps)
    z, zp = st["z"], info["proposal"]
    ref = eps / 4.0 * (np.sum(z * z, 1) - np.sum(zp * zp, 1))
    np.testing.assert_allclose(info["log_alpha"], ref, atol=1e-9)


def test_mala_step_multipliers():
    """Per-dimension steps eps_i = eps m_i: on N(0, I) the coordinates are independent, so
    log alpha = sum_i (eps_i/4)(z_i^2 - z'_i^2); m = 1 gives the plain MALA bit for bit;
    MH with multipliers scales each proposal coordinate."""
    prob, W, st = _std_normal_setup()
    d = prob["d"]
    m = np.linspace(0.5, 10.0, d)
    new, info = S.mala_step(prob, W, st, 5, 79, 0.3, mult=m)
    z, zp = st["z"], info["proposal"]
    ref = np.sum(0.3 * m / 4.0 * (z * z - zp * zp), axis=1)
    np.testing.assert_allclose(info["log_alpha"], ref, atol=1e-9)
    a, ia = S.mala_step(prob, W, st, 5, 79, 0.3)
    b, ib = S.mala_step(prob, W, st, 5, 79, 0.3, mult=np.ones(d))
    np.testing.assert_allclose(ia["log_alpha"], ib["log_alpha"], rtol=1e-13, atol=1e-13)
    assert np.array_equal(ia["proposal"], ib["proposal"])
    _, im = S.mh_step(prob, W, st, 5, 79, 0.7, mult=m)
    xi = ph.normals(79, np.arange(st["z"].shape[0], dtype=np.uint64), 5, ph.STREAM_NORMAL, 0, d)
    np.testing.assert_allclose(im["proposal"], st["z"] + 0.7 * m * xi, atol=1e-12)


def test_mala_with_multipliers_preserves_the_standard_normal():
    prob = make_problem("c1", with_mlp=False)
    W = dict(mu=prob["gauss_mean"], L=np.linalg.cholesky(prob["closed_cov"]))
    z = np.random.default_rng(31).normal(size=(20000, prob["d"]))
    st = S.init_state(prob, W, W["mu"] + z @ W["L"].T)
    m = np.array([1.0, 10.0, 1.0, 3.0, 0.3, 1.0])[:prob["d"]]
    new, info = S.mala_step(prob, W, st, 2, 80, 0.2, mult=m)
    n = z.shape[0]
    for i in range(prob["d"]):
        assert stats.kstest(new["z"][:, i], "norm").pvalue > 1e-4
    assert np.all(np.abs(new["z"].var(0) - 1) < 5 * np.sqrt(2.0 / n))
    assert 0.05 < info["accepted"].mean() < 0.95


def test_mala_small_step_accepts_everything():
    prob, W, st = _std_normal_setup()
    _, info = S.mala_step(prob, W, st, 5, 78, 1e-8)
    assert info["accepted"].mean() == 1.0


@pytest.mark.parametrize("eps,nl", [(0.1, 10), (0.5, 3), (1.3, 7)])
def test_hmc_energy_error_closed_form(eps, nl):
    """Leapfrog on N(0, I) conserves |q|^2/2 + (1 - eps^2/4)|z|^2/2 exactly, hence
    H_end - H_start = (eps^2/8)(|z_L|^2 - |z_0|^2)."""
    prob, W, st = _std_normal_setup()
    new, info = S.hmc_step(prob, W, st, 2, 79, eps, nl)
    z0, zl = st["z"], info["proposal"]
    ref = eps * eps / 8.0 * (np.sum(zl * zl, 1) - np.sum(z0 * z0, 1))
    np.testing.assert_allclose(info["h1"] - info["h0"], ref, atol=1e-8)


def test_leapfrog_reversibility_with_mlp():
    prob = make_problem("c2")
    W = dict(mu=prob["gauss_mean"], L=np.linalg.cholesky(prob["closed_cov"]))
    rng = np.random.default_rng(5)
    st = S.init_state(prob, W, W["mu"] + rng.normal(size=(4, 6)) @ W["L"].T)
    q = rng.normal(size=(4, 6))
    z1, q1, _, g1 = S.leapfrog(prob, W, st["z"], q, st["g"], 0.2, 10)
    z2, q2, _, _ = S.leapfrog(prob, W, z1, -q1, g1, 0.2, 10)
    np.testing.assert_allclose(z2, st["z"], atol=1e-12)
    np.testing.assert_allclose(-q2, q, atol=1e-12)


def test_leapfrog_energy_error_is_second_order():
    """At fixed trajectory length T = L eps the energy error shrinks as eps^2 (MLP on)."""
    prob = make_problem("c2")
    W = dict(mu=prob["gauss_mean"], L=np.linalg.cholesky(prob["closed_cov"]))
    rng = np.random.default_rng(6)
    st = S.init_state(prob, W, W["mu"] + rng.normal(size=(64, 6)) @ W["L"].T)
    q = rng.normal(size=(64, 6))
    errs = []
    for eps in (0.2, 0.1, 0.05):
        nl = int(round(1.0 / eps))
        z1, q1, lp1, _ = S.leapfrog(prob, W, st["z"], q, st["g"], eps, nl)
        dh = (-lp1 + 0.5 * np.sum(q1 * q1, 1)) - (-st["lp"] + 0.5 * np.sum(q * q, 1))
        errs.append(np.sqrt(np.mean(dh * dh)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.3 < r1 < 4.8 and 3.3 < r2 < 4.8


def test_stretch_variable_law():
    """z = ((a-1)u+1)^2/a has CDF (sqrt(a t) - 1)/(a - 1) on [1/a, a] and E z = (a+1+1/a)/3."""
    ids = np.arange(200000, dtype=np.uint64)
    _, ub = ph.uniforms2(3, ids, 0, ph.STREAM_AIES, 0, 0)
    for a in (2.0, 3.5):
        z = S.stretch_z(ub, a)
        assert z.min() >= 1 / a and z.max() <= a
        cdf = lambda t: np.clip((np.sqrt(a * t) - 1) / (a - 1), 0, 1)
        assert stats.kstest(z, cdf).pvalue > 1e-4
        assert abs(z.mean() - (a + 1 + 1 / a) / 3) < 5 * z.std() / np.sqrt(z.size)


def test_aies_log_alpha_closed_form():
    prob = make_problem("c2", with_mlp=False)
    L = np.linalg.cholesky(prob["closed_cov"])
    rng = np.random.default_rng(7)
    x = prob["gauss_mean"] + rng.normal(size=(64, 6)) @ L.T
    lp, _ = target.log_target(prob, x)
    new, info = S.aies_step(prob, dict(x=x, lp=lp), 4, 80, 2.0)
    # first half: partners from the original second half
    k = np.arange(32)
    j, zz = info["partner"][k], info["z"][k]
    y = x[j] + zz[:, None] * (x[k] - x[j])
    P = prob["gauss_prec"]
    r_y, r_x = y - prob["gauss_mean"], x[k] - prob["gauss_mean"]
    ref = 5 * np.log(zz) - 0.5 * np.einsum("ni,ij,nj->n", r_y, P, r_y) + 0.5 * np.einsum(
        "ni,ij,nj->n", r_x, P, r_x)
    np.testing.assert_allclose(info["log_alpha"][k], ref, atol=1e-8)
    assert np.all(j >= 32) and np.all(info["partner"][32:] < 32)


def test_aies_rejects_odd_ensemble():
    prob = make_problem("c2", with_mlp=False)
    x = np.tile(prob["gauss_mean"], (3, 1))
    with pytest.raises(ValueError):
        S.aies_step(prob, dict(x=x, lp=np.zeros(3)), 0, 1)


def _check_moments(samples, mean, cov, ess_frac, tol_cov=0.08):
    m, c = ensemble_moments(samples)
    sd = np.sqrt(np.diag(cov))
    n_eff = samples.shape[0] * samples.shape[1] * ess_frac
    assert np.all(np.abs(m - mean) / sd < 5.0 / np.sqrt(n_eff)), (m - mean) / sd
    Li = np.linalg.inv(np.linalg.cholesky(cov))
    dev = np.linalg.norm(Li @ c @ Li.T - np.eye(cov.shape[0]), 2)
    assert dev < tol_cov, dev


@pytest.mark.parametrize("sampler", ["mh", "mala", "hmc", "aies"])
def test_gaussian_recovery(sampler):
    prob = small_problem(d=3, with_mlp=False, seed=21)
    L = np.linalg.cholesky(prob["closed_cov"])
    W = dict(mu=prob["gauss_mean"], L=L)
    rng = np.random.default_rng(8)
    n = 512
    x0 = prob["gauss_mean"] + rng.normal(size=(n, 3)) @ L.T
    kw = dict(mh=dict(scale=2.4 / np.sqrt(3)), mala=dict(eps=0.6), hmc=dict(eps=0.5, n_leap=5),
              aies=dict(a=2.0))[sampler]
    if sampler == "aies":
        lp, _ = target.log_target(prob, x0)
        st = dict(x=x0, lp=lp)
    else:
        st = S.init_state(prob, W, x0)
    _, samp, acc = S.run(prob, W, sampler, st, 1001, 0, 300, **kw)
    frac = dict(mh=0.08, mala=0.2, hmc=0.3, aies=0.05)[sampler]
    _check_moments(samp[50:], prob["closed_mean"], prob["closed_cov"], frac)
    if sampler == "mh":
        assert 0.2 < acc.mean() < 0.45

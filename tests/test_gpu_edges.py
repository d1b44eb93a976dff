"""GPU edge cases against the FP64 oracle: the largest supported network shapes, the
deepest network, single chains, empty calls, and the smallest AIES ensemble.

Tolerances are those of test_gpu_parity.py (FP32: logL 2e-5 (1 + |logL|), gradient
2e-4 (1 + |g|); BF16: the emulator term within 2e-2)."""
import numpy as np
import pytest
import torch

import paper_2606_04895_amd as B
from oracle import samplers as OS, target as OT, philox as OP
from workloads import make_problem, small_problem

pytestmark = pytest.mark.gpu


def _pts(prob, n, seed):
    rng = np.random.default_rng(seed)
    sd = np.sqrt(np.diag(prob["gauss_cov"]))
    return prob["gauss_mean"] + rng.normal(size=(n, prob["d"])) * sd


def _check(prob, prec, n, tl, tg):
    ctx = B.best_init(prob, n_chains=16, precision=prec, seed=1)
    x = _pts(prob, n, 3)
    lp, g = B.best_logL_grad(ctx, x.T.copy())
    lo, go = OT.log_target(prob, x)
    assert np.all(np.isfinite(lp)) and np.all(np.isfinite(g))
    assert np.max(np.abs(lp - lo) / (1 + np.abs(lo))) < tl
    if tg is not None:
        assert np.max(np.abs(g.T - go) / (1 + np.abs(go))) < tg
    ctx.close()


@pytest.mark.parametrize("prec,tl,tg", [("bf16", 2e-2, None), ("fp32", 2e-5, 2e-4)])
def test_widest_network_and_largest_d(prec, tl, tg):
    """d = 32 (the largest input), width 2048 (BF16) / 1024 (FP32, whose 2048-wide
    activation buffers exceed the LDS budget)."""
    width = 2048 if prec == "bf16" else 1024
    prob = small_problem(d=32, width=width, n_hidden=2, seed=13)
    _check(prob, prec, 45, tl, tg)


def test_width_beyond_lds_budget_is_rejected():
    prob = small_problem(d=8, width=2048, n_hidden=2, seed=13)
    with pytest.raises(B.BestError) as e:
        B.best_init(prob, n_chains=16, precision="fp32", seed=1)
    assert e.value.code == 1


@pytest.mark.parametrize("prec,tl,tg", [("bf16", 2e-2, None), ("fp32", 2e-5, 2e-4)])
def test_deepest_network(prec, tl, tg):
    prob = small_problem(d=3, width=128, n_hidden=16, seed=17)
    _check(prob, prec, 21, tl, tg)


def test_empty_and_zero_step_calls():
    prob = small_problem(d=4, width=128, n_hidden=2)
    ctx = B.best_init(prob, n_chains=16, precision="fp32", seed=1)
    x0 = B.best_get_state(ctx)[0]
    empty = torch.empty((4, 0), dtype=torch.float64, device="cuda")
    lp, g = B.best_logL_grad(ctx, empty)
    assert lp.numel() == 0
    st = B.best_step(ctx, "mala", 0, eps=0.1)
    assert st["evals"] == 0 and st["accepted"] == 0
    assert np.array_equal(B.best_get_state(ctx)[0], x0)


@pytest.mark.parametrize("sampler,kw", [("mala", dict(eps=0.2)),
                                        ("mala", dict(eps=0.2, adapt_eps=True)),
                                        ("hmc", dict(eps=0.1, n_leapfrog=3)),
                                        ("nuts", dict(eps=0.2, max_depth=4)),
                                        ("aies", {})])
def test_record_thinning_and_capacity(sampler, kw):
    """Slot k of a call's record holds the state after step (k + 1) thin, as float32 of x;
    a record shorter than the call keeps its first slots and the memory past it is not
    touched; recording does not change the chains.  With adapt_eps every step is a launch
    of its own, so the slot index crosses launches; AIES records after both half-moves."""
    prob = small_problem(d=5, width=128, n_hidden=2)
    n, steps, d = 64, 9, prob["d"]

    def run(thin, cap, slots):
        ctx = B.best_init(prob, n_chains=n, precision="fp32", seed=8, init="gaussian",
                          init_point=prob["gauss_mean"], init_scale=0.1)
        B.best_set_whitening(ctx, prob["gauss_mean"], np.linalg.cholesky(prob["closed_cov"]))
        buf = torch.full((slots, d, n), float("nan"), dtype=torch.float32, device="cuda")
        B.best_step(ctx, sampler, steps, thin=thin, record=buf[:cap], **kw)
        x = B.best_get_state(ctx)[0]
        ctx.close()
        return buf.cpu().numpy(), x

    every, x_every = run(1, steps, steps)
    thinned, x_thin = run(3, 2, 4)
    assert np.array_equal(x_every, x_thin)
    assert np.array_equal(every[-1], x_every.astype(np.float32))
    assert np.array_equal(thinned[0], every[2]) and np.array_equal(thinned[1], every[5])
    assert np.all(np.isnan(thinned[2:]))          # past the capacity: untouched
    assert np.mean(np.any(every[-1] != every[0], axis=0)) > 0.2   # the chains moved


def _one_step_oracle(prob, ctx, sampler, kw, seed):
    """Oracle transition from the GPU's current state (same Philox streams)."""
    t = B.best_get_step_counter(ctx)
    x0, lp0, _ = B.best_get_state(ctx)
    x0 = x0.T.copy()
    if sampler == "aies":
        new, info = OS.aies_step(prob, dict(x=x0, lp=OT.log_target(prob, x0)[0]), t, seed,
                                 kw["stretch_a"])
        return x0, new["x"], info
    mu, L = B.best_get_whitening(ctx)
    W = dict(mu=mu, L=L)
    st = OS.init_state(prob, W, x0)
    fn = dict(mh=OS.mh_step, mala=OS.mala_step, hmc=OS.hmc_step)[sampler]
    args = dict(mh=(kw.get("mh_scale"),), mala=(kw.get("eps"),),
                hmc=(kw.get("eps"), kw.get("n_leapfrog")))[sampler]
    new, info = fn(prob, W, st, t, seed, *args)
    return x0, W["mu"][None, :] + new["z"] @ W["L"].T, info


def _lockstep_tiny(prob, n, sampler, kw, seed, steps=5):
    ctx = B.best_init(prob, n_chains=n, precision="fp32", seed=seed, init="gaussian",
                      init_point=prob["gauss_mean"], init_scale=0.05)
    B.best_set_whitening(ctx, prob["gauss_mean"], np.linalg.cholesky(prob["closed_cov"]))
    for _ in range(steps):
        x0, x_or, info = _one_step_oracle(prob, ctx, sampler, kw, seed)
        B.best_step(ctx, sampler, 1, **kw)
        x1 = B.best_get_state(ctx)[0].T
        bad = np.any(x1 != x0, axis=1) != info["accepted"]
        if bad.any():  # only where the decision is within rounding of the threshold
            assert np.all(np.abs(info["log_alpha"] - info["log_u"])[bad] < 1e-6)
        ok = ~bad
        scale = np.abs(x_or[ok]) + np.abs(x_or[ok] - x0[ok]) + 1e-12
        assert np.all(np.abs(x1[ok] - x_or[ok]) / scale < 1e-4)
    ctx.close()


@pytest.mark.parametrize("sampler,kw", [("mh", dict(mh_scale=2.4 / np.sqrt(5))),
                                        ("mala", dict(eps=0.008)),
                                        ("hmc", dict(eps=0.07, n_leapfrog=5))])
def test_single_chain_lockstep(sampler, kw):
    """One chain (a tile with 15 empty slots) follows the oracle step for step."""
    prob = small_problem(d=5, width=128, n_hidden=3, twist=True)
    _lockstep_tiny(prob, 1, sampler, kw, 0xBE58)


def test_de_needs_four_walkers():
    prob = small_problem(d=5, width=128, n_hidden=3)
    ctx = B.best_init(prob, n_chains=2, precision="fp32", seed=3)
    with pytest.raises(B.BestError) as e:
        B.best_step(ctx, "de", 1, de_sigma=0.1)
    assert e.value.code == 5
    ctx.close()


def test_two_walker_aies_lockstep():
    """The smallest AIES ensemble: each walker's only partner is the other one."""
    prob = small_problem(d=5, width=128, n_hidden=3, twist=True)
    _lockstep_tiny(prob, 2, "aies", dict(stretch_a=2.0), 0xBE59)


@pytest.mark.parametrize("sampler,kw,arg", [("mala", dict(eps=0.008), 0.008),
                                            ("mh", dict(mh_scale=0.3), 0.3)])
def test_step_multipliers_lockstep(sampler, kw, arg):
    """Per-dimension steps (MALA eps m_i, MH scale m_i) against the oracle; removing the
    multipliers restores the plain transition."""
    prob = small_problem(d=5, width=128, n_hidden=3, twist=True)
    m = np.array([3.0, 2.0, 1.0, 0.5, 0.25])  # smaller steps on the narrow twisted pair
    seed = 0xBE5A
    ctx = B.best_init(prob, n_chains=70, precision="fp32", seed=seed, init="gaussian",
                      init_point=prob["gauss_mean"], init_scale=0.05)
    B.best_set_whitening(ctx, prob["gauss_mean"], np.linalg.cholesky(prob["closed_cov"]))
    fn = OS.mala_step if sampler == "mala" else OS.mh_step
    for s in range(4):
        use = m if s < 3 else None
        B.best_set_step_multipliers(ctx, use)
        t = B.best_get_step_counter(ctx)
        x0 = B.best_get_state(ctx)[0].T.copy()
        mu, L = B.best_get_whitening(ctx)
        W = dict(mu=mu, L=L)
        new, info = fn(prob, W, OS.init_state(prob, W, x0), t, seed, arg, mult=use)
        x_or = W["mu"][None, :] + new["z"] @ W["L"].T
        B.best_step(ctx, sampler, 1, **kw)
        x1 = B.best_get_state(ctx)[0].T
        bad = np.any(x1 != x0, axis=1) != info["accepted"]
        if bad.any():
            assert np.all(np.abs(info["log_alpha"] - info["log_u"])[bad] < 1e-6)
        ok = ~bad
        scale = np.abs(x_or[ok]) + np.abs(x_or[ok] - x0[ok]) + 1e-12
        assert np.all(np.abs(x1[ok] - x_or[ok]) / scale < 1e-4)
        assert 0 < info["accepted"].mean()
    with pytest.raises(B.BestError) as e:
        B.best_set_step_multipliers(ctx, np.array([1.0, 0.0, 1.0, 1.0, 1.0]))
    assert e.value.code == 1
    ctx.close()


def test_reinit_matches_the_oracle_generators():
    """best_reinit: uniform draws in the box, the replicated point, and point + scale L xi
    with the current whitening factor, xi from the init stream at the step counter."""
    prob = small_problem(d=5, width=128, n_hidden=3, twist=True)
    seed = 0xBE5B
    ctx = B.best_init(prob, n_chains=37, precision="fp32", seed=seed)
    L = np.linalg.cholesky(prob["closed_cov"])
    B.best_set_whitening(ctx, prob["gauss_mean"], L)
    B.best_step(ctx, "mh", 3, mh_scale=0.3)
    t = B.best_get_step_counter(ctx)
    ids = np.arange(37, dtype=np.uint64)
    B.best_reinit(ctx, "gaussian", prob["gauss_mean"], 0.7)
    x, lp, g = B.best_get_state(ctx)
    _, Lc = B.best_get_whitening(ctx)
    ref = prob["gauss_mean"][None, :] + 0.7 * OP.init_normals(seed, ids, 5, step=t) @ Lc.T
    np.testing.assert_allclose(x.T, ref, rtol=1e-12, atol=1e-12)
    lo, go = OT.log_target(prob, x.T)
    assert np.max(np.abs(lp - lo) / (1 + np.abs(lo))) < 2e-5
    B.best_reinit(ctx, "uniform")
    ref = prob["lower"] + (prob["upper"] - prob["lower"]) * OP.init_uniforms(seed, ids, 5, step=t)
    np.testing.assert_allclose(B.best_get_state(ctx)[0].T, ref, rtol=1e-12, atol=1e-12)
    B.best_reinit(ctx, "replicated", prob["gauss_mean"])
    assert np.array_equal(B.best_get_state(ctx)[0].T, np.tile(prob["gauss_mean"], (37, 1)))
    B.best_reinit(ctx, "hypersphere", prob["gauss_mean"], 1.3)
    ref = prob["gauss_mean"][None, :] + 1.3 * OP.init_hypersphere(seed, ids, 5, step=t) @ Lc.T
    np.testing.assert_allclose(B.best_get_state(ctx)[0].T, ref, rtol=1e-12, atol=1e-12)
    with pytest.raises(B.BestError):
        B.best_reinit(ctx, "replicated", prob["upper"] + 1.0)
    ctx.close()


def test_hypersphere_initialisation_at_init_matches_the_oracle():
    """best_init with the hypersphere-based initialisation (Sec. 3.2): init_point +
    init_scale L0 r u with the initial whitening factor L0 = diag(0.1 (upper - lower)), on
    the C5 shape (d = 27, a ragged 1000 walkers)."""
    prob = make_problem("c5")
    seed, n = 0xBE5C, 1000
    pt = prob["gauss_mean"]
    ctx = B.best_init(prob, n_chains=n, precision="bf16", seed=seed, init="hypersphere",
                      init_point=pt, init_scale=2.0)
    L0 = np.diag(0.1 * (prob["upper"] - prob["lower"]))
    ref = pt[None, :] + 2.0 * OP.init_hypersphere(seed, np.arange(n, dtype=np.uint64), 27) @ L0.T
    x = B.best_get_state(ctx)[0].T
    np.testing.assert_allclose(x, ref, rtol=1e-12, atol=1e-12)
    w = (x - pt) / np.diag(L0)
    assert np.all(np.sqrt(np.sum(w * w, axis=1)) <= 2.0 + 1e-12)
    ctx.close()


def test_recentring_burn_in_and_trajectory():
    """Burn-in that re-centres the ensemble on its best-fit walker after every covariance
    window, keeping the trajectory; the Gaussian posterior mean is then recovered."""
    from paper_2606_04895_amd import driver
    from workloads import make_problem
    prob = make_problem("c2", with_mlp=False)
    n, d = 2048, 6
    ctx = B.best_init(prob, n_chains=n, precision="fp32", seed=5, init="uniform")
    traj = []
    driver.burn_in(ctx, "mala", 300, d, n, recenter=True, trajectory=traj)
    assert sum(int(r.shape[0]) for r in traj) == 300
    st, rec, wall, ess = driver.sample(ctx, "mala", 300, d, n)
    m = rec.double().mean(dim=(0, 2)).cpu().numpy()
    sd = np.sqrt(np.diag(prob["closed_cov"]))
    assert np.all(np.abs(m - prob["closed_mean"]) / (sd / np.sqrt(ess)) < 5)
    ctx.close()


@pytest.mark.parametrize("cfg,prec,n,tl,tg", [("c2", "bf16", 40000, 2e-2, None),
                                             ("c2", "fp32", 40000, 2e-5, 2e-4),
                                             ("c5", "bf16", 20000, 2e-2, None)])
def test_large_batch_eval_on_wider_tiles(cfg, prec, n, tl, tg):
    """A batch far larger than the context's chains is evaluated on the widest tile that
    still fills the CUs (C5 BF16: 32-chain tiles with the activations in global scratch);
    sampled points against the oracle; log pi bitwise equal to the context's own tile width
    (BF16 gradients may differ in rounding where the narrow tile keeps the activations in
    LDS in BF16 and the wide one in FP32 global scratch)."""
    from workloads import make_problem
    prob = make_problem(cfg)
    x = _pts(prob, n, 5)
    ctx = B.best_init(prob, n_chains=16, precision=prec, seed=1)
    lp, g = B.best_logL_grad(ctx, x.T.copy())
    ctx.close()
    narrow = B.best_init(prob, n_chains=16, precision=prec, seed=1, chains_per_block=16)
    lp16, g16 = B.best_logL_grad(narrow, x.T.copy())
    narrow.close()
    assert np.array_equal(lp, lp16)
    if prec == "fp32":  # same activation storage at both widths: identical gradients too
        assert np.array_equal(g, g16)
    idx = np.random.default_rng(7).choice(n, 150, replace=False)
    lo, go = OT.log_target(prob, x[idx])
    assert np.max(np.abs(lp[idx] - lo) / (1 + np.abs(lo))) < tl
    if tg is not None:
        assert np.max(np.abs(g[:, idx].T - go) / (1 + np.abs(go))) < tg

"""GPU parity for the smooth boundary penalty of Sec. 3.1 (box_penalty = 1) against the FP64
oracle: log pi and its gradient inside and outside the box, and HMC / NUTS transitions of
chains started at a face of the box so that trajectories cross it (tolerances as in
test_gpu_parity.py and test_gpu_nuts.py)."""
import numpy as np
import pytest

import paper_2606_04895_amd as B
from oracle import nuts as ON, samplers as OS, target as OT
from workloads import small_problem

pytestmark = pytest.mark.gpu


def _prob(d=5):
    prob = small_problem(d=d, width=128, n_hidden=3, seed=19)
    # a box of +-2 sigma so that trajectories reach its faces
    sd = np.sqrt(np.diag(prob["closed_cov"]))
    return dict(prob, lower=prob["gauss_mean"] - 2 * sd, upper=prob["gauss_mean"] + 2 * sd,
                box_penalty=1, penalty_width=0.05)


# d = 5 takes the eight-threads-per-chain form of the FP64 work, d = 12 the loop form
@pytest.mark.parametrize("d", [5, 12])
@pytest.mark.parametrize("prec,tl,tg", [("fp32", 2e-5, 2e-4), ("fp64", 1e-9, 1e-8)])
def test_penalised_logL_grad_inside_and_outside(prec, tl, tg, d):
    prob = _prob(d)
    rng = np.random.default_rng(3)
    width = prob["upper"] - prob["lower"]
    x = prob["lower"] + rng.uniform(-0.15, 1.15, size=(97, d)) * width
    ctx = B.best_init(prob, n_chains=16, precision=prec, seed=1)
    lp, g = B.best_logL_grad(ctx, x.T.copy())
    lo, go = OT.log_target(prob, x)
    out = ~np.all((x >= prob["lower"]) & (x <= prob["upper"]), axis=1)
    assert out.sum() > 20 and np.all(np.isfinite(lp))
    assert np.max(np.abs(lp - lo) / (1 + np.abs(lo))) < tl
    assert np.max(np.abs(g.T - go) / (1 + np.abs(go))) < tg
    ctx.close()


def _start_at_face(prob, n, seed):
    ctx = B.best_init(prob, n_chains=n, precision="fp32", seed=seed, init="gaussian",
                      init_point=prob["upper"] - 0.02 * (prob["upper"] - prob["lower"]),
                      init_scale=0.02)
    B.best_set_whitening(ctx, prob["gauss_mean"], np.linalg.cholesky(prob["closed_cov"]))
    return ctx


@pytest.mark.parametrize("d", [5, 12])
def test_hmc_lockstep_across_the_faces(d):
    prob = _prob(d)
    seed = 0xBE71
    ctx = _start_at_face(prob, 40, seed)
    crossed = 0
    for _ in range(3):
        t = B.best_get_step_counter(ctx)
        x0 = B.best_get_state(ctx)[0].T.copy()
        mu, L = B.best_get_whitening(ctx)
        W = dict(mu=mu, L=L)
        new, info = OS.hmc_step(prob, W, OS.init_state(prob, W, x0), t, seed, 0.2, 6)
        x_or = W["mu"][None, :] + new["z"] @ W["L"].T
        B.best_step(ctx, "hmc", 1, eps=0.2, n_leapfrog=6)
        x1 = B.best_get_state(ctx)[0].T
        bad = np.any(x1 != x0, axis=1) != info["accepted"]
        if bad.any():
            assert np.all(np.abs(info["log_alpha"] - info["log_u"])[bad] < 1e-6)
        ok = ~bad
        scale = np.abs(x_or[ok]) + np.abs(x_or[ok] - x0[ok]) + 1e-12
        assert np.all(np.abs(x1[ok] - x_or[ok]) / scale < 1e-4)
        crossed += int(np.sum(~np.all((x_or >= prob["lower"]) & (x_or <= prob["upper"]), axis=1)
                              & info["accepted"]))
    assert crossed > 0  # accepted end points outside the box: the penalty, not -inf
    ctx.close()


def test_nuts_lockstep_across_the_faces():
    prob = _prob()
    seed = 0xBE72
    ctx = _start_at_face(prob, 37, seed)
    mism = 0
    for _ in range(2):
        t = B.best_get_step_counter(ctx)
        x0 = B.best_get_state(ctx)[0].T.copy()
        mu, L = B.best_get_whitening(ctx)
        W = dict(mu=mu, L=L)
        st = OS.init_state(prob, W, x0)
        new, info = ON.nuts_step(prob, W, st, t, seed, 0.25, max_depth=5)
        x_or = W["mu"][None, :] + new["z"] @ W["L"].T
        out = B.best_step(ctx, "nuts", 1, eps=0.25, max_depth=5)
        x1 = B.best_get_state(ctx)[0].T
        rel = np.max(np.abs(x1 - x_or) / (np.abs(x_or) + np.abs(x_or - x0) + 1e-12), axis=1)
        mism += int((rel >= 1e-4).sum())
        if not (rel >= 1e-4).any():
            assert out["evals"] == int(info["n_leaves"].sum())
    assert mism <= 0.02 * 74
    ctx.close()

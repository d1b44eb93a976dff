"""GPU NUTS (Hoffman & Gelman efficient slice version, whitened space, identity mass)
against the FP64 oracle (oracle/nuts.py) on the same Philox streams.

Lockstep: from the GPU's state, one oracle transition and one GPU transition per step; a
tree's shape follows from many decisions on computed energies and dot products (slice
membership, divergence, U-turns), so a chain may take a different tree where one of them
sits within rounding of its threshold.  The bar: at most 2% of chain-steps differ, the
others end at the oracle's point within 1e-4 relative (FP32 GEMMs, as for HMC), and with no
differing chain the evaluation count equals the oracle's leaf count exactly and the summed
acceptance statistic agrees to 1e-6 relative per chain-step."""
import numpy as np
import pytest
import torch

import paper_2606_04895_amd as B
from oracle import adapt as OA, nuts as ON, samplers as OS
from workloads import make_problem, small_problem

pytestmark = pytest.mark.gpu


def _lockstep_nuts(prob, n, eps, max_depth, steps, seed, init_scale=0.05, cpb=0):
    ctx = B.best_init(prob, n_chains=n, precision="fp32", seed=seed, init="gaussian",
                      init_point=prob["gauss_mean"], init_scale=init_scale, chains_per_block=cpb)
    B.best_set_whitening(ctx, prob["gauss_mean"], np.linalg.cholesky(prob["closed_cov"]))
    mism, total, depths = 0, 0, []
    for _ in range(steps):
        t = B.best_get_step_counter(ctx)
        x0, _, _ = B.best_get_state(ctx)
        x0 = x0.T.copy()
        mu, L = B.best_get_whitening(ctx)
        W = dict(mu=mu, L=L)
        st = OS.init_state(prob, W, x0)
        new, info = ON.nuts_step(prob, W, st, t, seed, eps, max_depth=max_depth)
        x_or = W["mu"][None, :] + new["z"] @ W["L"].T
        out = B.best_step(ctx, "nuts", 1, eps=eps, max_depth=max_depth)
        x1 = B.best_get_state(ctx)[0].T
        scale = np.abs(x_or) + np.abs(x_or - x0) + 1e-12
        rel = np.max(np.abs(x1 - x_or) / scale, axis=1)
        bad = rel >= 1e-4
        mism += int(bad.sum())
        total += n
        depths.append(info["depth"])
        if not bad.any():
            assert out["evals"] == int(info["n_leaves"].sum())
            np.testing.assert_allclose(out["sum_accept_prob"], info["accept_stat"].sum(),
                                       rtol=1e-6 * n)
        moved_or = np.any(new["z"] != st["z"], axis=1)
        assert out["accepted"] == int(moved_or.sum()) or bad.any()
    ctx.close()
    assert mism <= 0.02 * total, (mism, total)
    return np.concatenate(depths)


def test_lockstep_small_twisted_ragged_tiles():
    """37 chains (three tiles of 16, the last ragged), trees of depth 1 to 5."""
    prob = small_problem(d=5, width=128, n_hidden=3, twist=True)
    depths = _lockstep_nuts(prob, 37, 0.07, 5, steps=3, seed=0xBE61)
    assert depths.min() <= 2 and depths.max() >= 4  # several tree shapes were exercised


def test_lockstep_depth_limit_reached():
    """A small step never turns within the depth limit: every tree has 2^D - 1 leaves."""
    prob = small_problem(d=5, width=128, n_hidden=3, twist=True)
    depths = _lockstep_nuts(prob, 20, 0.001, 4, steps=2, seed=0xBE62)
    assert np.all(depths == 4)


def test_lockstep_at_the_largest_depth():
    """The largest supported depth (12): a step too small to turn builds every tree to 4095
    leaves, with a pending sibling at every one of the twelve levels; 8 chains in one
    ragged tile."""
    prob = small_problem(d=3, width=128, n_hidden=2, seed=21)
    depths = _lockstep_nuts(prob, 8, 1e-4, B.BEST_NUTS_MAX_DEPTH, steps=1, seed=0xBE63)
    assert B.BEST_NUTS_MAX_DEPTH == 12 and np.all(depths == 12)


@pytest.mark.parametrize("cpb", [64, 16])
def test_lockstep_27_parameters_wide_tiles(cpb):
    """d = 27 (lane groups of 32 lanes per chain, 5 of them idle) in 64- and 16-chain tiles."""
    prob = small_problem(d=27, width=128, n_hidden=2, seed=11)
    _lockstep_nuts(prob, 70, 0.3, 6, steps=2, seed=0xBE71, cpb=cpb)


def test_lockstep_c2_network():
    prob = make_problem("c2")
    _lockstep_nuts(prob, 300, 0.4, 6, steps=2, seed=0xBE63, init_scale=0.3)


def test_single_chain_and_box_divergence():
    """One chain in a tile of 16, and a start at the edge of the prior box with a large
    step (past the leapfrog stability limit): the first leaf leaves the box (log pi = -inf),
    which stops the trajectory."""
    prob = small_problem(d=5, width=128, n_hidden=3, twist=True)
    _lockstep_nuts(prob, 1, 0.07, 6, steps=3, seed=0xBE64)
    ctx = B.best_init(prob, n_chains=16, precision="fp32", seed=5, init="replicated",
                      init_point=prob["upper"] - 1e-3 * (prob["upper"] - prob["lower"]))
    B.best_set_whitening(ctx, prob["gauss_mean"], np.linalg.cholesky(prob["closed_cov"]))
    st = B.best_step(ctx, "nuts", 3, eps=2.5, max_depth=6)
    x = B.best_get_state(ctx)[0]
    assert np.all(x >= prob["lower"][:, None]) and np.all(x <= prob["upper"][:, None])
    assert st["n_oob"] > 0
    assert st["evals"] < 3 * 16 * 63


def test_gaussian_posterior_recovery_bf16():
    """BF16 GEMMs on the 6-d Gaussian (no emulator term): mean within 5 Monte-Carlo
    standard errors (per-coordinate ESS), whitened covariance within 0.05 + 5 sqrt(2/ESS)."""
    prob = make_problem("c2", with_mlp=False)
    n = 4096
    ctx = B.best_init(prob, n_chains=n, precision="bf16", seed=3, init="gaussian",
                      init_point=prob["gauss_mean"], init_scale=0.5)
    B.best_set_whitening(ctx, prob["gauss_mean"], np.linalg.cholesky(prob["closed_cov"]))
    B.best_step(ctx, "nuts", 50, eps=0.5, max_depth=6)
    steps = 200
    rec = torch.empty((steps, 6, n), dtype=torch.float32, device="cuda")
    st = B.best_step(ctx, "nuts", steps, eps=0.5, max_depth=6, record=rec)
    s = rec.double().cpu().numpy().transpose(0, 2, 1)
    m, c = OA.ensemble_moments(s)
    ess = B.best_ess(ctx, rec)
    sd = np.sqrt(np.diag(prob["closed_cov"]))
    z = np.abs(m - prob["closed_mean"]) / (sd / np.sqrt(ess))
    assert np.all(z < 5), z
    Li = np.linalg.inv(np.linalg.cholesky(prob["closed_cov"]))
    dev = np.linalg.norm(Li @ c @ Li.T - np.eye(6), 2)
    assert dev < 0.05 + 5 * np.sqrt(2.0 / ess.min()), (dev, ess.min())
    # a 6-d standard normal at eps = 0.5: trajectories of a few leapfrog steps each
    per = st["evals"] / (steps * n)
    assert 3 <= per <= 31, per


def test_dual_averaging_reaches_target_statistic():
    """After 200 adaptation steps and finalising to the averaged iterate, the NUTS
    acceptance statistic over 60 steps x 2048 chains is within 0.03 of the target, the bar
    of the MALA / HMC dual-averaging test (measured offsets -0.0025 .. +0.0013 over three
    seeds, Monte-Carlo error of the mean about 0.001)."""
    prob = make_problem("c2")
    n = 2048
    ctx = B.best_init(prob, n_chains=n, precision="bf16", seed=3, init="gaussian",
                      init_point=prob["gauss_mean"], init_scale=0.5)
    B.best_set_whitening(ctx, prob["gauss_mean"], np.linalg.cholesky(prob["closed_cov"]))
    B.best_set_step_size(ctx, 0.05)
    B.best_step(ctx, "nuts", 200, adapt_eps=True, target_accept=0.8, max_depth=6)
    B.best_adapt(ctx, update_mean=False, finalize_da=True)
    st = B.best_step(ctx, "nuts", 60, max_depth=6)
    stat = st["sum_accept_prob"] / (60 * n)
    assert abs(stat - 0.8) < 0.03, (stat, st["eps"])


def test_nuts_arguments_are_validated():
    prob = small_problem(d=4, width=128, n_hidden=2)
    ctx = B.best_init(prob, n_chains=16, precision="fp32", seed=1)
    for depth in (0, B.BEST_NUTS_MAX_DEPTH + 1):
        with pytest.raises(B.BestError) as e:
            B.best_step(ctx, "nuts", 1, eps=0.1, max_depth=depth)
        assert e.value.code == 1
    ctx64 = B.best_init(prob, n_chains=16, precision="fp64", seed=1)
    with pytest.raises(B.BestError) as e:
        B.best_step(ctx64, "nuts", 1, eps=0.1, max_depth=3)
    assert e.value.code == 5

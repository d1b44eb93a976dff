"""Configuration C1 at its configured size on the GPU with the FP64 oracle beside it: 64
chains x 2000 random-walk MH steps (proposal (2.4^2 / 6) S, FP64 GEMMs) from the same exact
draws of N(mu, S) on the same Philox streams.  FP64 makes the two runs the same chains: every
recorded draw agrees to the float32 record's rounding and the final states to 1e-9
relative.  Prints both min-ESS/s (the oracle's on this host's cores)."""
import json
import os
import time

import numpy as np
import pytest

from oracle import ess as OE, samplers as OS
from paper_2606_04895_amd import configs

pytestmark = pytest.mark.gpu


def test_c1_full_configuration_runs_the_oracles_chains():
    prob, n, steps, burn, L, x0, scale = configs.c1_setup()
    print(f"c1: {n} chains x {steps} MH steps, FP64, oracle beside", flush=True)
    r, rec, x_gpu = configs.c1_gpu()
    W = dict(mu=prob["gauss_mean"], L=L)
    st = OS.init_state(prob, W, x0)
    zs = []
    t_prod = 0.0
    for t in range(steps):
        t0 = time.perf_counter()
        st, _ = OS.mh_step(prob, W, st, t, prob["seed"], scale)
        if t >= burn:
            t_prod += time.perf_counter() - t0
            zs.append(st["z"].copy())
    xs = np.stack(zs) @ L.T + prob["gauss_mean"]           # (T, n, d)
    rec_np = rec.double().cpu().numpy().transpose(0, 2, 1)   # (T, n, d)
    x32 = xs.astype(np.float32).astype(np.float64)
    assert np.all(np.abs(rec_np - x32) <= 1e-6 * (1.0 + np.abs(xs)))
    x_or = st["z"] @ L.T + prob["gauss_mean"]
    assert np.max(np.abs(x_gpu - x_or) / (np.abs(x_or) + 1.0)) < 1e-9
    oess = np.array([OE.ess(xs[:, :, i].T) for i in range(prob["d"])])
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        cores = os.cpu_count() or 1
    r["oracle"] = dict(production_s=t_prod, min_ess=float(oess.min()),
                       min_ess_per_s=float(oess.min()) / t_prod, nproc=cores,
                       kind="oracle (numpy FP64)")
    # the same chains: the ESS of the two records agree up to the float32 record
    assert abs(r["min_ess"] - oess.min()) < 1e-3 * oess.min()
    print(json.dumps(r), flush=True)


@pytest.mark.parametrize("prec,tol", [("bf16", 2e-2), ("fp16", 4e-3)])
def test_c3_logpi_error_on_posterior_draws_against_the_oracle(prec, tol):
    """C3 (12 parameters, MLP 12->1024x4->1) at its 16384 chains: HMC adapted for 1000 steps
    and run 200 more; on 2048 of the last draws the 16-bit log pi is compared with the FP64
    oracle.  The distribution is printed; the emulator term's error stays within the
    16-bit tolerance of the parity tests."""
    from oracle import target as OT
    import torch
    print(f"c3 {prec}: 16384 chains, HMC 1000 + 200 steps", flush=True)
    r, rec, ctx, prob = configs.c3_run(prec, True, 16384, 1000, 200, **configs.C3_INIT)
    x = rec[-1].double()                                     # [d][n], the last draws
    idx = torch.randperm(x.shape[1], generator=torch.Generator().manual_seed(1))[:2048]
    xs = x[:, idx.to(x.device)].contiguous()
    import paper_2606_04895_amd as B
    lp, _ = B.best_logL_grad(ctx, xs, want_grad=False)
    lo, _ = OT.log_target(prob, xs.T.cpu().numpy())
    err = np.abs(lp.cpu().numpy() - lo)
    out = dict(config="c3", precision=prec, draws=2048, accept=r["accept"],
               logpi_abs_err_vs_oracle=dict(p50=float(np.percentile(err, 50)),
                                            p99=float(np.percentile(err, 99)),
                                            max=float(err.max())))
    print(json.dumps(out), flush=True)
    assert np.all(np.isfinite(lp.cpu().numpy()))
    assert err.max() < tol, out
    ctx.close()


def _c3_exact_draws(prob, n, seed):
    """Exact draws of the emulator-off C3 target: the Gaussian block from the inverse of its
    precision block, the twisted pair from its latent construction (u ~ N(c, s_u^2),
    v = m_v + s_w xi - beta ((u - c)^2 - kappa))."""
    tw = prob["twist"]
    u, v = tw["u"], tw["v"]
    d = prob["d"]
    rng = np.random.default_rng(seed)
    g = [i for i in range(d) if i not in (u, v)]
    x = np.zeros((n, d))
    cov_g = np.linalg.inv(prob["gauss_prec"][np.ix_(g, g)])
    x[:, g] = prob["gauss_mean"][g] + rng.normal(size=(n, len(g))) @ np.linalg.cholesky(cov_g).T
    su = 1.0 / np.sqrt(prob["gauss_prec"][u, u])
    sw = 1.0 / np.sqrt(prob["gauss_prec"][v, v])
    x[:, u] = tw["center"] + su * rng.normal(size=n)
    x[:, v] = prob["gauss_mean"][v] + sw * rng.normal(size=n) - tw["beta"] * (
        (x[:, u] - tw["center"]) ** 2 - tw["kappa"])
    return x


@pytest.mark.parametrize("prec", ["bf16", "fp32"])
def test_c3_hmc_keeps_the_twisted_targets_closed_form_moments(prec):
    """Emulator-off C3 (the closed form is known): 8192 exact draws in, the closed-form
    whitening, 600 HMC steps (L = 10, eps 0.05) out.  The chains keep the mean (within
    0.05 sd) and the variances (within 10%; the pair's v has the heavy tail of (u - c)^2) of
    every coordinate, the twisted pair included: the transition leaves the non-Gaussian
    target invariant.  (From a central start a fixed step size reaches the pair's tails only
    slowly; that is mixing, not bias.)"""
    import paper_2606_04895_amd as B
    from workloads import make_problem
    prob = make_problem("c3", with_mlp=False)
    n = 8192
    x0 = _c3_exact_draws(prob, n, 11)
    sd = np.sqrt(np.diag(prob["closed_cov"]))
    ctx = B.best_init(prob, n_chains=n, precision=prec, seed=6)
    B.best_set_whitening(ctx, prob["gauss_mean"], np.linalg.cholesky(prob["closed_cov"]))
    B.best_set_state(ctx, x0.T.copy())
    st = B.best_step(ctx, "hmc", 600, eps=0.05, n_leapfrog=10)
    x = B.best_get_state(ctx)[0].T
    acc = st["accepted"] / (600 * n)
    merr = np.abs(x.mean(0) - prob["closed_mean"]) / sd
    vr = x.var(0) / sd ** 2
    print(json.dumps(dict(config="c3 emulator off", precision=prec, accept=acc,
                          max_mean_err_sd=float(merr.max()),
                          var_ratio=[round(float(a), 3) for a in vr])), flush=True)
    assert 0.5 < acc < 0.99
    assert np.all(merr < 0.05) and np.all(np.abs(vr - 1.0) < 0.1), (merr, vr)
    ctx.close()

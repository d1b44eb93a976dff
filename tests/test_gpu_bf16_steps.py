"""One fused BF16 (and FP16) MALA / HMC transition against the FP64 oracle on the same Philox
streams, at the C2 workload's shape (4096 chains, 6 -> 512 x 4 -> 1).

Two comparisons per transition:
  1. Replay: the transition is recomputed on the host in FP64 (the oracle's sampler
     arithmetic: proposal, leapfrog, energies, log alpha) with every log pi and gradient
     taken from the library's own 16-bit evaluation (best_logL_grad).  This isolates the
     fused kernel's sampler arithmetic from the emulator's rounding: accept decisions must
     agree except within 1e-6 of the threshold, and states within 1e-6 relative.
  2. Oracle: the same transition in the FP64 oracle (FP64 emulator).  The 16-bit emulator
     moves log alpha by at most the measured max |log alpha(replay) - log alpha(oracle)|
     over the chains; decisions may differ only where |log alpha - log u| is below twice
     that, and the accepted states differ by the replay-vs-oracle state difference (the
     proposal moves with the 16-bit gradient), at most twice its measured maximum plus
     1e-9.
"""
import numpy as np
import pytest
import torch

import paper_2606_04895_amd as B
from oracle import philox as OP, samplers as OS
from workloads import make_problem

pytestmark = pytest.mark.gpu

SEED = 0x5EED16


def _setup(prec, n=4096):
    prob = make_problem("c2")
    ctx = B.best_init(prob, n_chains=n, precision=prec, seed=SEED)
    L = np.linalg.cholesky(prob["closed_cov"])
    B.best_set_whitening(ctx, prob["gauss_mean"], L)
    # chains in the typical set: draws of the Gaussian part (the emulator term moves the
    # posterior by O(1) in whitened units), log pi re-evaluated by the library
    xi = np.random.default_rng(SEED).normal(size=(n, prob["d"]))
    B.best_set_state(ctx, (prob["gauss_mean"] + xi @ L.T).T.copy())
    return prob, ctx


def _eval(ctx, x):
    """log pi and grad_x at x (n, d) from the library's own evaluation."""
    xt = torch.tensor(np.ascontiguousarray(x.T), device="cuda")
    lp, g = B.best_logL_grad(ctx, xt)
    return lp.cpu().numpy(), g.cpu().numpy().T


def _replay_mala(ctx, W, x0, lp0, g0, t, eps):
    mu, L = W["mu"], W["L"]
    n, d = x0.shape
    ld = np.sum(np.log(np.diag(L)))
    z = np.linalg.solve(L, (x0 - mu).T).T
    gz = g0 @ L
    xi = OP.normals(SEED, np.arange(n, dtype=np.uint64), t, OP.STREAM_NORMAL, 0, d)
    zp = z + eps * gz + np.sqrt(2 * eps) * xi
    xp = mu + zp @ L.T
    lpp, gpx = _eval(ctx, xp)
    gzp = gpx @ L
    with np.errstate(invalid="ignore"):
        fwd = np.sum((zp - z - eps * gz) ** 2, 1) / (4 * eps)
        rev = np.sum((z - zp - eps * gzp) ** 2, 1) / (4 * eps)
        la = (lpp + ld) - (lp0 + ld) - rev + fwd
    lu = np.log(OP.accept_uniform(SEED, np.arange(n, dtype=np.uint64), t))
    acc = lu < la
    return np.where(acc[:, None], xp, x0), acc, la, lu


def _replay_hmc(ctx, prob, W, x0, lp0, g0, t, eps, n_leap):
    mu, L = W["mu"], W["L"]
    n, d = x0.shape
    z = np.linalg.solve(L, (x0 - mu).T).T
    gz = g0 @ L
    q = OP.normals(SEED, np.arange(n, dtype=np.uint64), t, OP.STREAM_NORMAL, 0, d)
    h0 = -lp0 + 0.5 * np.sum(q * q, 1)
    lp = None
    for _ in range(n_leap):
        q = q + 0.5 * eps * gz
        z = z + eps * q
        lp, gx = _eval(ctx, mu + z @ L.T)
        gz = gx @ L
        q = q + 0.5 * eps * gz
    x1 = mu + z @ L.T
    with np.errstate(invalid="ignore"):
        la = h0 - (-lp + 0.5 * np.sum(q * q, 1))
    lu = np.log(OP.accept_uniform(SEED, np.arange(n, dtype=np.uint64), t))
    acc = lu < la
    return np.where(acc[:, None], x1, x0), acc, la, lu


def _rel(a, b, x0):
    return np.abs(a - b) / (np.abs(b) + np.abs(b - x0) + 1e-12)


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
@pytest.mark.parametrize("sampler", ["mala", "hmc"])
def test_half_precision_step_against_replay_and_oracle(prec, sampler):
    prob, ctx = _setup(prec)
    eps, n_leap = (0.6, 1) if sampler == "mala" else (0.2, 10)
    mu, L = B.best_get_whitening(ctx)
    W = dict(mu=mu, L=L)
    for _ in range(2):
        t = B.best_get_step_counter(ctx)
        x0, lp0, g0 = B.best_get_state(ctx)
        x0, g0 = x0.T.copy(), g0.T.copy()
        if sampler == "mala":
            x_rp, acc_rp, la_rp, lu = _replay_mala(ctx, W, x0, lp0, g0, t, eps)
            new, info = OS.mala_step(prob, W, OS.init_state(prob, W, x0), t, SEED, eps)
            B.best_step(ctx, "mala", 1, eps=eps)
        else:
            x_rp, acc_rp, la_rp, lu = _replay_hmc(ctx, prob, W, x0, lp0, g0, t, eps, n_leap)
            new, info = OS.hmc_step(prob, W, OS.init_state(prob, W, x0), t, SEED, eps, n_leap)
            B.best_step(ctx, "hmc", 1, eps=eps, n_leapfrog=n_leap)
        x1 = B.best_get_state(ctx)[0].T
        acc_gpu = np.any(x1 != x0, axis=1)
        # 1. the fused kernel against the replay on the library's own evaluations
        bad = acc_gpu != acc_rp
        assert np.all(np.abs(la_rp - lu)[bad] < 1e-6), np.abs(la_rp - lu)[bad]
        assert _rel(x1[~bad], x_rp[~bad], x0[~bad]).max() < 1e-6
        # 2. against the FP64 oracle, with the band the 16-bit emulator itself opens
        x_or = W["mu"][None, :] + new["z"] @ W["L"].T
        fin = np.isfinite(la_rp) & np.isfinite(info["log_alpha"])
        dla = np.max(np.abs(la_rp - info["log_alpha"])[fin])
        assert dla < (0.05 if prec == "bf16" else 0.01), dla
        bad_or = acc_gpu != info["accepted"]
        assert np.all(np.abs(info["log_alpha"] - info["log_u"])[bad_or] < 2 * dla + 1e-9)
        both = acc_gpu & info["accepted"]
        dx_rp = np.abs(x_rp - x_or)[both]
        dx = np.abs(x1 - x_or)[both]
        assert np.all(dx <= 2 * dx_rp + 1e-9 * (1 + np.abs(x_or[both])))
        assert bad_or.mean() < 0.01
        assert 0.3 < info["accepted"].mean() <= 1.0
    ctx.close()


@pytest.mark.parametrize("d", [12, 17, 27, 32])
@pytest.mark.parametrize("sampler", ["mala", "hmc"])
def test_wide_lane_groups_against_replay(d, sampler):
    """BF16 on 32-chain tiles with 8 < d <= 32 runs the wide lane-group form of the FP64
    work (sixteen threads per chain, components i and i + 16 in thread i).  The fused
    transition is checked against the host replay on the library's own evaluations, as in
    comparison 1 above; 262 chains leave a ragged last tile.  d = 17 leaves one second
    component (thread 0's), d = 32 fills every slot of both halves."""
    from workloads import small_problem
    _wide_replay(small_problem(d=d, width=128, n_hidden=3), sampler)


@pytest.mark.parametrize("sampler", ["mala", "hmc"])
def test_wide_lane_groups_on_the_27_parameter_network(sampler):
    """The same check on the 27-parameter workload's network (27 -> 1024 x 5 -> 1) at
    32-chain tiles: its two 64 KiB activation buffers leave LDS room for the launch
    constants only, so the tile scratch of the wide form lives in global memory."""
    _wide_replay(make_problem("c5"), sampler)


def _wide_replay(prob, sampler):
    d = prob["d"]
    n = 262
    ctx = B.best_init(prob, n_chains=n, precision="bf16", seed=SEED, chains_per_block=32)
    L = np.linalg.cholesky(prob["closed_cov"])
    B.best_set_whitening(ctx, prob["gauss_mean"], L)
    xi = np.random.default_rng(SEED + d).normal(size=(n, d))
    B.best_set_state(ctx, (prob["gauss_mean"] + 0.5 * xi @ L.T).T.copy())
    eps, n_leap = (0.15, 1) if sampler == "mala" else (0.1, 5)
    mu, Lw = B.best_get_whitening(ctx)
    W = dict(mu=mu, L=Lw)
    accepted = 0
    for _ in range(2):
        t = B.best_get_step_counter(ctx)
        x0, lp0, g0 = B.best_get_state(ctx)
        x0, g0 = x0.T.copy(), g0.T.copy()
        if sampler == "mala":
            x_rp, acc_rp, la_rp, lu = _replay_mala(ctx, W, x0, lp0, g0, t, eps)
            B.best_step(ctx, "mala", 1, eps=eps)
        else:
            x_rp, acc_rp, la_rp, lu = _replay_hmc(ctx, prob, W, x0, lp0, g0, t, eps, n_leap)
            B.best_step(ctx, "hmc", 1, eps=eps, n_leapfrog=n_leap)
        x1 = B.best_get_state(ctx)[0].T
        acc_gpu = np.any(x1 != x0, axis=1)
        bad = acc_gpu != acc_rp
        assert np.all(np.abs(la_rp - lu)[bad] < 1e-6), np.abs(la_rp - lu)[bad]
        assert _rel(x1[~bad], x_rp[~bad], x0[~bad]).max() < 1e-6
        accepted += int(acc_gpu.sum())
    assert accepted > 0.1 * 2 * n, accepted
    # three steps in one launch end bitwise where three one-step launches end (the tile
    # scratch carries nothing from one step to the next)
    x_mid, lp_mid, g_mid = B.best_get_state(ctx)
    t_mid = B.best_get_step_counter(ctx)
    kw = dict(eps=eps) if sampler == "mala" else dict(eps=eps, n_leapfrog=n_leap)
    ends = []
    for split in ((3,), (1, 1, 1)):
        B.best_set_state(ctx, x_mid, lp_mid, g_mid)
        B.best_set_step_counter(ctx, t_mid)
        for k in split:
            B.best_step(ctx, sampler, k, **kw)
        ends.append(B.best_get_state(ctx))
    for a, b in zip(*ends):
        assert np.array_equal(a, b)
    ctx.close()

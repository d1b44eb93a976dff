"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the same seeded
inputs and the same Philox streams.

Tolerances (from the rounding of each GEMM type; the FP64 accept arithmetic is common):
  FP64 GEMMs  logL abs 1e-9 * (1 + |logL|), grad rel 1e-8
  FP32 GEMMs  logL abs 2e-5 * (1 + |logL|), grad abs 2e-4 * (1 + |g|)
  FP16 / BF16 the emulator term (coef * MLP) within 2e-2 (bf16) / 4e-3 (fp16) absolute;
              its gradient within one unit roundoff of the type times (1 + |emulator-term
              gradient|): 2^-8 = 3.9e-3 (bf16), 2^-11 = 4.9e-4 (fp16).  Rounding weights,
              activations and deltas to the type in an FP64 simulation of the network gives
              at most 8.6e-4 (bf16) and 1.0e-4 (fp16) on these workloads.
  lockstep    accept decisions equal except where |log alpha - log u| < band
              (1e-6 for FP32, 1e-9 for FP64); accepted states within 1e-4 relative (FP32)
"""
import numpy as np
import pytest
import torch

import paper_2606_04895_amd as B
from oracle import samplers as OS, target as OT, philox as OP
from workloads import make_problem, small_problem

pytestmark = pytest.mark.gpu

TOL = {"fp64": (1e-9, 1e-8), "fp32": (2e-5, 2e-4), "fp16": (4e-3, 2.0 ** -11),
       "bf16": (2e-2, 2.0 ** -8)}
HALF = ("fp16", "bf16")


def _grad_err(prob, prec, x, g_gpu, go):
    """Gradient error on the scale the tolerance is stated for: (1 + |g|) for FP32/FP64,
    (1 + |gradient of the emulator term|) for the 16-bit types, whose error comes from the
    emulator alone."""
    if prec in HALF:
        _, mg = OT.mlp_part(prob, x)
        return np.abs(g_gpu - go) / (1.0 + np.abs(mg))
    return np.abs(g_gpu - go) / (1.0 + np.abs(go))


def _points(prob, n, seed, spread=2.0):
    rng = np.random.default_rng(seed)
    sd = np.sqrt(np.diag(prob["closed_cov"])) if prob.get("closed_cov") is not None else \
        0.25 * (prob["upper"] - prob["lower"])
    x = prob["gauss_mean"] + rng.normal(size=(n, prob["d"])) * sd * spread \
        if prob.get("closed_cov") is not None else \
        prob["lower"] + rng.uniform(size=(n, prob["d"])) * (prob["upper"] - prob["lower"])
    return x


def _check_eval(prob, prec, n, seed=0, ctx=None):
    ctx = ctx or B.best_init(prob, n_chains=16, precision=prec, seed=1)
    x = _points(prob, n, seed)
    lp, g = B.best_logL_grad(ctx, x.T.copy())
    lo, go = OT.log_target(prob, x)
    tl, tg = TOL[prec]
    scale = 1.0 + np.abs(lo)
    err_l = np.abs(lp - lo) / scale
    assert np.all(np.isfinite(lp)) and np.all(np.isfinite(g))
    assert err_l.max() < tl, (prec, err_l.max())
    err_g = _grad_err(prob, prec, x, g.T, go)
    assert err_g.max() < tg, (prec, err_g.max())
    return err_l.max()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16", "fp16"])
@pytest.mark.parametrize("n", [1, 37, 333])
def test_logL_grad_small_problem(prec, n):
    prob = small_problem(d=5, width=128, n_hidden=3, twist=True)
    _check_eval(prob, prec, n)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_logL_grad_single_hidden_layer(prec):
    prob = small_problem(d=3, width=128, n_hidden=1)
    _check_eval(prob, prec, 50)


@pytest.mark.parametrize("name,prec", [("c1", "fp64"), ("c2", "fp32"), ("c2", "bf16"),
                                       ("c3", "bf16"), ("c5", "bf16"), ("c5", "fp32")])
def test_logL_grad_config_shapes(name, prec):
    prob = make_problem(name)
    _check_eval(prob, prec, 203, seed=3)


def test_logL_grad_full_c2_batch_sampled():
    """C2 at its full 4096 chains in the launch configuration of the benchmark; the oracle
    checks a sample of 256 chains one by one."""
    prob = make_problem("c2")
    for prec in ("fp32", "bf16"):
        ctx = B.best_init(prob, n_chains=4096, precision=prec, seed=2)
        x = _points(prob, 4096, 11)
        xt = torch.tensor(x.T.copy(), device="cuda")
        lp, g = B.best_logL_grad(ctx, xt)
        idx = np.random.default_rng(0).choice(4096, 256, replace=False)
        lo, go = OT.log_target(prob, x[idx])
        tl, tg = TOL[prec]
        assert np.max(np.abs(lp.cpu().numpy()[idx] - lo) / (1 + np.abs(lo))) < tl
        err_g = _grad_err(prob, prec, x[idx], g.cpu().numpy()[:, idx].T, go)
        assert err_g.max() < tg, (prec, err_g.max())


def test_box_and_nonfinite_handling():
    prob = small_problem(d=4, width=128, n_hidden=2)
    ctx = B.best_init(prob, n_chains=16, precision="fp32", seed=1)
    x = np.stack([prob["gauss_mean"], prob["upper"] + 1.0, prob["lower"]]).T.copy()
    lp, g = B.best_logL_grad(ctx, x)
    assert np.isfinite(lp[0]) and lp[1] == -np.inf and np.isfinite(lp[2])
    assert np.all(np.isfinite(g))


def test_emulator_fallback_and_plain_model():
    prob = make_problem("c4")
    for mode in (1, 2):
        p = dict(prob, plain_mode=mode)
        ctx = B.best_init(p, n_chains=16, precision="fp32", seed=1)
        rng = np.random.default_rng(5)
        inside = p["train_lo"] + rng.uniform(size=(20, 6)) * (p["train_hi"] - p["train_lo"])
        outside = p["lower"] + rng.uniform(size=(20, 6)) * (p["upper"] - p["lower"])
        x = np.concatenate([inside, outside])
        lp, g = B.best_logL_grad(ctx, x.T.copy())
        lo, go = OT.log_target(p, x)
        np.testing.assert_allclose(lp, lo, rtol=1e-9, atol=2e-5)
        np.testing.assert_allclose(g.T, go, rtol=1e-7, atol=2e-4 * (1 + np.abs(go).max()))


# ---------------------------------------------------------------------------------------
# Lockstep single-step parity
# ---------------------------------------------------------------------------------------
def _oracle_from_gpu(prob, ctx):
    x, lp, g = B.best_get_state(ctx)
    mu, L = B.best_get_whitening(ctx)
    W = dict(mu=mu, L=L)
    st = OS.init_state(prob, W, x.T)
    return x.T, W, st


def _lockstep(prob, prec, sampler, n, steps=3, band=1e-6, state_tol=1e-4, **kw):
    ctx = B.best_init(prob, n_chains=n, precision=prec, seed=0xBE57, init="gaussian",
                      init_point=prob["gauss_mean"], init_scale=0.05)
    mu = prob["gauss_mean"]
    L = np.linalg.cholesky(prob["closed_cov"])
    B.best_set_whitening(ctx, mu, L)
    seed = 0xBE57
    mism = 0
    for s in range(steps):
        t = B.best_get_step_counter(ctx)
        x0, W, st = _oracle_from_gpu(prob, ctx)
        if sampler == "aies":
            lp0, _ = OT.log_target(prob, x0)
            new, info = OS.aies_step(prob, dict(x=x0, lp=lp0), t, seed, kw["stretch_a"])
            x_or = new["x"]
        elif sampler == "de":
            lp0, _ = OT.log_target(prob, x0)
            new, info = OS.de_step(prob, dict(x=x0, lp=lp0), t, seed, kw["de_sigma"])
            x_or = new["x"]
        else:
            fn = dict(mh=OS.mh_step, mala=OS.mala_step, hmc=OS.hmc_step)[sampler]
            args = dict(mh=(kw.get("mh_scale"),), mala=(kw.get("eps"),),
                        hmc=(kw.get("eps"), kw.get("n_leapfrog")))[sampler]
            new, info = fn(prob, W, st, t, seed, *args)
            x_or = W["mu"][None, :] + new["z"] @ W["L"].T
        B.best_step(ctx, sampler, 1, **kw)
        x1, _, _ = B.best_get_state(ctx)
        x1 = x1.T
        acc_gpu = np.any(x1 != x0, axis=1)
        acc_or = info["accepted"]
        bad = acc_gpu != acc_or
        if bad.any():
            gap = np.abs(info["log_alpha"] - info["log_u"])[bad]
            assert np.all(gap < band), (sampler, prec, gap)
            mism += int(bad.sum())
        ok = ~bad
        scale = np.abs(x_or[ok]) + np.abs(x_or[ok] - x0[ok]) + 1e-12
        rel = np.abs(x1[ok] - x_or[ok]) / scale
        assert rel.max() < state_tol, (sampler, prec, rel.max())
        assert 0 < acc_or.mean() <= 1.0
    return mism


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("sampler,kw", [
    ("mh", dict(mh_scale=2.4 / np.sqrt(5))),
    ("mala", dict(eps=0.008)),
    ("hmc", dict(eps=0.07, n_leapfrog=5)),
    ("aies", dict(stretch_a=2.0)),
    ("de", dict(de_sigma=0.2)),
])
def test_lockstep_small(prec, sampler, kw):
    if prec == "fp64" and sampler in ("mala", "hmc"):
        pytest.skip("FP64 gradient samplers are switched off in the library: an earlier build "
                    "of this path faulted on the GPU and the cause is not yet shown")
    prob = small_problem(d=5, width=128, n_hidden=3, twist=True)
    band, tol = (1e-9, 1e-10) if prec == "fp64" else (1e-6, 1e-4)
    _lockstep(prob, prec, sampler, 262, steps=3, band=band, state_tol=tol, **kw)


@pytest.mark.parametrize("d", [8, 9, 12])
@pytest.mark.parametrize("prec,sampler,kw", [
    ("fp32", "mala", dict(eps=0.008)),
    ("fp32", "hmc", dict(eps=0.07, n_leapfrog=5)),
    ("fp64", "mh", dict(mh_scale=0.5)),
])
def test_lockstep_both_forms_of_the_fp64_work(d, prec, sampler, kw):
    """The FP64 work around the emulator has two forms: eight threads per chain for
    d <= 8, (component, chain) loops above.  d = 8 is the largest for the first, 9 and 12
    take the second; twisted pair and a ragged last tile (262 chains) in each."""
    prob = small_problem(d=d, width=128, n_hidden=3, twist=True)
    band, tol = (1e-9, 1e-10) if prec == "fp64" else (1e-6, 1e-4)
    _lockstep(prob, prec, sampler, 262, steps=3, band=band, state_tol=tol, **kw)


@pytest.mark.parametrize("sampler,kw", [("mala", dict(eps=0.5)),
                                        ("hmc", dict(eps=0.3, n_leapfrog=10))])
def test_lockstep_c2_fp32(sampler, kw):
    prob = make_problem("c2")
    _lockstep(prob, "fp32", sampler, 1000, steps=2, **kw)


def test_lockstep_c1_fp64_mh():
    prob = make_problem("c1")
    _lockstep(prob, "fp64", "mh", 64, steps=5, band=1e-9, state_tol=1e-10,
              mh_scale=2.4 / np.sqrt(6))


# ---------------------------------------------------------------------------------------
# Determinism and error paths
# ---------------------------------------------------------------------------------------
def test_bitwise_determinism_across_runs_and_tile_widths():
    prob = small_problem(d=5, width=128, n_hidden=3)
    outs = []
    for cpb in (16, 32, 16, 64):
        ctx = B.best_init(prob, n_chains=200, precision="fp32", seed=9, chains_per_block=cpb)
        B.best_step(ctx, "mala", 7, eps=0.3)
        outs.append(B.best_get_state(ctx)[0])
    assert np.array_equal(outs[0], outs[2])
    assert np.array_equal(outs[0], outs[1])
    assert np.array_equal(outs[0], outs[3])
    # the 16-bit HMC kernel at 16- and 64-chain tiles (activations in LDS at both widths)
    hm = []
    for cpb in (16, 64):
        ctx = B.best_init(prob, n_chains=200, precision="bf16", seed=9, chains_per_block=cpb)
        B.best_step(ctx, "hmc", 4, eps=0.1, n_leapfrog=5)
        hm.append(B.best_get_state(ctx)[0])
    assert np.array_equal(hm[0], hm[1])


def test_resume_from_checkpoint_is_bitwise():
    prob = small_problem(d=5, width=128, n_hidden=2)
    a = B.best_init(prob, n_chains=64, precision="fp32", seed=4)
    B.best_step(a, "hmc", 6, eps=0.2, n_leapfrog=4)
    xa = B.best_get_state(a)[0]
    b = B.best_init(prob, n_chains=64, precision="fp32", seed=4)
    B.best_step(b, "hmc", 3, eps=0.2, n_leapfrog=4)
    x_mid, lp_mid, g_mid = B.best_get_state(b)
    c = B.best_init(prob, n_chains=64, precision="fp32", seed=4)
    B.best_set_state(c, x_mid, lp_mid, g_mid)
    B.best_set_step_counter(c, 3)
    B.best_step(c, "hmc", 3, eps=0.2, n_leapfrog=4)
    assert np.array_equal(B.best_get_state(c)[0], xa)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("d", [5, 12])
@pytest.mark.parametrize("sampler,kw", [
    ("mh", dict(mh_scale=0.8)), ("mala", dict(eps=0.2)), ("hmc", dict(eps=0.1, n_leapfrog=4)),
    ("nuts", dict(eps=0.2, max_depth=5)), ("aies", {}), ("de", {})])
def test_launch_split_is_bitwise(prec, d, sampler, kw):
    """Four transitions as one launch, as 1 + 3 and as 2 + 1 + 1 end in the same state, bit
    for bit: each step's randomness is keyed by its counter and nothing but the chain state
    passes from one step to the next (d = 5: lane groups of eight; d = 12: the loop form)."""
    prob = small_problem(d=d, width=128, n_hidden=2)
    ends, counters = [], []
    for split in ((4,), (1, 3), (2, 1, 1)):
        ctx = B.best_init(prob, n_chains=96, precision=prec, seed=6, init="gaussian",
                          init_point=prob["gauss_mean"], init_scale=0.1)
        B.best_set_whitening(ctx, prob["gauss_mean"], np.linalg.cholesky(prob["closed_cov"]))
        x_init = B.best_get_state(ctx)[0]
        for k in split:
            B.best_step(ctx, sampler, k, **kw)
        ends.append(B.best_get_state(ctx))
        counters.append(B.best_get_step_counter(ctx))
        ctx.close()
    assert counters[0] == counters[1] == counters[2]
    assert np.mean(np.any(ends[0][0] != x_init, axis=0)) > 0.2   # the chains moved
    for e in ends[1:]:
        for a, b in zip(ends[0], e):
            assert np.array_equal(a, b)


def test_fp64_gradient_samplers_are_refused():
    prob = small_problem(d=4, width=128, n_hidden=2)
    ctx = B.best_init(prob, n_chains=32, precision="fp64", seed=1)
    for s in ("mala", "hmc"):
        with pytest.raises(B.BestError) as e:
            B.best_step(ctx, s, 1, eps=0.1, n_leapfrog=2)
        assert e.value.code == 5


def test_error_codes():
    prob = small_problem(d=4, width=128, n_hidden=2)
    ctx = B.best_init(prob, n_chains=33, precision="fp32", seed=1)
    with pytest.raises(B.BestError) as e:
        B.best_step(ctx, "aies", 1, stretch_a=2.0)
    assert e.value.code == 5
    with pytest.raises(B.BestError) as e:
        B.best_step(ctx, "hmc", 1, eps=0.1, n_leapfrog=0)
    assert e.value.code == 1
    with pytest.raises(B.BestError) as e:
        B.best_step(ctx, "mh", 1, mh_scale=-1)
    assert e.value.code == 1
    bad_L = np.eye(4)
    bad_L[0, 1] = 1.0
    with pytest.raises(B.BestError):
        B.best_set_whitening(ctx, np.zeros(4), bad_L)


def test_nonfinite_weights_are_rejected_and_counted():
    prob = small_problem(d=4, width=128, n_hidden=2)
    p = prob["mlp_params"].copy()
    p[3] = np.nan
    ctx = B.best_init(prob, n_chains=32, precision="fp32", seed=1)
    with pytest.raises(B.BestError):
        B.best_set_mlp(ctx, p, 0.5)


def test_logL_grad_point_major_layout():
    """BEST_AOS: [n][d] points and gradients, device and host pointers, equal to the
    structure-of-arrays call element for element (a ragged 333 points on C2)."""
    prob = make_problem("c2")
    ctx = B.best_init(prob, n_chains=64, precision="fp32", seed=2)
    x = _points(prob, 333, 21)
    lp0, g0 = B.best_logL_grad(ctx, torch.tensor(x.T.copy(), device="cuda"))
    lp1, g1 = B.best_logL_grad(ctx, torch.tensor(x, device="cuda"), aos=True)
    assert torch.equal(lp0, lp1) and torch.equal(g0.T, g1)
    lp2, g2 = B.best_logL_grad(ctx, x, aos=True)
    assert np.array_equal(lp2, lp0.cpu().numpy()) and np.array_equal(g2, g1.cpu().numpy())
    lp3, _ = B.best_logL_grad(ctx, torch.tensor(x, device="cuda"), want_grad=False, aos=True)
    torch.testing.assert_close(lp3, lp0, rtol=1e-12, atol=1e-12)

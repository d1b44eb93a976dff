"""The learned part end to end on the GPU: plain-model pairs -> trained emulator ->
MALA on the emulator (plain fallback outside the training box) -> importance weights by
the plain likelihood, and what the emulator gains over sampling the plain model."""
import numpy as np
import pytest
import torch

import paper_2606_04895_amd as B
from paper_2606_04895_amd import driver
from oracle import target as OT
from workloads import make_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def trained():
    prob = make_problem("c4")
    return prob, driver.train_emulator(prob, n_train=32768, epochs=40, batch=512,
                                       precision="fp32", seed=5, lr0=2e-3, lr1=1e-5)


def test_training_loss_falls(trained):
    _, tr = trained
    # measured: the last epoch's loss is 1.2e-4 of the first
    assert tr["losses"][-1] < 2e-3 * tr["losses"][0], tr["losses"][::5]


def test_emulator_matches_plain_model_near_the_mode(trained):
    prob, tr = trained
    emu = driver.emulator_problem(prob, tr)
    ctx = B.best_init(emu, n_chains=16, precision="fp32", seed=1)
    rng = np.random.default_rng(3)
    ts = prob["plain"]["theta_star"]
    x = ts + rng.normal(size=(200, 6)) * 0.002 / prob["plain"]["invscale"]
    lp, _ = B.best_logL_grad(ctx, x.T.copy())
    lo, _ = OT.plain_logL(prob["plain"], x)
    err = lp - lo
    # a constant offset cancels in sampling; the spread is what matters.  With this test's
    # training budget (32768 pairs, 40 epochs) the emulator captures most of the variation:
    # measured, the error's spread is 0.14 of the plain log-likelihood's (1.8 against 13.1)
    assert np.std(err) < 0.2 * np.std(lo), (np.std(err), np.std(lo))


def test_sampling_the_emulator_with_importance_weights_and_gain(trained):
    prob, tr = trained
    emu = driver.emulator_problem(prob, tr)
    plain = dict(prob, plain_mode=2)
    n, warm, steps = 1024, 300, 200
    res = {}
    for name, p, prec in (("emulator", emu, "bf16"), ("plain", plain, "fp32")):
        ts = prob["plain"]["theta_star"]
        ctx = B.best_init(p, n_chains=n, precision=prec, seed=9, init="gaussian",
                          init_point=ts, init_scale=0.02)
        driver.burn_in(ctx, "mala", warm, 6, n)
        st, rec, wall, ess = driver.sample(ctx, "mala", steps, 6, n)
        res[name] = dict(evals_per_s=st["evals"] / wall, min_ess_per_s=ess.min() / wall,
                         rec=rec, accept=st["accepted"] / (n * steps))
    # importance weights of the emulator's samples under the plain likelihood
    rec = res["emulator"]["rec"][steps // 2:]
    xs = rec.permute(1, 0, 2).reshape(6, -1).double().contiguous()
    ctx_p = B.best_init(plain, n_chains=16, precision="fp32", seed=1)
    ctx_e = B.best_init(emu, n_chains=16, precision="bf16", seed=1)
    lp, _ = B.best_logL_grad(ctx_p, xs, want_grad=False)
    le, _ = B.best_logL_grad(ctx_e, xs, want_grad=False)
    w, kish = B.best_importance_weights(lp, le)
    frac = kish / xs.shape[1]
    # measured: Kish fraction 0.46; acceptance 0.57 for both (the dual-averaging target);
    # the emulator 19x the plain model's evals/s and min-ESS/s at about the same min-ESS
    assert frac > 0.25, frac
    assert abs(res["emulator"]["accept"] - 0.57) < 0.1 and abs(res["plain"]["accept"] - 0.57) < 0.1
    assert res["emulator"]["evals_per_s"] > 5 * res["plain"]["evals_per_s"], res
    assert res["emulator"]["min_ess_per_s"] > 5 * res["plain"]["min_ess_per_s"], res

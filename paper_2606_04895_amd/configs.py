"""The smaller and the learned configurations at their configured sizes, one JSON object per
line (the benchmark line itself, C2, is bench.py; the C5 sampler comparison is compare.py):

* c1: 6 parameters, Gaussian (cond 1e3) + 0.5 MLP(6->128->128->1), random-walk MH with the
  proposal (2.4^2 / 6) S (whitened by L = chol S, scale 2.4 / sqrt 6), 64 chains x 2000
  steps started from exact draws of N(mu, S), the first 500 discarded, FP64 GEMMs.  (The
  FP64 oracle's run of the same chains beside it is tests/test_gpu_configs.py.)
* c3: 12 parameters (10-d Gaussian + the twisted pair standing in for (N_eff, m_s)),
  MLP 12->1024x4->1, HMC (L = 10) at 16384 chains in BF16 and FP16: 1000 adaptation + 2000
  production steps, min-ESS/s, the log pi error of each precision against the library's FP32
  GEMM path on posterior draws (the error against the FP64 oracle on such draws is
  tests/test_gpu_configs.py; FP64 GEMMs at width 1024 exceed the LDS budget), and, with
  the emulator term off, the posterior moments against the closed form (the twisted pair's
  mean and variances).
* c4: the learned emulator: 2e5 Latin-hypercube pairs in the training box from the plain
  spectrum model, MLP 6->512x4->1 trained by the library's Adam kernels, then MALA with 4096
  chains on the emulator (BF16 and FP32; plain model outside the training box) and on the
  plain model alone: min-ESS/s of each, the gain, and the Kish ESS of the importance weights
  of the emulator's draws under the plain likelihood.

Usage:  python -m paper_2606_04895_amd.configs c1 | c3 | c4 [--quick] [--json f]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))


def _emit(out, rec):
    print(json.dumps(rec), flush=True)
    out.append(rec)


def _per_s(ess, flags, seconds, B):
    """min ESS / seconds, or None when any parameter's ESS is flagged (frozen chains, or a
    window shorter than the autocorrelation)."""
    if any(int(f) != B.A.BEST_ESS_OK for f in flags):
        return None
    return float(ess.min()) / seconds


def _percentiles(v):
    a = np.abs(np.asarray(v))
    return dict(p50=float(np.percentile(a, 50)), p99=float(np.percentile(a, 99)),
                max=float(a.max()))


def c1_setup(quick=False):
    """The c1 problem, chain count, steps, discarded steps, whitening factor L = chol S,
    start points (exact draws of N(mu, S)) and MH scale."""
    from workloads import make_problem
    prob = make_problem("c1")
    d, n = prob["d"], 64 if not quick else 16
    steps, burn = (2000, 500) if not quick else (200, 50)
    L = np.linalg.cholesky(prob["closed_cov"])
    x0 = prob["gauss_mean"] + np.random.default_rng(prob["seed"]).normal(size=(n, d)) @ L.T
    return prob, n, steps, burn, L, x0, 2.4 / np.sqrt(d)


def c1_gpu(quick=False):
    """Runs c1 on the GPU; returns (record, recorded draws [T][d][n] CUDA, final x (n, d))."""
    import paper_2606_04895_amd as B
    from paper_2606_04895_amd import driver
    prob, n, steps, burn, L, x0, scale = c1_setup(quick)
    d = prob["d"]
    ctx = B.best_init(prob, n_chains=n, precision="fp64", seed=prob["seed"])
    B.best_set_whitening(ctx, prob["gauss_mean"], L)
    B.best_set_state(ctx, x0.T.copy())
    b = B.best_step(ctx, "mh", burn, mh_scale=scale)
    st, rec, wall, _ = driver.sample(ctx, "mh", steps - burn, d, n, mh_scale=scale, ess=False)
    ess, flags = B.best_ess(ctx, rec, flags=True)
    x_gpu = B.best_get_state(ctx)[0].T.copy()
    ks = st["ms"] * 1e-3
    r = dict(kind="config_run", config="c1", precision="fp64", sampler="mh", chains=n,
             steps=steps, discarded=burn, accept=(b["accepted"] + st["accepted"]) / (steps * n),
             production_kernel_s=ks, production_wall_s=wall,
             min_ess=float(ess.min()), ess_flags=[B.ESS_FLAGS[int(f)] for f in flags],
             min_ess_per_s=_per_s(ess, flags, ks, B), evals_per_s=st["evals"] / ks)
    ctx.close()
    return r, rec, x_gpu


def run_c1(args, out):
    r, _, _ = c1_gpu(args.quick)
    _emit(out, r)


def _error_vs(B, prob, xs, prec_ctx, ref_prec="fp32"):
    """log pi at draws xs ([d][m] CUDA float64): error of prec_ctx against a context of the
    same problem with ref_prec GEMMs."""
    cr = B.best_init(prob, n_chains=16, precision=ref_prec, seed=1)
    lpr, _ = B.best_logL_grad(cr, xs, want_grad=False)
    lpp, _ = B.best_logL_grad(prec_ctx, xs, want_grad=False)
    cr.close()
    return _percentiles((lpp - lpr).cpu().numpy())


def c3_run(prec, with_mlp=True, n=16384, warm=1000, steps=2000, init="uniform",
           init_scale=1.0, schedule=None, recenter=False):
    """HMC (L = 10) on c3: returns (record, recorded draws [T][d][n], context, problem)."""
    import paper_2606_04895_amd as B
    from paper_2606_04895_amd import driver
    from workloads import make_problem
    prob = make_problem("c3", with_mlp=with_mlp)
    d = prob["d"]
    ctx = B.best_init(prob, n_chains=n, precision=prec, seed=prob["seed"], init=init,
                      init_scale=init_scale)
    t_adapt = driver.burn_in(ctx, "hmc", warm, d, n, schedule=schedule, recenter=recenter)
    if steps == 0:
        return dict(adapt_s=t_adapt), None, ctx, prob
    st, rec, wall, _ = driver.sample(ctx, "hmc", steps, d, n, chunk=250, ess=False)
    ess, flags = B.best_ess(ctx, rec, flags=True)
    ks = st["ms"] * 1e-3
    r = dict(kind="config_run", config="c3", emulator_term=with_mlp, precision=prec,
             sampler="hmc", n_leapfrog=10, chains=n, init=init, init_scale=init_scale,
             schedule=schedule or driver.SCHEDULE["hmc"], recenter=recenter,
             adaptation_steps=warm,
             production_steps=steps, adapt_s=t_adapt, production_kernel_s=ks,
             accept=st["accepted"] / (steps * n), eps=st["eps"],
             min_ess=float(ess.min()), ess_flags=[B.ESS_FLAGS[int(f)] for f in flags],
             min_ess_per_s=_per_s(ess, flags, ks, B), evals_per_s=st["evals"] / ks,
             nonfinite=st["n_nonfinite"])
    return r, rec, ctx, prob


# c3 starts from the hypersphere-based perturbation of the box centre (Sec. 3.2), radius a
# quarter of the initial whitening scale (about one marginal sd): from a uniform start in the
# +-20 sd box the far walkers' gradients drive dual averaging to a step size 12x too small and
# the ensemble never contracts within the warm-up.
C3_INIT = dict(init="hypersphere", init_scale=0.25)


def run_c3(args, out):
    import torch
    import paper_2606_04895_amd as B

    n = 16384 if not args.quick else 2048
    warm, steps = (1000, 2000) if not args.quick else (200, 200)
    for with_mlp in (True, False):
        for prec in ("bf16", "fp16"):
            r, rec, ctx, prob = c3_run(prec, with_mlp, n, warm, steps, **C3_INIT)
            d = prob["d"]
            x = rec[steps // 2:].double().permute(1, 0, 2).reshape(d, -1)
            if with_mlp:
                idx = torch.randperm(x.shape[1], generator=torch.Generator().manual_seed(3))[:4096]
                xs = x[:, idx.to(x.device)].contiguous()
                r["logpi_error_vs_fp32_gemms"] = _error_vs(B, prob, xs, ctx)
            else:
                r.update(_closed_form_moments(prob, x))
                r["mc_se_mean_sd"] = float(1.0 / np.sqrt(max(r["min_ess"], 1.0)))
            del x, rec
            torch.cuda.synchronize()
            _emit(out, r)
            ctx.close()
    # the twisted pair mixes slowly under one global step size: a long thinned run of the
    # emulator-off target, moments against the closed form over its second half
    n_l, steps_l, thin = (4096, 40000, 20) if not args.quick else (1024, 2000, 10)
    r, _, ctx, prob = c3_run("bf16", False, n_l, warm, 0, **C3_INIT)
    d = prob["d"]
    rec = torch.empty((steps_l // thin, d, n_l), dtype=torch.float32, device="cuda")
    st = B.best_step(ctx, "hmc", steps_l, n_leapfrog=10, thin=thin, record=rec)
    x = rec[rec.shape[0] // 2:].double().permute(1, 0, 2).reshape(d, -1)
    ess, flags = B.best_ess(ctx, rec[rec.shape[0] // 2:].contiguous(), flags=True)
    rl = dict(kind="config_long_run", config="c3", emulator_term=False, precision="bf16",
              sampler="hmc", chains=n_l, adaptation_steps=warm, production_steps=steps_l,
              thin=thin, production_kernel_s=st["ms"] * 1e-3,
              accept=st["accepted"] / (steps_l * n_l), eps=st["eps"],
              min_ess_thinned=float(ess.min()), ess_flags=[B.ESS_FLAGS[int(f)] for f in flags],
              **_closed_form_moments(prob, x))
    _emit(out, rl)
    del x, rec
    ctx.close()


def _closed_form_moments(prob, x):
    """Moments of draws x ([d][m] CUDA float64) against the closed form of the emulator-off
    c3 target: mean mu and variances diag(closed_cov); the twisted pair is (6, 7)."""
    m = x.mean(1).cpu().numpy()
    v = x.var(1).cpu().numpy()
    sd = np.sqrt(np.diag(prob["closed_cov"]))
    gauss = [i for i in range(prob["d"]) if i not in (6, 7)]
    return dict(gauss_max_mean_err_sd=float(np.max(np.abs(m - prob["closed_mean"])[gauss] / sd[gauss])),
                gauss_var_ratio_min=float(np.min(v[gauss] / sd[gauss] ** 2)),
                gauss_var_ratio_max=float(np.max(v[gauss] / sd[gauss] ** 2)),
                pair_mean_err_sd=[float((m[i] - prob["closed_mean"][i]) / sd[i]) for i in (6, 7)],
                pair_var_ratio=[float(v[i] / sd[i] ** 2) for i in (6, 7)])


def run_c4(args, out):
    import torch
    import paper_2606_04895_amd as B
    from paper_2606_04895_amd import driver
    from workloads import make_problem

    prob = make_problem("c4")
    d = prob["d"]
    n_train, epochs = (200000, 60) if not args.quick else (32768, 10)
    n = 4096 if not args.quick else 1024
    warm, steps = (1000, 4000) if not args.quick else (200, 200)
    tr = driver.train_emulator(prob, n_train=n_train, epochs=epochs, batch=1024,
                               precision="fp32", seed=prob["seed"], lr0=2e-3, lr1=1e-5)
    _emit(out, dict(kind="config_training", config="c4", pairs=n_train, epochs=epochs,
                    batch=1024, loss_first=tr["losses"][0], loss_last=tr["losses"][-1],
                    data_s=tr["data_s"], train_s=tr["train_s"], y_mu=tr["y_mu"],
                    y_sigma=tr["y_sigma"]))
    emu = driver.emulator_problem(prob, tr)
    plain = dict(prob, plain_mode=2)
    ts = prob["plain"]["theta_star"]
    res = {}
    for name, p, prec in (("emulator", emu, "bf16"), ("emulator", emu, "fp32"),
                          ("plain", plain, "fp32")):
        ctx = B.best_init(p, n_chains=n, precision=prec, seed=prob["seed"] + 1, init="gaussian",
                          init_point=ts, init_scale=0.02)
        t_adapt = driver.burn_in(ctx, "mala", warm, d, n)
        st, rec, wall, _ = driver.sample(ctx, "mala", steps, d, n, chunk=500, ess=False)
        ess, flags = B.best_ess(ctx, rec, flags=True)
        ks = st["ms"] * 1e-3
        r = dict(kind="config_run", config="c4", target=name, precision=prec, sampler="mala",
                 chains=n, adaptation_steps=warm, production_steps=steps, adapt_s=t_adapt,
                 production_kernel_s=ks, accept=st["accepted"] / (steps * n), eps=st["eps"],
                 min_ess=float(ess.min()), ess_flags=[B.ESS_FLAGS[int(f)] for f in flags],
                 min_ess_per_s=_per_s(ess, flags, ks, B), evals_per_s=st["evals"] / ks)
        if name == "emulator":
            xs = rec[steps // 2:].permute(1, 0, 2).reshape(d, -1).double()
            idx = torch.randperm(xs.shape[1], generator=torch.Generator().manual_seed(5))[:65536]
            xs = xs[:, idx.to(xs.device)].contiguous()
            cp = B.best_init(plain, n_chains=16, precision="fp32", seed=1)
            lp, _ = B.best_logL_grad(cp, xs, want_grad=False)
            le, _ = B.best_logL_grad(ctx, xs, want_grad=False)
            _, kish = B.best_importance_weights(lp, le)
            r["importance_draws"] = int(xs.shape[1])
            r["kish_ess"] = float(kish)
            r["kish_fraction"] = float(kish) / xs.shape[1]
            r["logL_emu_minus_plain"] = _percentiles((le - lp - (le - lp).mean()).cpu().numpy())
            cp.close()
        res[(name, prec)] = r
        del rec
        torch.cuda.synchronize()
        _emit(out, r)
        ctx.close()
    def gain(a, b):
        return None if a is None or b is None else a / b
    base = res[("plain", "fp32")]["min_ess_per_s"]
    _emit(out, dict(kind="config_gain", config="c4",
                    emulator_bf16_over_plain=gain(res[("emulator", "bf16")]["min_ess_per_s"], base),
                    emulator_fp32_over_plain=gain(res[("emulator", "fp32")]["min_ess_per_s"], base)))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("config", choices=["c1", "c3", "c4"])
    ap.add_argument("--quick", action="store_true")
    ap.add_argument("--json", default=None)
    args = ap.parse_args()
    out = []
    {"c1": run_c1, "c3": run_c3, "c4": run_c4}[args.config](args, out)
    if args.json:
        with open(args.json, "w") as f:
            json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()

"""Sampler comparison on the 27-parameter workload (6 cosmological-like + 21 linear nuisance
parameters, Gaussian part plus a 27 -> 1024 x 5 -> 1 tanh emulator in BF16 GEMMs; --config c3
gives the 12-parameter twisted target of the second experiment): AIES (stretch move, a = 2,
two half-ensembles), NUTS (maximum depth 8), MALA and HMC (10 leapfrog steps), each after its
own burn-in with covariance and (for the gradient samplers) step-size adaptation, compared on
min-ESS/s (the smallest multi-chain ESS over the parameters divided by the production wall
time), on emulator evaluations per second, and on the convergence metrics of Sec. 4.1: R - 1
of the production chains, and the credible metric (68% and 95%) and sliced Wasserstein
distance (500 directions) against a reference posterior from a long MALA run, in the
reference's whitened coordinates; a second independent reference run gives the noise floor
of the last two, as the paper does with its reference runs.

For NUTS it also reports the mean number of leaves per transition and the efficiency of the
lockstep tile execution: useful evaluations per second against the HMC transition's rate on
the same ensemble (every HMC evaluation is useful).

Usage:  python -m paper_2606_04895_amd.compare [--chains N] [--json out.json]
Every result is printed as one JSON object per line.
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", default="c5")
    ap.add_argument("--chains", type=int, default=65536)
    ap.add_argument("--precision", default="bf16")
    ap.add_argument("--max-depth", type=int, default=8)
    ap.add_argument("--json", default=None)
    ap.add_argument("--quick", action="store_true")
    ap.add_argument("--sw-steps", type=int, default=8,
                    help="last steps of each run whose draws enter the sliced Wasserstein")
    ap.add_argument("--recenter", action="store_true",
                    help="re-centre the ensemble on its best-fit walker after each covariance "
                         "window of the burn-in (gradient samplers, MH and the reference)")
    ap.add_argument("--scale", type=float, default=1.0,
                    help="multiply every warm-up and production length")
    args = ap.parse_args()
    import torch
    import paper_2606_04895_amd as B
    from paper_2606_04895_amd import driver
    from workloads import make_problem

    prob = make_problem(args.config)
    d, n = prob["d"], args.chains
    plan = {  # (warm-up steps, production steps): the same lengths for every sampler
        "aies": (2000, 2000),
        "mala": (2000, 2000),
        "hmc": (2000, 2000),
        "nuts": (2000, 2000),
    }
    if args.quick:
        plan = {k: (max(50, w // 10), max(50, s // 10)) for k, (w, s) in plan.items()}
    plan = {k: (int(w * args.scale), int(s * args.scale)) for k, (w, s) in plan.items()}
    results = []

    def emit(obj):
        results.append(obj)
        print(json.dumps(obj), flush=True)

    def run(sampler, seed, warm, steps):
        ctx = B.best_init(prob, n_chains=n, precision=args.precision, seed=seed, init="uniform")
        t_burn = driver.burn_in(ctx, sampler, warm, d, n, max_depth=args.max_depth,
                                recenter=args.recenter)
        st, rec, wall, _ = driver.sample(ctx, sampler, steps, d, n, max_depth=args.max_depth,
                                         ess=False)
        ess, flags = B.best_ess(ctx, rec, flags=True)
        return ctx, st, rec, wall, (ess, flags), t_burn

    # reference posterior: two independent long MALA runs (the second sets the noise floor of
    # the credible metric and the sliced Wasserstein distance, as in Sec. 4.1)
    ref_warm, ref_steps = (200, 400) if args.quick else (2000, 4000)
    ref_warm, ref_steps = int(ref_warm * args.scale), int(ref_steps * args.scale)
    ref = {}

    def metrics(ctx, prod, tail):
        W = ref["W"]
        out = dict(rminus1=B.best_rhat(ctx, prod))
        for a in (0.68, 0.95):
            lo0, hi0 = ref["lim"][a]
            out[f"cm{int(a * 100)}"] = B.best_credible(ctx, prod, a, whitening=W, ref=(lo0, hi0))[2]
        out["sliced_w"] = B.best_sliced_wasserstein(ctx, tail, ref["tail"], 500, 0x5EED,
                                                    whitening=W)
        return out

    for k in range(2):
        ctx, st, rec, wall, ess, _ = run("mala", 0xF00D + k, ref_warm, ref_steps)
        keep = rec[ref_steps // 2:].contiguous()
        tail = rec[-args.sw_steps:].contiguous()
        del rec
        if k == 0:
            # the reference whitening from the library's own moments and Cholesky (the
            # adaptation path), over the retained half of the run; the run is finished, so
            # its context's whitening may change
            B.best_adapt(ctx, samples=keep, update_mean=True)
            mu, L = B.best_get_whitening(ctx)
            ref.update(W=(mu, L), tail=tail, ctx=ctx,
                       lim={a: B.best_credible(ctx, keep, a, whitening=(mu, L))[:2]
                            for a in (0.68, 0.95)})
        else:
            floor = metrics(ctx, keep, tail)
            emit(dict(kind="metric_reference_pair", config=args.config, reference="mala",
                      chains=n, warmup=ref_warm, steps=ref_steps, sw_draws=args.sw_steps * n,
                      min_ess=float(ess[0].min()), **floor))
            ctx.close()
        del keep
        torch.cuda.synchronize()

    for i, (sampler, (warm, steps)) in enumerate(plan.items()):
        ctx, st, rec, wall, ess, t_burn = run(sampler, 0xC5 + i, warm, steps)
        prod = rec[steps // 2:].contiguous()
        m = metrics(ctx, prod, rec[-args.sw_steps:].contiguous())
        del prod
        ess, flags = ess
        # a min-ESS/s only for a converged run: no flagged ESS and R - 1 below 0.1
        reason = None
        if any(int(f) != B.A.BEST_ESS_OK for f in flags):
            reason = "ESS flagged: " + ",".join(sorted({B.ESS_FLAGS[int(f)] for f in flags}))
        elif not m["rminus1"] < 0.1:
            reason = f"not converged: R - 1 = {m['rminus1']:.3g}"
        row = dict(kind="sampler_comparison", config=args.config, precision=args.precision,
                   sampler=sampler, chains=n, d=d, warmup=warm, steps=steps,
                   burn_in_s=t_burn, production_s=wall, min_ess=float(ess.min()),
                   min_ess_per_s=None if reason else float(ess.min()) / wall,
                   min_ess_null_reason=reason, evals=int(st["evals"]),
                   evals_per_s=st["evals"] / wall,
                   accept=st["sum_accept_prob"] / (steps * n), eps=st["eps"], **m)
        del rec
        torch.cuda.synchronize()
        if sampler == "nuts":
            row["max_depth"] = args.max_depth
            row["leaves_per_transition"] = st["evals"] / (steps * n)
            # lockstep efficiency: HMC on the same ensemble and step size, 10 leapfrog steps
            B.best_step(ctx, "hmc", 2, eps=st["eps"], n_leapfrog=10)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            h = B.best_step(ctx, "hmc", 20, eps=st["eps"], n_leapfrog=10)
            torch.cuda.synchronize()
            row["hmc_evals_per_s"] = h["evals"] / (time.perf_counter() - t0)
            row["lockstep_efficiency"] = row["evals_per_s"] / row["hmc_evals_per_s"]
        emit(row)
        ctx.close()
    ref["ctx"].close()
    if args.json:
        with open(args.json, "w") as f:
            json.dump(results, f, indent=1)


if __name__ == "__main__":
    main()

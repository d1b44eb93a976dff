"""Sampler comparison on the 27-parameter workload (6 cosmological-like + 21 linear nuisance
parameters, Gaussian part plus a 27 -> 1024 x 5 -> 1 tanh emulator in BF16 GEMMs): AIES
(stretch move, a = 2, two half-ensembles), NUTS (maximum depth 8) and MALA, each after its
own burn-in with covariance and (for the gradient samplers) step-size adaptation, compared on
min-ESS/s (the smallest multi-chain ESS over the parameters divided by the production wall
time), on emulator evaluations per second, and on the posterior moments they reach.

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
    args = ap.parse_args()
    import torch
    import paper_2606_04895_amd as B
    from paper_2606_04895_amd import driver
    from workloads import make_problem

    prob = make_problem(args.config)
    d, n = prob["d"], args.chains
    plan = {  # (warm-up steps, production steps)
        "aies": (2000, 2000),
        "mala": (1000, 2000),
        "nuts": (400, 300),
    }
    if args.quick:
        plan = {k: (max(50, w // 10), max(50, s // 10)) for k, (w, s) in plan.items()}
    results = []

    def emit(obj):
        results.append(obj)
        print(json.dumps(obj), flush=True)

    moments = {}
    for sampler, (warm, steps) in plan.items():
        ctx = B.best_init(prob, n_chains=n, precision=args.precision, seed=0xC5 + len(moments),
                          init="uniform")
        t_burn = driver.burn_in(ctx, sampler, warm, d, n, max_depth=args.max_depth)
        st, rec, wall, ess = driver.sample(ctx, sampler, steps, d, n, max_depth=args.max_depth)
        r = rec[steps // 2:].double()
        mean = r.mean(dim=(0, 2))
        flat = r.permute(0, 2, 1).reshape(-1, d)
        cov = torch.cov(flat.T)
        moments[sampler] = (mean.cpu().numpy(), cov.cpu().numpy())
        del rec, r, flat
        torch.cuda.synchronize()
        row = dict(kind="sampler_comparison", config=args.config, precision=args.precision,
                   sampler=sampler, chains=n, d=d, warmup=warm, steps=steps,
                   burn_in_s=t_burn, production_s=wall, min_ess=float(ess.min()),
                   min_ess_per_s=float(ess.min()) / wall, evals=int(st["evals"]),
                   evals_per_s=st["evals"] / wall,
                   accept=st["sum_accept_prob"] / (steps * n), eps=st["eps"])
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

    # agreement of the three posteriors (second half of each production run), in units of
    # the marginal standard deviations of the NUTS run
    sd = np.sqrt(np.diag(moments["nuts"][1]))
    for a_, b_ in (("aies", "nuts"), ("mala", "nuts"), ("aies", "mala")):
        ma, ca = moments[a_]
        mb, cb = moments[b_]
        emit(dict(kind="posterior_agreement", config=args.config, pair=f"{a_}-{b_}",
                  max_mean_diff_sigma=float(np.max(np.abs(ma - mb) / sd)),
                  max_sd_rel_diff=float(np.max(np.abs(np.sqrt(np.diag(ca)) /
                                                      np.sqrt(np.diag(cb)) - 1)))))
    if args.json:
        with open(args.json, "w") as f:
            json.dump(results, f, indent=1)


if __name__ == "__main__":
    main()

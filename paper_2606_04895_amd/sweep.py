"""Secondary measurements on one GPU (the benchmark line itself is bench.py):

* throughput sweep: standalone best_logL_grad evaluations per second against the number of
  points N for the C2, C3 and C5 networks in BF16 and FP32 (the batched-evaluation curve of
  the paper's Fig. 1, re-measured), and HMC evaluations per second inside the sampler;
* NUTS on the C2 workload: leaves per transition and useful evaluations per second;
* the BF16 / FP32 pair on the C3 network at 4096 chains;
* BF16 accuracy: the error of BF16 log pi against the FP64 GEMM path on posterior samples,
  and the posterior moments of BF16 chains against FP32 chains on the C2 workload.

Usage:  python -m paper_2606_04895_amd.sweep [--quick] [--json out.json]
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


def _flops(d, H, nh):
    return 2 * (d * H + (nh - 1) * H * H + H + (nh - 1) * H * H + d * H)


def eval_rate(B, torch, prob, prec, n, reps, grad=True):
    """Evaluations per second of best_logL_grad on n device-resident points."""
    ctx = B.best_init(prob, n_chains=16, precision=prec, seed=5)
    rng = np.random.default_rng(n)
    x = prob["lower"] + rng.uniform(size=(n, prob["d"])) * (prob["upper"] - prob["lower"])
    xt = torch.tensor(x.T.copy(), device="cuda")
    lp = torch.empty(n, dtype=torch.float64, device="cuda")
    g = torch.empty((prob["d"], n), dtype=torch.float64, device="cuda") if grad else None
    out = (lp, g)
    B.best_logL_grad(ctx, xt, want_grad=grad, out=out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        B.best_logL_grad(ctx, xt, want_grad=grad, out=out)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    ctx.close()
    return n / (ms * 1e-3), ms


def hmc_rate(B, prob, prec, n, steps=20):
    ctx = B.best_init(prob, n_chains=n, precision=prec, seed=5)
    B.best_set_step_size(ctx, 0.2)
    B.best_step(ctx, "hmc", 2, n_leapfrog=10)
    st = B.best_step(ctx, "hmc", steps, n_leapfrog=10)
    ctx.close()
    return st["evals"] / (st["ms"] * 1e-3)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true")
    ap.add_argument("--json", default=None)
    args = ap.parse_args()
    import torch
    import paper_2606_04895_amd as B
    from paper_2606_04895_amd import driver
    from workloads import make_problem

    results = []

    def emit(obj):
        results.append(obj)
        print(json.dumps(obj), flush=True)

    ns = [64, 256, 1024, 4096, 16384, 65536]
    nets = ["c2", "c3", "c5"]
    if args.quick:
        ns, nets = [256, 4096], ["c2"]
    # ---- throughput vs N (standalone and in-sampler) ----
    for name in nets:
        prob = make_problem(name)
        d, H, nh = prob["d"], prob["width"], prob["n_hidden"]
        for prec in ("bf16", "fp32"):
            for n in ns:
                reps = max(3, min(200, 2_000_000 // n))
                rate, ms = eval_rate(B, torch, prob, prec, n, reps)
                emit(dict(kind="eval_sweep", net=f"{d}->{H}x{nh}->1", config=name, prec=prec, n=n,
                          evals_per_s=rate, ms_per_call=ms,
                          tflops=rate * _flops(d, H, nh) / 1e12))
            for n in (4096, 16384):
                if args.quick and n > 4096:
                    continue
                rate = hmc_rate(B, prob, prec, n)
                emit(dict(kind="hmc_rate", net=f"{d}->{H}x{nh}->1", config=name, prec=prec, n=n,
                          evals_per_s=rate, tflops=rate * _flops(d, H, nh) / 1e12))

    # ---- NUTS on the C2 workload at 4096 chains: leaves per transition and the useful
    #      evaluation rate of the lockstep tiles against HMC's on the same ensemble ----
    prob = make_problem("c2")
    ctx = B.best_init(prob, n_chains=4096, precision="bf16", seed=9, init="uniform")
    driver.burn_in(ctx, "nuts", 300, prob["d"], 4096)
    st = B.best_step(ctx, "nuts", 20 if args.quick else 100, max_depth=8)
    steps = 20 if args.quick else 100
    hm = B.best_step(ctx, "hmc", 20, eps=st["eps"], n_leapfrog=10)
    emit(dict(kind="nuts_rate", config="c2", prec="bf16", n=4096, steps=steps,
              leaves_per_transition=st["evals"] / (steps * 4096),
              evals_per_s=st["evals"] / (st["ms"] * 1e-3), eps=st["eps"],
              accept_stat=st["sum_accept_prob"] / (steps * 4096),
              hmc_evals_per_s=hm["evals"] / (hm["ms"] * 1e-3)))
    ctx.close()

    # ---- host-pointer mode (PCIe copies inside the call) on C2 at 4096 points ----
    prob = make_problem("c2")
    c = B.best_init(prob, n_chains=16, precision="bf16", seed=5)
    xh = (prob["lower"][:, None] + np.random.default_rng(0).uniform(size=(prob["d"], 4096))
          * (prob["upper"] - prob["lower"])[:, None])
    B.best_logL_grad(c, xh)
    t0 = time.perf_counter()
    for _ in range(20):
        B.best_logL_grad(c, xh)
    dt = (time.perf_counter() - t0) / 20
    c.close()
    emit(dict(kind="eval_host_ptrs", config="c2", prec="bf16", n=4096, evals_per_s=4096 / dt,
              ms_per_call=dt * 1e3))

    # ---- BF16 accuracy against the FP64 GEMM path on posterior samples (C2) ----
    prob = make_problem("c2")
    d = prob["d"]
    n = 4096
    ctx = B.best_init(prob, n_chains=n, precision="bf16", seed=11, init="uniform")
    driver.burn_in(ctx, "hmc", 1000, d, n)
    st, rec, wall, ess = driver.sample(ctx, "hmc", 1000 if not args.quick else 200, d, n)
    ctx.close()
    pts = rec[-1].double()  # [d][n] final ensemble
    ref = B.best_init(prob, n_chains=16, precision="fp64", seed=1)
    lp64, g64 = B.best_logL_grad(ref, pts.contiguous())
    ref.close()
    for prec in ("bf16", "fp16", "fp32"):
        c = B.best_init(prob, n_chains=16, precision=prec, seed=1)
        lp, g = B.best_logL_grad(c, pts.contiguous())
        c.close()
        err = (lp - lp64).abs().cpu().numpy()
        gerr = ((g - g64).norm(dim=0) / g64.norm(dim=0).clamp_min(1e-300)).cpu().numpy()
        emit(dict(kind="logpi_error_vs_fp64", config="c2", prec=prec, n_points=n,
                  abs_err_median=float(np.median(err)), abs_err_p99=float(np.quantile(err, 0.99)),
                  abs_err_max=float(err.max()), grad_rel_err_median=float(np.median(gerr)),
                  grad_rel_err_p99=float(np.quantile(gerr, 0.99))))

    # ---- posterior moments: BF16 chains against FP32 chains (C2, HMC and MALA) ----
    steps = 1000 if args.quick else 4000
    for sampler in ("hmc", "mala"):
        mom = {}
        for prec in ("fp32", "bf16"):
            c = B.best_init(prob, n_chains=n, precision=prec, seed=21 if prec == "fp32" else 22,
                            init="uniform")
            driver.burn_in(c, sampler, 1000, d, n)
            st, rec, wall, ess = driver.sample(c, sampler, steps, d, n)
            c.close()
            r = rec.double().permute(0, 2, 1).reshape(-1, d)
            mean = r.mean(0)
            cov = torch.cov(r.T)
            mom[prec] = (mean.cpu().numpy(), cov.cpu().numpy(), float(ess.min()))
            del rec, r
            torch.cuda.synchronize()
        m32, c32, ess32 = mom["fp32"]
        m16, c16, ess16 = mom["bf16"]
        sd = np.sqrt(np.diag(c32))
        ess_min = min(ess32, ess16)
        emit(dict(kind="posterior_bf16_vs_fp32", config="c2", sampler=sampler, steps=steps,
                  chains=n, min_ess=ess_min,
                  max_mean_diff_sigma=float(np.max(np.abs(m16 - m32) / sd)),
                  mc_error_sigma=float(np.sqrt(2.0 / ess_min)),
                  max_sd_rel_diff=float(np.max(np.abs(np.sqrt(np.diag(c16)) / sd - 1))),
                  max_corr_diff=float(np.max(np.abs(c16 / np.outer(np.sqrt(np.diag(c16)),
                                                                     np.sqrt(np.diag(c16)))
                                                     - c32 / np.outer(sd, sd))))))

    # ---- BF16 / FP32 pair on the C3 network at 4096 chains ----
    if not args.quick:
        prob3 = make_problem("c3")
        for sampler in ("mala", "hmc"):
            rates = {}
            for prec in ("bf16", "fp32"):
                c = B.best_init(prob3, n_chains=4096, precision=prec, seed=31, init="uniform")
                driver.burn_in(c, sampler, 200, prob3["d"], 4096)
                st, rec, wall, ess = driver.sample(c, sampler, 200, prob3["d"], 4096, ess=True)
                c.close()
                rates[prec] = dict(evals_per_s=st["evals"] / wall, min_ess_per_s=float(ess.min()) / wall)
                del rec
            emit(dict(kind="c3_net_pair", sampler=sampler, chains=4096, steps=200, warmup=200,
                      bf16=rates["bf16"], fp32=rates["fp32"],
                      speedup_evals=rates["bf16"]["evals_per_s"] / rates["fp32"]["evals_per_s"]))

    if args.json:
        with open(args.json, "w") as f:
            json.dump(results, f, indent=1)


if __name__ == "__main__":
    main()

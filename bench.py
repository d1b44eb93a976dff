#!/usr/bin/env python
"""Benchmark of the batched emulator sampler on one MI355X.

Metric: min-ESS/s and emulator logL+grad evals/s at 4096 chains, BF16-MFMA vs FP32.
Workload (default, "c2"): 6-parameter Gaussian (cond 1e3) + 0.5*MLP(6->512x4->1, tanh)
target, 4096 chains, MALA and HMC (L = 10) in whitened space.  For each precision the run
is: uniform init in the prior box, `--warmup` adaptation steps (three windows ending at
1/4, 1/2 and 1 of the warmup, dual-averaged step size towards 0.57 / 0.8 inside each
window, covariance re-estimated from the second half of each window), then `--steps`
timed production steps with every step recorded, then the multi-chain ESS.

A "step" of the timed region is one ensemble iteration of MALA plus one of HMC at BF16
(every chain advances once under each sampler).  value = BF16 emulator logL+grad evals/s
over those production runs; FP32 is timed the same way and reported beside it.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"bf16": 2.5e15, "fp16": 2.5e15, "fp32": 157.3e12, "fp64": 78.6e12}


def flops_per_eval(d, H, nh):
    """Algorithmic flops of one logL+grad evaluation (2 per multiply-add)."""
    fwd = d * H + (nh - 1) * H * H + H
    bwd = (nh - 1) * H * H + d * H
    return 2 * (fwd + bwd)


def gemm_flops_per_eval(H, nh):
    return 2 * 2 * (nh - 1) * H * H


KERNEL_SOURCES = os.path.join(ROOT, "paper_2606_04895_amd", "csrc")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pmc_step_kernel_bf16_hmc_c2.txt")


def kernel_source_hash():
    """sha256 over the HIP/C++ sources of the library (names and contents, sorted)."""
    import hashlib
    h = hashlib.sha256()
    for name in sorted(os.listdir(KERNEL_SOURCES)):
        path = os.path.join(KERNEL_SOURCES, name)
        if os.path.isfile(path):
            h.update(name.encode())
            with open(path, "rb") as f:
                h.update(f.read())
    return h.hexdigest()


def measured_traffic(steps, chains, n_leap):
    """HBM bytes per production launch of the dominant kernel, from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE, each scaled by the factor a plain device copy of
    known size gives).  None if the summary is missing, was taken for another launch shape,
    or the kernel sources have changed since."""
    try:
        with open(TRAFFIC_FILE) as f:
            kv = dict(ln.split("=", 1) for ln in f.read().splitlines() if "=" in ln and not ln.startswith("#"))
        kv = {k.strip(): v.strip() for k, v in kv.items()}
        if kv.get("source_sha256") != kernel_source_hash():
            return None
        if (int(kv["steps"]), int(kv["chains"]), int(kv["n_leapfrog"])) != (steps, chains, n_leap):
            return None
        return float(kv["hbm_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def run_chain(B, torch, prob, prec, sampler, n, warmup, steps, seed, n_leap):
    from paper_2606_04895_amd import driver

    d = prob["d"]
    ctx = B.best_init(prob, n_chains=n, precision=prec, seed=seed, init="uniform")
    t_adapt = driver.burn_in(ctx, sampler, warmup, d, n, n_leap=n_leap)
    st, rec, wall, ess = driver.sample(ctx, sampler, steps, d, n, n_leap=n_leap)
    mean = rec.double().mean(dim=(0, 2)).cpu().numpy()
    out = dict(wall_s=wall, kernel_ms=st["ms"], evals=st["evals"],
               accept=st["accepted"] / (steps * n), eps=st["eps"], adapt_s=t_adapt,
               min_ess=float(ess.min()), ess=[float(v) for v in ess],
               min_ess_per_s=float(ess.min()) / wall, evals_per_s=st["evals"] / wall,
               nonfinite=st["n_nonfinite"], post_mean=[float(v) for v in mean])
    del rec
    ctx.close()
    return out


def cpu_baseline(prob, n, budget_s, seed):
    """The oracle (numpy FP64) running MALA on the same workload for a bounded sample."""
    import numpy as np
    from oracle import samplers as OS

    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        cores = os.cpu_count() or 1
    W = dict(mu=prob["gauss_mean"], L=np.linalg.cholesky(prob["closed_cov"]))
    rng = np.random.default_rng(seed)
    x0 = prob["gauss_mean"] + rng.normal(size=(n, prob["d"])) @ W["L"].T
    st = OS.init_state(prob, W, x0)
    t0 = time.perf_counter()
    done = 0
    while time.perf_counter() - t0 < budget_s:
        st, _ = OS.mala_step(prob, W, st, done, seed, 0.5)
        done += 1
    el = time.perf_counter() - t0
    return dict(value=done * n / el, unit="emulator logL+grad evals/s", cores=int(cores),
                kind="oracle",
                sample=f"oracle MALA, {n} chains x {done} steps of the c2 workload "
                       f"(FP64 numpy, {el:.1f} s)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--warmup", type=int, default=1000)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--chains", type=int, default=4096)
    ap.add_argument("--precisions", default="bf16,fp32")
    ap.add_argument("--samplers", default="mala,hmc")
    ap.add_argument("--n-leapfrog", type=int, default=10)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--seed", type=int, default=0xBE570002)
    ap.add_argument("--calib-copy-mib", type=int, default=256,
                    help="plain device copy of this many MiB at the start (the reference "
                         "launch for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the sampler's chains "
                                   "would shard across GPUs with one small all-reduce per "
                                   "adaptation window, which is not built here"}))
        sys.exit(2)

    import torch
    import paper_2606_04895_amd as B
    from workloads import make_problem

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU"}))
        sys.exit(1)
    prob = make_problem(args.config)
    d, H, nh = prob["d"], prob["width"], prob["n_hidden"]
    if args.calib_copy_mib:
        n = args.calib_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"# calibration copy: {n * 4} bytes read, {n * 4} bytes written", file=sys.stderr)
        del src, dst
    precs = args.precisions.split(",")
    samplers = args.samplers.split(",")
    results = {}
    for prec in precs:
        results[prec] = {}
        for s in samplers:
            r = run_chain(B, torch, prob, prec, s, args.chains, args.warmup, args.steps,
                          args.seed, args.n_leapfrog)
            results[prec][s] = r
            print(f"# {prec} {s}: {r['evals_per_s']:.3e} evals/s, min-ESS/s {r['min_ess_per_s']:.3e}, "
                  f"accept {r['accept']:.3f}, eps {r['eps']:.3g}, wall {r['wall_s']:.2f}s",
                  file=sys.stderr, flush=True)
    head = precs[0]
    wall = sum(results[head][s]["wall_s"] for s in samplers)
    evals = sum(results[head][s]["evals"] for s in samplers)
    value = evals / wall
    fpe = flops_per_eval(d, H, nh)
    # dominant kernel: the fused HMC step kernel at the head precision (one launch of --steps)
    dom = "hmc" if "hmc" in samplers else samplers[0]
    r = results[head][dom]
    achieved = r["evals"] * fpe / (r["kernel_ms"] * 1e-3)
    traffic = measured_traffic(args.steps, args.chains, args.n_leapfrog) \
        if (head, dom, args.config) == ("bf16", "hmc", "c2") else None
    roof = dict(bound="mfma", kernel=f"step_kernel<{head}, production> ({dom})",
                achieved=achieved / 1e12, peak=PEAK[head] / 1e12, unit="TFLOP/s",
                frac=achieved / PEAK[head], traffic=traffic, flops_per_eval=fpe,
                evals_per_launch=r["evals"], launch_ms=r["kernel_ms"])
    line = dict(
        metric="min-ESS/s and emulator logL+grad evals/s at 4096 chains, bf16-MFMA vs fp32",
        value=value, unit="emulator logL+grad evals/s", n_gpus=1, steps=args.steps,
        warmup=args.warmup, ms_per_step=wall / args.steps * 1e3, higher_is_better=True,
        scaling="weak", vs_baseline=None, dtype=head, data="synthetic",
        config=dict(workload=f"{args.config}: d={d} Gaussian(cond 1e3)+0.5*MLP {d}->{H}x{nh}->1 "
                             f"tanh, {args.chains} chains, {'+'.join(samplers)} "
                             f"(HMC L={args.n_leapfrog}), whitened, adapted",
                    n_chains=args.chains, config_id=args.config),
        min_ess_per_s={p: {s: results[p][s]["min_ess_per_s"] for s in samplers} for p in precs},
        evals_per_s={p: {s: results[p][s]["evals_per_s"] for s in samplers} for p in precs},
        results=results, roofline=roof)
    if len(precs) > 1:
        line["speedup_vs_" + precs[1]] = {
            s: dict(min_ess_per_s=results[head][s]["min_ess_per_s"] / results[precs[1]][s]["min_ess_per_s"],
                    evals_per_s=results[head][s]["evals_per_s"] / results[precs[1]][s]["evals_per_s"])
            for s in samplers}
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(prob, args.chains, args.cpu_budget, args.seed)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

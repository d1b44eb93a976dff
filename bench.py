#!/usr/bin/env python
"""Benchmark of the batched emulator sampler on one MI355X.

Metric: min-ESS/s and emulator logL+grad evals/s at 4096 chains, BF16-MFMA vs FP32.
Workload (default, "c2"): 6-parameter Gaussian (cond 1e3) + 0.5*MLP(6->512x4->1, tanh)
target, 4096 chains, MALA and HMC (L = 10) in whitened space, the same fused sampler with
BF16 or FP32 hidden-layer GEMMs.  For each precision and sampler, whatever the flags:

  1. uniform initialisation in the prior box;
  2. the workload's 1000 adaptation steps (windows doubling from 10 steps for MALA, ending
     at 1/4, 1/2 and 1 of the warm-up for HMC; dual-averaged step size towards acceptance
     0.57 / 0.8 inside each window; covariance and mean re-estimated from the second half
     of each window), outside every timed region;
  3. `--warmup` W untimed production steps (in launches of the timed shape, so at least W);
  4. the timed region: `--steps` K production steps, one launch, every step recorded;
  5. the ESS run: the workload's 4000 production steps (in launches of K steps, recorded),
     the multi-chain ESS of its draws, and min-ESS/s = min ESS / the run's kernel time
     (HIP events).  min-ESS/s is null, with the reason, when the ESS is flagged (frozen or
     untruncated chains) or the acceptance is more than 0.15 from its target.

A "step" of the timed region is one ensemble iteration of MALA plus one of HMC at BF16
(every chain advances once under each sampler).  value = BF16 emulator logL+grad evals/s
over the two timed launches; FP32 is timed the same way and reported beside it.
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


ADAPT_STEPS = 1000      # the workload's adaptation steps (5000 steps, adapted over the first 1000)
ESS_STEPS = 4000        # the workload's production steps
TARGET = {"mala": 0.57, "hmc": 0.8}
ACCEPT_BAND = 0.15
GOLDEN = os.path.join(ROOT, "tests", "golden", "c2_posterior_oracle.json")


def oracle_reference(config):
    """The FP64 oracle's posterior summary of the workload (two independent long runs,
    written by tests/golden/make_c2_posterior.py), or None."""
    if config != "c2":
        return None
    try:
        with open(GOLDEN) as f:
            return json.load(f)
    except (OSError, ValueError):
        return None


def posterior_error(rec, ref):
    """Largest |mean - mean_ref| / sd_ref and the range of the variance ratios of the
    recorded draws ([T][d][n]) against the oracle's first run."""
    import numpy as np
    if ref is None:
        return None
    x = rec.double().permute(0, 2, 1).reshape(-1, rec.shape[1])
    m = x.mean(0).cpu().numpy()
    v = x.var(0).cpu().numpy()
    m0 = np.array(ref["runs"][0]["mean"])
    v0 = np.diag(np.array(ref["runs"][0]["cov"]))
    ratio = v / v0
    return dict(max_mean_err_sd=float(np.max(np.abs(m - m0) / np.sqrt(v0))),
                var_ratio_min=float(ratio.min()), var_ratio_max=float(ratio.max()),
                noise_floor_mean_sd=float(np.max(ref["noise_floor"]["mean_diff_over_sd"])))


def run_chain(B, torch, prob, prec, sampler, n, warmup, steps, seed, n_leap, ref):
    from paper_2606_04895_amd import driver

    d = prob["d"]
    ctx = B.best_init(prob, n_chains=n, precision=prec, seed=seed, init="uniform")
    t_adapt = driver.burn_in(ctx, sampler, ADAPT_STEPS, d, n, n_leap=n_leap)
    if warmup > 0:
        driver.sample(ctx, sampler, -(-warmup // steps) * steps, d, n, n_leap=n_leap,
                      chunk=steps, record=False, ess=False)
    # timed region: K production steps, one launch
    st, rec, wall, _ = driver.sample(ctx, sampler, steps, d, n, n_leap=n_leap, ess=False)
    del rec
    # ESS run: the workload's production length, in launches of the timed shape
    est, erec, _, _ = driver.sample(ctx, sampler, ESS_STEPS, d, n, n_leap=n_leap, chunk=steps,
                                    ess=False)
    ess, flags = B.best_ess(ctx, erec, flags=True)
    ess_s = est["ms"] * 1e-3
    accept = est["accepted"] / (ESS_STEPS * n)
    reason = None
    if any(int(f) != B.A.BEST_ESS_OK for f in flags):
        reason = "ESS flagged: " + ",".join(B.ESS_FLAGS[int(f)] for f in flags)
    elif abs(accept - TARGET[sampler]) > ACCEPT_BAND:
        reason = f"acceptance {accept:.3f} is more than {ACCEPT_BAND} from {TARGET[sampler]}"
    out = dict(wall_s=wall, kernel_ms=st["ms"], evals=st["evals"],
               accept_timed=st["accepted"] / (steps * n), eps=st["eps"], adapt_s=t_adapt,
               adapt_steps=ADAPT_STEPS, ess_steps=ESS_STEPS, ess_kernel_s=ess_s,
               accept=accept, min_ess=float(ess.min()), ess=[float(v) for v in ess],
               ess_flags=[B.ESS_FLAGS[int(f)] for f in flags],
               min_ess_per_s=None if reason else float(ess.min()) / ess_s,
               min_ess_null_reason=reason, evals_per_s=st["evals"] / wall,
               nonfinite=st["n_nonfinite"] + est["n_nonfinite"],
               posterior_vs_oracle=posterior_error(erec, ref))
    del erec
    ctx.close()
    return out


def host_info():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        nproc = os.cpu_count() or 1
    return model, nproc


def cpu_baseline(prob, n, budget_s, seed, ref):
    """The oracle (numpy FP64) running MALA on the same workload for a bounded sample, on
    this host's cores; plus the oracle's own min-ESS/s from its long runs of the workload
    (256 chains x 5000 steps, stored with the host they ran on)."""
    import numpy as np
    from oracle import samplers as OS

    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        cores = os.cpu_count() or 1
    model, nproc = host_info()
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
    out = dict(value=done * n / el, unit="emulator logL+grad evals/s", cores=int(cores),
               kind="oracle",
               sample=f"oracle MALA, {n} chains x {done} steps of the c2 workload "
                      f"(FP64 numpy, {el:.1f} s; cores = BLAS threads)",
               cpu_model=model, nproc=nproc)
    if ref is not None:
        r = ref["runs"][0]
        out["oracle_min_ess_per_s"] = dict(
            value=r["min_ess_per_s"], min_ess=r["min_ess"],
            production_s=r["production_wall_s"], accept=r["accept"],
            sample=f"oracle MALA, {ref['n_chains']} chains, {ref['warmup']} warm-up + "
                   f"{ref['production']} production steps",
            host=ref["host"], source="tests/golden/c2_posterior_oracle.json")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=10)
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
    ref = oracle_reference(args.config)
    results = {}
    for prec in precs:
        results[prec] = {}
        for s in samplers:
            r = run_chain(B, torch, prob, prec, s, args.chains, args.warmup, args.steps,
                          args.seed, args.n_leapfrog, ref)
            results[prec][s] = r
            mes = r["min_ess_per_s"]
            print(f"# {prec} {s}: {r['evals_per_s']:.3e} evals/s, min-ESS/s "
                  f"{'null (' + r['min_ess_null_reason'] + ')' if mes is None else f'{mes:.3e}'}, "
                  f"accept {r['accept']:.3f}, eps {r['eps']:.3g}, timed {r['wall_s']:.2f}s, "
                  f"posterior vs oracle {r['posterior_vs_oracle']}",
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
        def ratio(a, b):
            return None if a is None or b is None else a / b
        line["speedup_vs_" + precs[1]] = {
            s: dict(min_ess_per_s=ratio(results[head][s]["min_ess_per_s"],
                                        results[precs[1]][s]["min_ess_per_s"]),
                    evals_per_s=results[head][s]["evals_per_s"] / results[precs[1]][s]["evals_per_s"])
            for s in samplers}
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(prob, args.chains, args.cpu_budget, args.seed, ref)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

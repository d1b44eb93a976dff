"""Write tests/golden/c2_posterior_oracle.json: the FP64 oracle's posterior summary of the
C2 workload with the emulator term on, from two independent long oracle runs.

Test infrastructure: calls only the oracle and the seeded input generator.  Each run is the
C2 recipe at the oracle's size: 256 chains started uniformly in the prior box, 1000 MALA
warm-up steps (windows doubling from 10 steps, each followed by a covariance / mean update
from its second half; dual averaging of the step size towards acceptance 0.57 inside every
window; a last step-size-only window), then 4000 production steps.  The two runs differ in
their Philox seed only.  Stored per run: the posterior mean and covariance of x over the
production draws, the per-parameter multi-chain ESS (and its flags), the acceptance, the
final step size, and the production wall time on this host (with its CPU model and thread
count), which gives the oracle's own min-ESS/s.  Also stored: the noise floor between the
two runs, |mean_a - mean_b| / sd and the variance ratios, the run-to-run scatter that a
comparison against one of them inherits.

Usage:  python tests/golden/make_c2_posterior.py   (about 3 minutes on 8 cores)
"""
from __future__ import annotations

import json
import os
import platform
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import adapt as OA, ess as OE, samplers as OS  # noqa: E402
from workloads import make_problem  # noqa: E402

N_CHAINS, WARMUP, PRODUCTION = 256, 1000, 4000
TARGET = 0.57
SEEDS = (0xC2A0_0001, 0xC2A0_0002)
OUT = os.path.join(HERE, "c2_posterior_oracle.json")


def windows(warmup, first=10):
    """(length, update covariance) pairs: first, 2 first, ... then a step-size-only tail of
    a fifth of the warm-up."""
    tail = max(20, warmup // 5)
    body, plan, w, used = warmup - tail, [], first, 0
    while used + w <= body:
        plan.append((w, True))
        used += w
        w *= 2
    if body > used:
        plan.append((body - used, True))
    plan.append((tail, False))
    return plan


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        return os.cpu_count() or 1


def one_run(prob, seed):
    d = prob["d"]
    x0 = OS.init_uniform(prob, seed, N_CHAINS)
    W = dict(mu=0.5 * (prob["lower"] + prob["upper"]),
             L=np.diag(0.1 * (prob["upper"] - prob["lower"])))
    st = OS.init_state(prob, W, x0)
    t, eps = 0, 0.5
    for w, update in windows(WARMUP):
        da = OA.DualAveraging(eps, TARGET)
        xs = []
        for _ in range(w):
            st, info = OS.mala_step(prob, W, st, t, seed, da.eps)
            da.update(float(np.mean(info["accept_prob"])))
            xs.append(W["mu"][None, :] + st["z"] @ W["L"].T)
            t += 1
        eps = max(da.final, 1e-12)
        if update:
            keep = np.stack(xs[w // 2:] if w >= 4 else xs)
            mean, cov = OA.ensemble_moments(keep)
            L, _ = OA.regularised_cholesky(cov)
            W = dict(mu=mean, L=L)
            st = OS.init_state(prob, W, xs[-1])
    draws = np.empty((PRODUCTION, N_CHAINS, d))
    acc = 0.0
    t0 = time.perf_counter()
    for s in range(PRODUCTION):
        st, info = OS.mala_step(prob, W, st, t, seed, eps)
        draws[s] = W["mu"][None, :] + st["z"] @ W["L"].T
        acc += float(np.mean(info["accepted"]))
        t += 1
    wall = time.perf_counter() - t0
    m, per, flags = OE.min_ess(draws)
    flat = draws.reshape(-1, d)
    return dict(seed=seed, eps=eps, accept=acc / PRODUCTION, mean=flat.mean(0).tolist(),
                cov=np.cov(flat.T).tolist(), ess=per.tolist(), ess_flags=flags.tolist(),
                min_ess=m, production_wall_s=wall, min_ess_per_s=m / wall,
                evals_per_s=PRODUCTION * N_CHAINS / wall)


def main():
    prob = make_problem("c2")
    runs = []
    for seed in SEEDS:
        r = one_run(prob, seed)
        print(f"seed {seed:#x}: accept {r['accept']:.3f} eps {r['eps']:.3f} "
              f"min ESS {r['min_ess']:.0f} ({r['production_wall_s']:.0f} s)", flush=True)
        runs.append(r)
    a, b = (np.array(r["mean"]) for r in runs)
    ca, cb = (np.array(r["cov"]) for r in runs)
    sd = np.sqrt(np.diag(ca))
    out = dict(
        workload="c2: d=6 Gaussian(cond 1e3)+0.5*MLP 6->512x4->1 tanh, FP64 oracle MALA",
        n_chains=N_CHAINS, warmup=WARMUP, production=PRODUCTION, target_accept=TARGET,
        host=dict(cpu_model=cpu_model(), nproc=os.cpu_count(), blas_threads=blas_threads()),
        runs=runs,
        noise_floor=dict(mean_diff_over_sd=(np.abs(a - b) / sd).tolist(),
                         var_ratio=(np.diag(cb) / np.diag(ca)).tolist()),
        generator="tests/golden/make_c2_posterior.py")
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()

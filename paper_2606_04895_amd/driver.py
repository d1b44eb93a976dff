"""Host-side drivers over the C ABI: the burn-in schedule of Sec. 4 and the learned-emulator
pipeline.  Control flow only; every computation is a library call.

Burn-in (Sec. 3.2, Sec. 4, Sec. 4.3): the warm-up is split into windows that double in
length from a short first one (10 steps), or that end at 1/4, 1/2 and all of the warm-up.
Inside a window the step size follows dual averaging towards the sampler's target
acceptance; at its end the step size is set to the averaged iterate and the covariance and
mean are re-estimated from the second half of the window (best_adapt), then dual averaging
restarts from the new step size.  Short early windows let the whitening follow the
ensemble while it contracts from the prior box; a last step-size-only window tunes the
step under the final whitening.  AIES uses no whitening and no step
size, so its warm-up is a single plain run (Sec. 4: one long burn-in).
"""
from __future__ import annotations

import time

import numpy as np

from . import (best_adapt, best_ess, best_get_state, best_init, best_logL_grad, best_reinit,
               best_normalise_inputs, best_set_mlp, best_set_step_size, best_standardise,
               best_step, Trainer)

TARGET_ACCEPT = {"mala": 0.57, "hmc": 0.8, "nuts": 0.8}
# Dual averaging lowers the step size without bound while nothing is accepted (chains far in
# the tails of a sharply curved target); between windows it is kept at or above this floor
# so that a window never starts from a step size that has underflowed to zero.
EPS_FLOOR = 1e-12
EPS0 = {"mala": 0.5, "hmc": 0.3, "nuts": 0.5}


def window_plan(warmup, schedule="doubling", first=10):
    """Adaptation windows as (length, re-estimate covariance) pairs.
    "doubling": windows of first, 2 first, 4 first, ... steps with a covariance update after
    each, the last of them absorbing the remainder, then a final step-size-only window of a
    fifth of the warm-up (at least 20 steps) under the final whitening.
    "thirds": windows ending at 1/4, 1/2 and all of the warm-up, each followed by an update."""
    if warmup <= 0:
        return []
    if schedule == "thirds":
        ends = sorted(set([0, max(1, warmup // 4), max(1, warmup // 2), warmup]))
        return [(b - a, True) for a, b in zip(ends[:-1], ends[1:])]
    tail = max(20, warmup // 5) if warmup >= 4 * first else 0
    body = warmup - tail
    plan, w, used = [], first, 0
    while used + w < body:
        plan.append([w, True])
        used += w
        w *= 2
    if plan and body - used < w // 2:
        plan[-1][0] += body - used
    elif body - used > 0:
        plan.append([body - used, True])
    if tail:
        plan.append([tail, False])
    return [tuple(p) for p in plan]


# Default window schedule per sampler (measured on the c2 workload from a uniform start in
# the prior box): MALA and MH need the short early windows to follow the contracting
# ensemble; HMC reaches the typical set within the first window and tunes its step size
# better over the long windows.  NUTS needs the short early windows too: on the 27-parameter
# workload the thirds schedule left it at eps 0.08 and 49 leaves per transition with a
# whitening that was still off, the doubling schedule at eps 0.73, 7 leaves and ESS/draw 3.
SCHEDULE = {"mala": "doubling", "mh": "doubling", "hmc": "thirds", "nuts": "doubling"}


def burn_in(ctx, sampler, warmup, d, n, n_leap=10, mh_scale=None, stretch_a=2.0,
            schedule=None, max_depth=8, recenter=False, trajectory=None):
    """Burn-in with covariance windows (and dual averaging for the gradient samplers).

    recenter: after each covariance window, re-initialise the ensemble as Gaussian draws
    around its best-fit walker (largest log pi) with the new whitening, the burn-in loop of
    Sec. 4 in which the covariance and the best-fit point are updated together.
    trajectory: a list that receives every window's record ([w][d][n] device floats; for
    AIES and DE the whole burn-in run), the burn-in trajectories of the results object of
    Sec. 3.1."""
    import torch

    schedule = schedule or SCHEDULE.get(sampler, "doubling")

    kw = dict(n_leapfrog=n_leap, stretch_a=stretch_a, max_depth=max_depth,
              mh_scale=mh_scale if mh_scale else 2.4 / np.sqrt(d))
    t0 = time.perf_counter()
    if sampler in ("aies", "de"):
        if warmup:
            rec = torch.empty((warmup, d, n), dtype=torch.float32, device="cuda") \
                if trajectory is not None else None
            best_step(ctx, sampler, warmup, record=rec, **kw)
            if rec is not None:
                trajectory.append(rec)
        return time.perf_counter() - t0
    gradient = sampler in TARGET_ACCEPT
    if gradient:
        best_set_step_size(ctx, EPS0[sampler])
    for w, update_cov in window_plan(warmup, schedule):
        rec = torch.empty((w, d, n), dtype=torch.float32, device="cuda") \
            if (update_cov or trajectory is not None) else None
        if gradient:
            st = best_step(ctx, sampler, w, record=rec, adapt_eps=True,
                           target_accept=TARGET_ACCEPT[sampler], **kw)
        else:
            st = best_step(ctx, sampler, w, record=rec, **kw)
        if update_cov:
            keep = rec[w // 2:] if w >= 4 else rec
            info = best_adapt(ctx, samples=keep.contiguous(), update_mean=True,
                              finalize_da=gradient, reset_da=gradient,
                              target_accept=TARGET_ACCEPT.get(sampler, 0.0))
            if gradient and not info["eps"] >= EPS_FLOOR:
                best_set_step_size(ctx, EPS_FLOOR)
            if recenter:
                x, lp, _ = best_get_state(ctx)
                best_reinit(ctx, "gaussian", x[:, int(np.argmax(lp))], 1.0)
        elif gradient:
            # step size only: the averaged iterate, dual averaging restarted from it
            best_set_step_size(ctx, max(st["eps_bar"], EPS_FLOOR))
        if trajectory is not None and rec is not None:
            trajectory.append(rec)
        del rec
    torch.cuda.synchronize()
    return time.perf_counter() - t0


_SUMMED = ("accepted", "evals", "n_nonfinite", "n_oob", "n_recorded", "sum_accept_prob", "ms")


def sample(ctx, sampler, steps, d, n, n_leap=10, mh_scale=None, stretch_a=2.0, ess=True,
           max_depth=8, chunk=None, record=True):
    """Timed production run with every step recorded; returns (stats, record, wall_s, ess).
    chunk: launch at most this many steps per best_step call (the record continues across
    calls and the Philox step counter makes the chains identical to one long call); the
    count fields and the kernel time `ms` of the returned stats are summed over the calls."""
    import torch

    kw = dict(n_leapfrog=n_leap, stretch_a=stretch_a, max_depth=max_depth,
              mh_scale=mh_scale if mh_scale else 2.4 / np.sqrt(d))
    rec = torch.empty((steps, d, n), dtype=torch.float32, device="cuda") if record else None
    chunk = steps if not chunk else int(chunk)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = None
    for s0 in range(0, steps, chunk):
        k = min(chunk, steps - s0)
        r = best_step(ctx, sampler, k, record=rec[s0:s0 + k] if rec is not None else None, **kw)
        if st is None:
            st = r
        else:
            for f in _SUMMED:
                st[f] += r[f]
            st["eps"], st["eps_bar"] = r["eps"], r["eps_bar"]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    e = best_ess(ctx, rec) if (ess and rec is not None) else None
    return st, rec, wall, e


def train_emulator(prob, n_train, epochs, batch=1024, precision="fp32", seed=0,
                   lr0=1e-3, lr1=1e-5, plain_precision="fp32"):
    """Latin-hypercube design in the training box -> plain log L on the device ->
    standardised targets -> minibatch Adam.  Returns a dict with the trained flat parameter
    vector, the target scale (mean, std) and the per-epoch losses."""
    import torch
    from workloads import latin_hypercube, minibatch_permutations, xavier_mlp

    rng = np.random.default_rng(seed)
    d, w, nh = prob["d"], prob["width"], prob["n_hidden"]
    t0 = time.perf_counter()
    u = latin_hypercube(rng, n_train, d)
    x = prob["train_lo"] + u * (prob["train_hi"] - prob["train_lo"])
    plain = dict(prob, plain_mode=2)
    ctx = best_init(plain, n_chains=16, precision=plain_precision, seed=seed)
    xt = torch.tensor(x.T.copy(), device="cuda")
    ll, _ = best_logL_grad(ctx, xt, want_grad=False)
    y, mu, sig = best_standardise(ll)
    th = best_normalise_inputs(xt, prob["in_center"], prob["in_invscale"])
    t_data = time.perf_counter() - t0
    tr = Trainer(d, w, nh, xavier_mlp(rng, d, w, nh), precision=precision)
    perms = minibatch_permutations(rng, n_train, epochs)
    nb = n_train // batch
    losses = []
    t1 = time.perf_counter()
    for e in range(epochs):
        pe = torch.tensor(perms[e], device="cuda")
        losses.append(tr.epoch(th, y, pe, batch, lr0, lr1, e * nb, epochs * nb))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    out = dict(params=tr.params(), y_mu=mu, y_sigma=sig, losses=losses, data_s=t_data,
               train_s=t_train, n_train=n_train, epochs=epochs)
    tr.close()
    ctx.close()
    return out


def emulator_problem(prob, trained):
    """The sampling target built on the trained emulator: y_mu + y_sigma * MLP inside the
    training box, the plain likelihood outside it."""
    return dict(prob, plain_mode=1, mlp_params=trained["params"], mlp_coef=trained["y_sigma"],
                offset=trained["y_mu"])

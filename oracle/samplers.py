"""Sampler transitions, vectorised over chains, in float64.

All gradient-based samplers and MH work in the whitened space of Sec. 2.2 (Algorithm 1):
the state of chain c is (z_c, lp_c = log pi_z(z_c), g_c = grad_z log pi_z(z_c)), the
whitening W = (mu, L) is fixed during a transition.  AIES works in the original space
(Sec. 2.2 footnote: an affine transform does not change it).

Randomness comes from the Philox counter layout in `philox` (step t is counter word c1).
Accept rule everywhere: accept iff log u < log alpha, with u strictly inside (0, 1);
a NaN log alpha never accepts.

MH    (Sec. 1, Sec. 2.1):  z' = z + s xi,  log alpha = lp(z') - lp(z)
MALA  (Sec. 2.1, the discretised Langevin proposal):
      z' = z + eps g(z) + sqrt(2 eps) xi,   proposal N(z + eps g(z), 2 eps I);
      log alpha = lp(z') - lp(z) + log q(z | z') - log q(z' | z),
      log q(a | b) = -|a - b - eps g(b)|^2 / (4 eps)
      Per-dimension step multipliers (Sec. 4.3, larger steps for chosen whitened
      dimensions): eps_i = eps m_i in the drift, the noise and q; MH scales xi_i by m_i.
HMC   (Sec. 2.1 eq. hamiltonian with the identity mass of Sec. 2.2):
      q ~ N(0, I);  H = -lp(z) + |q|^2 / 2;  n_leap kick-drift-kick leapfrog steps;
      log alpha = H(start) - H(end).  Intermediate points use the unbounded density; only
      the end point is tested against the prior box.
AIES  (Sec. 2.3, stretch move):  the ensemble is split in halves S0 = [0, N/2), S1;
      each walker k of the active half takes a partner j uniform in the other half and
      z = ((a-1) u + 1)^2 / a;  y = x_j + z (x_k - x_j);
      log alpha = (d - 1) ln z + lp(y) - lp(x_k)   (Goodman & Weare 2010);
      S0 moves first against S1, then S1 against the updated S0.
DE    (Sec. 2.3, differential-evolution move of the ensemble sampler): with the same two
      half-ensembles, walker i takes two distinct partners j != k of the other half and
      y = x_i + gamma (x_j - x_k),  gamma = (1 + eta) 2.38 / sqrt(2 d),  eta ~ N(0, s^2);
      the proposal is symmetric (the pair (k, j) with the same gamma reverses it), so
      log alpha = lp(y) - lp(x_i).  Philox stream 7, sub = half: block 0 gives the
      partner uniforms (j from the first, k from the second among the other half's
      walkers except j), block 1 the normal for eta (first member).
"""
from __future__ import annotations

import numpy as np

from . import philox as ph
from .target import hard_box, whitened, log_target


def _accept(log_alpha, log_u):
    with np.errstate(invalid="ignore"):
        acc = log_u < log_alpha
        prob = np.where(np.isnan(log_alpha), 0.0, np.exp(np.minimum(0.0, log_alpha)))
    return acc, prob


def _chains(n, chains):
    return np.arange(n, dtype=np.uint64) if chains is None else np.asarray(chains, dtype=np.uint64)


def mh_step(prob, W, st, t, seed, scale, chains=None, params=None, mult=None):
    """mult: optional per-dimension step multipliers m (d,): z' = z + scale m xi."""
    z, lp = st["z"], st["lp"]
    n, d = z.shape
    ids = _chains(n, chains)
    xi = ph.normals(seed, ids, t, ph.STREAM_NORMAL, 0, d)
    zp = z + scale * xi if mult is None else z + (scale * np.asarray(mult))[None, :] * xi
    lpp, gp, _ = whitened(prob, W["mu"], W["L"], zp, params)
    log_alpha = lpp - lp
    log_u = np.log(ph.accept_uniform(seed, ids, t))
    acc, aprob = _accept(log_alpha, log_u)
    new = dict(z=np.where(acc[:, None], zp, z), lp=np.where(acc, lpp, lp),
               g=np.where(acc[:, None], gp, st["g"]) if "g" in st else gp)
    return new, dict(accepted=acc, log_alpha=log_alpha, log_u=log_u, accept_prob=aprob,
                     proposal=zp)


def mala_step(prob, W, st, t, seed, eps, chains=None, params=None, mult=None):
    """mult: optional per-dimension step multipliers m (d,): dimension i uses the step
    eps m_i in the drift, the noise sqrt(2 eps m_i) and its proposal density."""
    z, lp, g = st["z"], st["lp"], st["g"]
    n, d = z.shape
    ids = _chains(n, chains)
    xi = ph.normals(seed, ids, t, ph.STREAM_NORMAL, 0, d)
    if mult is not None:
        e = eps * np.asarray(mult, dtype=np.float64)[None, :]
        zp = z + e * g + np.sqrt(2.0 * e) * xi
        lpp, gp, _ = whitened(prob, W["mu"], W["L"], zp, params)
        with np.errstate(invalid="ignore"):
            log_q_rev = -np.sum((z - zp - e * gp) ** 2 / (4.0 * e), axis=1)
            log_q_fwd = -np.sum((zp - z - e * g) ** 2 / (4.0 * e), axis=1)
            log_alpha = lpp - lp + log_q_rev - log_q_fwd
        log_u = np.log(ph.accept_uniform(seed, ids, t))
        acc, aprob = _accept(log_alpha, log_u)
        new = dict(z=np.where(acc[:, None], zp, z), lp=np.where(acc, lpp, lp),
                   g=np.where(acc[:, None], gp, g))
        return new, dict(accepted=acc, log_alpha=log_alpha, log_u=log_u, accept_prob=aprob,
                         proposal=zp)
    zp = z + eps * g + np.sqrt(2.0 * eps) * xi
    lpp, gp, _ = whitened(prob, W["mu"], W["L"], zp, params)
    with np.errstate(invalid="ignore"):
        log_q_rev = -np.sum((z - zp - eps * gp) ** 2, axis=1) / (4.0 * eps)
        log_q_fwd = -np.sum((zp - z - eps * g) ** 2, axis=1) / (4.0 * eps)
        log_alpha = lpp - lp + log_q_rev - log_q_fwd
    log_u = np.log(ph.accept_uniform(seed, ids, t))
    acc, aprob = _accept(log_alpha, log_u)
    new = dict(z=np.where(acc[:, None], zp, z), lp=np.where(acc, lpp, lp),
               g=np.where(acc[:, None], gp, g))
    return new, dict(accepted=acc, log_alpha=log_alpha, log_u=log_u, accept_prob=aprob,
                     proposal=zp)


def leapfrog(prob, W, z, q, g, eps, n_leap, params=None):
    """n_leap kick-drift-kick steps on H = -lp_z(z) + |q|^2/2 with the unbounded density.
    Returns (z, q, lp, g) at the end point (lp unbounded)."""
    lp = None
    for _ in range(n_leap):
        q = q + 0.5 * eps * g
        z = z + eps * q
        lp, g, _ = whitened(prob, W["mu"], W["L"], z, params, with_box=False)
        q = q + 0.5 * eps * g
    return z, q, lp, g


def hmc_step(prob, W, st, t, seed, eps, n_leap, chains=None, params=None):
    z0, lp0, g0 = st["z"], st["lp"], st["g"]
    n, d = z0.shape
    ids = _chains(n, chains)
    q0 = ph.normals(seed, ids, t, ph.STREAM_NORMAL, 0, d)
    h0 = -lp0 + 0.5 * np.sum(q0 * q0, axis=1)
    z1, q1, lp1, g1 = leapfrog(prob, W, z0, q0, g0, eps, n_leap, params)
    x1 = W["mu"][None, :] + z1 @ W["L"].T
    inside = np.all((x1 >= prob["lower"]) & (x1 <= prob["upper"]), axis=1)
    if hard_box(prob):
        lp1 = np.where(inside, lp1, -np.inf)
    h1 = -lp1 + 0.5 * np.sum(q1 * q1, axis=1)
    with np.errstate(invalid="ignore"):
        log_alpha = h0 - h1
    log_u = np.log(ph.accept_uniform(seed, ids, t))
    acc, aprob = _accept(log_alpha, log_u)
    new = dict(z=np.where(acc[:, None], z1, z0), lp=np.where(acc, lp1, lp0),
               g=np.where(acc[:, None], g1, g0))
    return new, dict(accepted=acc, log_alpha=log_alpha, log_u=log_u, accept_prob=aprob,
                     proposal=z1, momentum=q0, h0=h0, h1=h1)


def stretch_z(u, a):
    """Inverse CDF of g(z) proportional to 1/sqrt(z) on [1/a, a] (Sec. 2.3)."""
    return ((a - 1.0) * u + 1.0) ** 2 / a


def aies_step(prob, st, t, seed, a=2.0, params=None):
    """One full AIES iteration (both halves).  st = dict(x (N, d), lp (N,))."""
    x, lp = st["x"].copy(), st["lp"].copy()
    n, d = x.shape
    if n % 2:
        raise ValueError("AIES needs an even number of walkers")
    half = n // 2
    info = dict(accepted=np.zeros(n, bool), log_alpha=np.zeros(n), log_u=np.zeros(n),
                accept_prob=np.zeros(n), partner=np.zeros(n, np.int64), z=np.zeros(n))
    for h in (0, 1):
        act = np.arange(h * half, (h + 1) * half)
        comp0 = (1 - h) * half
        ua, ub = ph.uniforms2(seed, act.astype(np.uint64), t, ph.STREAM_AIES, h, 0)
        j = comp0 + np.minimum(np.floor(ua * half).astype(np.int64), half - 1)
        zz = stretch_z(ub, a)
        y = x[j] + zz[:, None] * (x[act] - x[j])
        lpy, _ = log_target(prob, y, params)
        with np.errstate(invalid="ignore"):
            log_alpha = (d - 1) * np.log(zz) + lpy - lp[act]
        log_u = np.log(ph.accept_uniform(seed, act.astype(np.uint64), t, sub=h))
        acc, aprob = _accept(log_alpha, log_u)
        x[act] = np.where(acc[:, None], y, x[act])
        lp[act] = np.where(acc, lpy, lp[act])
        info["accepted"][act] = acc
        info["log_alpha"][act] = log_alpha
        info["log_u"][act] = log_u
        info["accept_prob"][act] = aprob
        info["partner"][act] = j
        info["z"][act] = zz
    return dict(x=x, lp=lp), info


STREAM_DE = 7
DE_GAMMA0 = 2.38


def de_step(prob, st, t, seed, sigma_gamma, params=None):
    """One differential-evolution iteration of the ensemble (both halves, Sec. 2.3).
    st = dict(x (N, d), lp (N,)); needs N even and N >= 4."""
    x, lp = st["x"].copy(), st["lp"].copy()
    n, d = x.shape
    if n % 2 or n < 4:
        raise ValueError("the DE move needs an even number of walkers >= 4")
    half = n // 2
    info = dict(accepted=np.zeros(n, bool), log_alpha=np.zeros(n), log_u=np.zeros(n),
                accept_prob=np.zeros(n), partners=np.zeros((n, 2), np.int64),
                gamma=np.zeros(n))
    g0 = DE_GAMMA0 / np.sqrt(2.0 * d)
    for h in (0, 1):
        act = np.arange(h * half, (h + 1) * half)
        comp0 = (1 - h) * half
        ua, ub = ph.uniforms2(seed, act.astype(np.uint64), t, STREAM_DE, h, 0)
        jj = np.minimum(np.floor(ua * half).astype(np.int64), half - 1)
        kk = np.minimum(np.floor(ub * (half - 1)).astype(np.int64), half - 2)
        kk = np.where(kk >= jj, kk + 1, kk)
        eta = sigma_gamma * ph.normals(seed, act.astype(np.uint64), t, STREAM_DE, h, 3)[:, 2]
        gamma = (1.0 + eta) * g0
        y = x[act] + gamma[:, None] * (x[comp0 + jj] - x[comp0 + kk])
        lpy, _ = log_target(prob, y, params)
        log_alpha = lpy - lp[act]
        log_u = np.log(ph.accept_uniform(seed, act.astype(np.uint64), t, sub=h))
        acc, aprob = _accept(log_alpha, log_u)
        x[act] = np.where(acc[:, None], y, x[act])
        lp[act] = np.where(acc, lpy, lp[act])
        info["accepted"][act] = acc
        info["log_alpha"][act] = log_alpha
        info["log_u"][act] = log_u
        info["accept_prob"][act] = aprob
        info["partners"][act] = np.stack([comp0 + jj, comp0 + kk], axis=1)
        info["gamma"][act] = gamma
    return dict(x=x, lp=lp), info


def init_state(prob, W, x, params=None):
    """Whitened state from positions x (n, d): z = L^{-1}(x - mu)."""
    z = np.linalg.solve(W["L"], (np.atleast_2d(x) - W["mu"][None, :]).T).T
    lp, g, _ = whitened(prob, W["mu"], W["L"], z, params)
    return dict(z=z, lp=lp, g=g)


def init_uniform(prob, seed, n):
    u = ph.init_uniforms(seed, np.arange(n, dtype=np.uint64), prob["d"])
    return prob["lower"][None, :] + (prob["upper"] - prob["lower"])[None, :] * u


def run(prob, W, sampler, st, seed, t0, n_steps, eps=None, scale=None, n_leap=10,
        a=2.0, params=None):
    """Run n_steps transitions, return (state, samples in x-space (n_steps, N, d), acc)."""
    samples, accs = [], []
    for t in range(t0, t0 + n_steps):
        if sampler == "mh":
            st, info = mh_step(prob, W, st, t, seed, scale, params=params)
        elif sampler == "mala":
            st, info = mala_step(prob, W, st, t, seed, eps, params=params)
        elif sampler == "hmc":
            st, info = hmc_step(prob, W, st, t, seed, eps, n_leap, params=params)
        elif sampler == "aies":
            st, info = aies_step(prob, st, t, seed, a, params=params)
        else:
            raise ValueError(sampler)
        if sampler == "aies":
            samples.append(st["x"].copy())
        else:
            samples.append(W["mu"][None, :] + st["z"] @ W["L"].T)
        accs.append(info["accept_prob"])
    return st, np.stack(samples), np.stack(accs)

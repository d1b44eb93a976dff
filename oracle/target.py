"""Target log-densities, their gradients, and the whitened density of Sec. 2.2, in float64.

log pi(x) for the declarative targets sampled here:

  inside the prior box [lower, upper] (Sec. 3.1 bounds; a hard box, i.e. a uniform prior):
      gauss_coef * G(phi(x))  +  part(x)  + offset
  outside: -inf (the gradient returned there is that of the unbounded expression)
  or, with box_penalty = 1, the smooth penalty of Sec. 3.1 instead of -inf:
      - sum_i [exp(r_i / w) - 1 - r_i / w],  r_i = (distance of x_i outside [l_i, u_i]) /
      (u_i - l_i), w = penalty_width: zero with zero slope at the faces (the density stays
      differentiable) and growing exponentially outside.

  G(y)    = -1/2 (y - m)^T P (y - m)                      (Gaussian part, precision P)
  phi(x)  = x except phi_v = x_v + beta((x_u - c)^2 - kappa) (twisted "banana" pair, unit
            Jacobian, Haario, Saksman & Tamminen 1999)
  part(x) = mlp_coef * MLP(theta_hat),  theta_hat = (x - in_center) * in_invscale
            (plain_mode 0);  the same inside the emulator's training box and the plain
            spectrum log-likelihood outside it (plain_mode 1);  plain everywhere (mode 2)

Whitened density (Sec. 2.2, eq. log_prob_transform and Algorithm 1):
  x = mu + L z,   log pi_z(z) = log pi(mu + L z) + sum_i log L_ii,   grad_z = L^T grad_x.
"""
from __future__ import annotations

import numpy as np

from . import mlp as _mlp


def normalise(prob, x):
    return (np.asarray(x) - prob["in_center"]) * prob["in_invscale"]


def in_box(lo, hi, x):
    x = np.asarray(x)
    return np.all((x >= lo) & (x <= hi), axis=-1)


def gauss_part(prob, x):
    """G(phi(x)) and its gradient with respect to x."""
    x = np.asarray(x, dtype=np.float64)
    y = x.copy()
    tw = prob.get("twist")
    if tw is not None:
        du = x[:, tw["u"]] - tw["center"]
        y[:, tw["v"]] = x[:, tw["v"]] + tw["beta"] * (du * du - tw["kappa"])
    r = y - prob["gauss_mean"]
    pr = r @ prob["gauss_prec"].T
    val = -0.5 * np.einsum("ni,ni->n", r, pr)
    gy = -pr  # d G / d y  (P symmetric)
    gx = gy.copy()
    if tw is not None:
        # Jacobian of phi: d y_v / d x_u = 2 beta (x_u - c); chain rule adds to grad_u
        gx[:, tw["u"]] += gy[:, tw["v"]] * 2.0 * tw["beta"] * du
    return val, gx


def plain_logL(plain, theta):
    """Spectrum model: S_j = sum_m A_m exp(-gam_m x_j) cos(2 pi k_m x_j + phi_m) with
    A_m = exp(a_m . t), gam_m = gamma0_m exp(g_m . t), phi_m = pi tanh(p_m . t),
    t = (theta - center) * invscale;  logL = -1/2 sum_j (S_j - data_j)^2 / sigma_j^2.
    Returns (logL (n,), grad (n, d)) with the analytic gradient."""
    theta = np.atleast_2d(np.asarray(theta, dtype=np.float64))
    n, d = theta.shape
    xg, data, w2 = plain["xgrid"], plain["data"], plain["inv_sigma2"]
    a, g, p, k, g0 = plain["a"], plain["g"], plain["p"], plain["k"], plain["gamma0"]
    val = np.empty(n)
    grad = np.empty((n, d))
    chunk = 256
    for s in range(0, n, chunk):
        t = (theta[s:s + chunk] - plain["center"]) * plain["invscale"]
        amp = np.exp(t @ a.T)                        # (c, M)
        gam = g0[None, :] * np.exp(t @ g.T)          # (c, M)
        th = np.tanh(t @ p.T)
        phs = np.pi * th
        e = np.exp(-gam[:, :, None] * xg[None, None, :])                  # (c, M, J)
        arg = 2.0 * np.pi * k[None, :, None] * xg[None, None, :] + phs[:, :, None]
        co, si = np.cos(arg), np.sin(arg)
        spec = np.einsum("cm,cmj->cj", amp, e * co)
        r = (spec - data[None, :]) * w2[None, :]
        val[s:s + chunk] = -0.5 * np.einsum("cj,cj->c", spec - data[None, :], r)
        s_ec = np.einsum("cj,cmj->cm", r, e * co)
        s_xec = np.einsum("cj,cmj->cm", r * xg[None, :], e * co)
        s_es = np.einsum("cj,cmj->cm", r, e * si)
        # d spec_j / d t = sum_m [E C dA - x E C A dgam - A E S dphi]
        coef_a = s_ec * amp                           # multiplies a_m
        coef_g = -s_xec * amp * gam                   # multiplies g_m
        coef_p = -s_es * amp * np.pi * (1.0 - th * th)  # multiplies p_m
        dt = coef_a @ a + coef_g @ g + coef_p @ p     # d(sum r S)/dt
        grad[s:s + chunk] = -dt * plain["invscale"]
    return val, grad


def mlp_part(prob, x, params=None):
    p = prob["mlp_params"] if params is None else params
    th = normalise(prob, x)
    out, gth = _mlp.value_and_input_grad(p, th, prob["d"], prob["width"], prob["n_hidden"])
    return prob["mlp_coef"] * out, prob["mlp_coef"] * gth * prob["in_invscale"]


def hard_box(prob):
    """True when the prior box is hard (-inf outside), False with the smooth penalty."""
    return not prob.get("box_penalty", 0)


def box_penalty(prob, x):
    """The smooth boundary penalty P(x) >= 0 and its gradient (n, d)."""
    lo, hi = prob["lower"], prob["upper"]
    width = hi - lo
    w = float(prob.get("penalty_width", 0.01))
    over = np.maximum(x - hi, 0.0) / width
    under = np.maximum(lo - x, 0.0) / width
    r = over + under
    p = np.sum(np.expm1(r / w) - r / w, axis=1)
    dr = np.where(over > 0, 1.0, np.where(under > 0, -1.0, 0.0)) / width
    return p, (np.expm1(r / w) / w) * dr


def log_target(prob, x, params=None, with_box=True):
    """log pi(x) and grad_x log pi(x) for a batch x (n, d)."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    n, d = x.shape
    lp = np.full(n, float(prob.get("offset", 0.0)))
    g = np.zeros((n, d))
    if prob["gauss_coef"] != 0.0:
        gv, gg = gauss_part(prob, x)
        lp += prob["gauss_coef"] * gv
        g += prob["gauss_coef"] * gg
    mode = prob.get("plain_mode", 0)
    if mode == 0:
        mv, mg = mlp_part(prob, x, params)
        lp += mv
        g += mg
    else:
        if mode == 1:
            inside = in_box(prob["train_lo"], prob["train_hi"], x)
        else:
            inside = np.zeros(n, dtype=bool)
        if inside.any():
            mv, mg = mlp_part(prob, x[inside], params)
            lp[inside] += mv
            g[inside] += mg
        if (~inside).any():
            pv, pg = plain_logL(prob["plain"], x[~inside])
            lp[~inside] += pv
            g[~inside] += pg
    if not hard_box(prob):
        pv, pg = box_penalty(prob, x)
        lp -= pv
        g -= pg
    elif with_box:
        lp = np.where(in_box(prob["lower"], prob["upper"], x), lp, -np.inf)
    return lp, g


def whitened(prob, mu, L, z, params=None, with_box=True):
    """Algorithm 1: x = mu + L z;  log pi_z = log pi(x) + sum log diag L;  grad_z = L^T grad_x."""
    z = np.atleast_2d(z)
    x = mu[None, :] + z @ L.T
    lp, gx = log_target(prob, x, params, with_box)
    return lp + np.sum(np.log(np.diag(L))), gx @ L, x

"""Emulator training, importance weights and Kish ESS, in float64.

Not in the paper itself (its emulators come from the CLiENT framework it cites); this is the
learned part of the method here: an MLP is fitted to (theta, logL) pairs that the plain spectrum
model produces, then used as the sampling target, and the plain likelihood assesses it.

  standardise     y_hat = (y - y_mu) / y_sigma (population std);  emulator logL = y_mu + y_sigma MLP
  loss            mean over the minibatch of (MLP(theta_hat_c) - y_hat_c)^2
  gradient        upstream d loss / d out_c = 2 (out_c - y_hat_c) / B, back-propagated
  Adam            Kingma & Ba (2015): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
                  p -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps),
                  b1 = 0.9, b2 = 0.999, eps = 1e-8
  minibatches     epoch e uses the permutation perm[e]; batch i is perm[e][iB:(i+1)B],
                  the ragged tail of an epoch is dropped
  learning rate   cosine decay from lr0 to lr1 over the total number of Adam steps
  weights         log w_i = logL_plain(x_i) - logL_emu(x_i), normalised by log-sum-exp;
                  Kish ESS = (sum w)^2 / sum w^2
"""
from __future__ import annotations

import numpy as np

from . import mlp as _mlp


def standardise(y):
    y = np.asarray(y, dtype=np.float64)
    mu, sig = float(y.mean()), float(y.std())
    return (y - mu) / sig, mu, sig


def mse_loss_grad(params, th, y_hat, d, width, n_hidden):
    out, _ = _mlp.forward(params, th, d, width, n_hidden)
    r = out - y_hat
    up = 2.0 * r / r.shape[0]
    g, _ = _mlp.param_grad(params, th, up, d, width, n_hidden)
    return float(np.mean(r * r)), g


class Adam:
    def __init__(self, n, b1=0.9, b2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.b1, self.b2, self.eps = b1, b2, eps

    def step(self, params, grad, lr):
        self.t += 1
        self.m = self.b1 * self.m + (1.0 - self.b1) * grad
        self.v = self.b2 * self.v + (1.0 - self.b2) * grad * grad
        mh = self.m / (1.0 - self.b1 ** self.t)
        vh = self.v / (1.0 - self.b2 ** self.t)
        return params - lr * mh / (np.sqrt(vh) + self.eps)


def cosine_lr(step, total, lr0, lr1):
    return lr1 + 0.5 * (lr0 - lr1) * (1.0 + np.cos(np.pi * step / max(total, 1)))


def train(params, th, y_hat, perms, batch, lr0, lr1, d, width, n_hidden):
    """Minibatch Adam over the given epoch permutations; returns (params, losses)."""
    n = th.shape[0]
    nb = n // batch
    total = nb * len(perms)
    opt = Adam(params.size)
    losses = []
    step = 0
    for perm in perms:
        for i in range(nb):
            idx = perm[i * batch:(i + 1) * batch]
            loss, g = mse_loss_grad(params, th[idx], y_hat[idx], d, width, n_hidden)
            params = opt.step(params, g, cosine_lr(step, total, lr0, lr1))
            losses.append(loss)
            step += 1
    return params, np.array(losses)


def importance_weights(logl_plain, logl_emu):
    lw = np.asarray(logl_plain, dtype=np.float64) - np.asarray(logl_emu, dtype=np.float64)
    w = np.exp(lw - np.max(lw))
    return w / w.sum()


def kish_ess(w):
    w = np.asarray(w, dtype=np.float64)
    return float(w.sum() ** 2 / np.sum(w * w))

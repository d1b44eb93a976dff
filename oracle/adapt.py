"""Covariance adaptation and step-size adaptation (Sec. 3.2, Sec. 4, Sec. 4.3), float64.

Sec. 3.2: after each burn-in iteration the empirical covariance of the walker ensemble is
computed, regularised through a Cholesky factorisation that enforces positive
definiteness, and used for the whitening transform of Algorithm 1.

Readings used here (the paper gives no formulas for these):
  * moments are pooled over every chain and every retained step of the window; the
    covariance uses the unbiased 1/(n-1) normalisation; the whitening mean is the
    ensemble mean;
  * regularisation: symmetrise, try Cholesky (a pivot must exceed 1e-12 * mean(diag S) to
    count as positive); on failure add lam * mean(diag S) * I with lam = 1e-10, 1e-9, ...,
    1e-2 and retry; if all fail the factorisation is reported as failed;
  * step size: dual averaging of Hoffman & Gelman (2014, Sec. 3.2) on the chain-averaged
    acceptance probability, gamma = 0.05, t0 = 10, kappa = 0.75, mu = log(10 eps0).
"""
from __future__ import annotations

import numpy as np


def ensemble_moments(samples):
    """samples: (..., d) pooled over all leading axes -> (mean (d,), cov (d, d))."""
    x = np.asarray(samples, dtype=np.float64).reshape(-1, np.shape(samples)[-1])
    n = x.shape[0]
    mean = x.mean(0)
    r = x - mean
    cov = r.T @ r / (n - 1)
    return mean, cov


PIVOT_FLOOR = 1e-12


def cholesky_lower(a, floor=0.0):
    """Plain Cholesky-Banachiewicz; returns L, or None if a pivot is not finite and above
    `floor` (numerical positive definiteness)."""
    a = np.asarray(a, dtype=np.float64)
    d = a.shape[0]
    L = np.zeros_like(a)
    for i in range(d):
        for j in range(i + 1):
            s = a[i, j] - np.dot(L[i, :j], L[j, :j])
            if i == j:
                if not (s > floor) or not np.isfinite(s):
                    return None
                L[i, i] = np.sqrt(s)
            else:
                L[i, j] = s / L[j, j]
    return L


def regularised_cholesky(cov):
    """Returns (L, jitter_used).  Raises np.linalg.LinAlgError if every jitter fails.
    A pivot counts as positive only above PIVOT_FLOOR * mean(diag S), so a rank-deficient
    covariance takes the jitter path whatever its rounding."""
    s = 0.5 * (np.asarray(cov) + np.asarray(cov).T)
    scale = float(np.mean(np.diag(s)))
    floor = PIVOT_FLOOR * scale if np.isfinite(scale) else 0.0
    L = cholesky_lower(s, floor)
    if L is not None:
        return L, 0.0
    lam = 1e-10
    while lam <= 1e-2 * (1 + 1e-12):
        L = cholesky_lower(s + lam * scale * np.eye(s.shape[0]), floor)
        if L is not None:
            return L, lam * scale
        lam *= 10.0
    raise np.linalg.LinAlgError("covariance is not positive definite after jitter")


class DualAveraging:
    """Hoffman & Gelman (2014) dual averaging of log step size towards a target
    acceptance delta."""

    def __init__(self, eps0, delta, gamma=0.05, t0=10.0, kappa=0.75):
        self.mu = np.log(10.0 * eps0)
        self.delta, self.gamma, self.t0, self.kappa = delta, gamma, t0, kappa
        self.h_bar = 0.0
        self.log_eps_bar = 0.0
        self.m = 0
        self.eps = eps0

    def update(self, accept_stat):
        self.m += 1
        m = self.m
        w = 1.0 / (m + self.t0)
        self.h_bar = (1.0 - w) * self.h_bar + w * (self.delta - accept_stat)
        log_eps = self.mu - np.sqrt(m) / self.gamma * self.h_bar
        eta = m ** (-self.kappa)
        self.log_eps_bar = eta * log_eps + (1.0 - eta) * self.log_eps_bar
        self.eps = float(np.exp(log_eps))
        return self.eps

    @property
    def final(self):
        return float(np.exp(self.log_eps_bar))

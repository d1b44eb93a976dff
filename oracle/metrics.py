"""Convergence metrics of the paper's Sec. 4.1 (Gelman-Rubin type R - 1, the credible metric,
the sliced Wasserstein distance), float64, plain definitions.  Test infrastructure only: the
library's HIP path never imports this module.

Samples come as the sampler record, shape (T, d, N): T draws of N chains (float32 on the
device; read here as float64).

R - 1 (Sec. 4.1, the multivariate statistic with diagonal normalisation):
    chain means m_c (d), chain covariances C_c (unbiased, 1/(T-1));
    B = covariance of the chain means (unbiased, 1/(N-1)),  W = mean over chains of C_c;
    D = diag(sqrt(B_ii)),  B~ = D^-1 B D^-1,  W~ = D^-1 W D^-1;
    R - 1 = max_i |lambda_i|,  lambda = eigenvalues of W~^-1 B~.

Credible metric (Sec. 4.1): for parameter i and level alpha,
    Delta_i = (|hi_i - hi0_i| + |lo_i - lo0_i|) / (hi0_i - lo0_i),   metric = max_i Delta_i,
where (lo, hi) are the equal-tailed limits, the sample quantiles at (1 - alpha)/2 and
(1 + alpha)/2 of all T N draws of parameter i, and (lo0, hi0) the reference limits.
Sample quantile at level p of n sorted values v: h = (n - 1) p, k = floor(h),
    q = v_k + (h - k)(v_{k+1} - v_k)    (v_{k+1} = v_k when k = n - 1).
With whitening (mu, L) the draws are first mapped to z = L^-1 (x - mu).

Sliced Wasserstein distance (Sec. 4.1): the mean over K fixed unit directions w_k of the
1-d Wasserstein-1 distance between the projections {w_k . x} of the two sample sets,
    W1(P, Q) = integral |F_P(t) - F_Q(t)| dt   (empirical CDFs),
evaluated on the merged sorted projections.  Directions: w_k = xi_k / |xi_k| with xi_k the
d normals of Philox counter (chain k, step 0, stream 6, sub 0).  Optional whitening as for
the credible metric.
"""
from __future__ import annotations

import numpy as np

from . import philox as ph

STREAM_PROJ = 6


def _draws(rec, mu=None, L=None):
    """(T, d, N) record -> (T*N, d) float64 draws, optionally whitened."""
    r = np.asarray(rec, dtype=np.float64)
    x = r.transpose(0, 2, 1).reshape(-1, r.shape[1])
    if mu is not None:
        x = np.linalg.solve(np.asarray(L, dtype=np.float64), (x - mu).T).T
    return x


def rhat_minus_one(rec):
    """Sec. 4.1, multivariate R - 1 with the diagonal normalisation of B."""
    r = np.asarray(rec, dtype=np.float64)
    T, d, N = r.shape
    chains = r.transpose(2, 0, 1)  # (N, T, d)
    means = chains.mean(axis=1)  # (N, d)
    covs = np.stack([np.cov(chains[c], rowvar=False, ddof=1).reshape(d, d) for c in range(N)])
    W = covs.mean(axis=0)
    B = np.cov(means, rowvar=False, ddof=1).reshape(d, d)
    dinv = 1.0 / np.sqrt(np.diag(B))
    Bt = B * np.outer(dinv, dinv)
    Wt = W * np.outer(dinv, dinv)
    lam = np.linalg.eigvals(np.linalg.solve(Wt, Bt))
    return float(np.max(np.abs(lam)))


def quantile(v, p):
    """Sample quantile at level p of the values v (the linear rule in the header)."""
    s = np.sort(np.asarray(v, dtype=np.float64))
    n = s.shape[0]
    h = (n - 1) * p
    k = int(np.floor(h))
    if k >= n - 1:
        return float(s[n - 1])
    return float(s[k] + (h - k) * (s[k + 1] - s[k]))


def credible_limits(rec, alpha, mu=None, L=None):
    """Equal-tailed limits (lo[d], hi[d]) at level alpha of every parameter."""
    x = _draws(rec, mu, L)
    a = (1.0 - alpha) / 2.0
    lo = np.array([quantile(x[:, i], a) for i in range(x.shape[1])])
    hi = np.array([quantile(x[:, i], 1.0 - a) for i in range(x.shape[1])])
    return lo, hi


def credible_metric(rec, alpha, lo0, hi0, mu=None, L=None):
    """Sec. 4.1 credible metric: max over parameters of the limit error / reference width."""
    lo, hi = credible_limits(rec, alpha, mu, L)
    delta = (np.abs(hi - hi0) + np.abs(lo - lo0)) / (hi0 - lo0)
    return float(np.max(delta)), lo, hi


def directions(d, k, seed):
    """The K fixed unit projection directions (k, d)."""
    xi = ph.normals(seed, np.arange(k, dtype=np.uint64), 0, STREAM_PROJ, 0, d)
    return xi / np.linalg.norm(xi, axis=1, keepdims=True)


def w1_1d(p, q):
    """Wasserstein-1 distance between the empirical distributions of p and q: the integral
    of |F_p - F_q| over the merged sorted support."""
    p = np.sort(np.asarray(p, dtype=np.float64))
    q = np.sort(np.asarray(q, dtype=np.float64))
    allv = np.sort(np.concatenate([p, q]))
    gaps = np.diff(allv)
    fp = np.searchsorted(p, allv[:-1], side="right") / p.shape[0]
    fq = np.searchsorted(q, allv[:-1], side="right") / q.shape[0]
    return float(np.sum(np.abs(fp - fq) * gaps))


def sliced_wasserstein(rec_a, rec_b, n_proj, seed, mu=None, L=None):
    """Sec. 4.1 sliced Wasserstein distance between two records (mean of K 1-d W1)."""
    xa = _draws(rec_a, mu, L)
    xb = _draws(rec_b, mu, L)
    w = directions(xa.shape[1], n_proj, seed)
    return float(np.mean([w1_1d(xa @ w[k], xb @ w[k]) for k in range(n_proj)]))

"""Multi-chain effective sample size (the throughput metric reported with the samplers; not in
the paper).

For one parameter with M chains of length T (x_{m,t}):
    chain means xbar_m, within-chain variance W = mean_m s_m^2 (1/(T-1)),
    B/T = variance of the chain means (1/(M-1)),  var+ = (T-1)/T W + B/T
    autocovariance gamma_{m,t} = (1/T) sum_{s<T-t} (x_{m,s}-xbar_m)(x_{m,s+t}-xbar_m)
    rho_0 = 1,  rho_t = 1 - (W - mean_m gamma_{m,t}) / var+    (t >= 1)
Geyer (1992) initial positive sequence on pair sums P_k = rho_{2k} + rho_{2k+1}: keep
k = 0, 1, ... while P_k > 0, then make the kept P_k non-increasing (initial monotone);
    tau = max(-1 + 2 sum_k P_k, 1 / log10(M T)),   ESS = M T / tau.
The floor on tau (as in Stan; Vehtari et al. 2021) bounds ESS by M T log10(M T) for
antithetic chains, where the truncated sum can fall below 1/2 and tau would go negative.
The autocovariances are computed here with numpy's FFT (zero-padded to avoid wrap-around).
"""
from __future__ import annotations

import numpy as np


def autocov_fft(x):
    """x (M, T) -> gamma (M, T) with 1/T normalisation, centred per chain."""
    x = np.asarray(x, dtype=np.float64)
    M, T = x.shape
    y = x - x.mean(1, keepdims=True)
    nfft = 1 << int(np.ceil(np.log2(2 * T)))
    f = np.fft.rfft(y, n=nfft, axis=1)
    ac = np.fft.irfft(f * np.conj(f), n=nfft, axis=1)[:, :T]
    return ac / T


def rho_hat(x):
    x = np.asarray(x, dtype=np.float64)
    M, T = x.shape
    means = x.mean(1)
    W = np.mean(x.var(1, ddof=1))
    b_over_t = means.var(ddof=1) if M > 1 else 0.0
    var_plus = (T - 1) / T * W + b_over_t
    gam = autocov_fft(x).mean(0)
    rho = 1.0 - (W - gam) / var_plus
    rho[0] = 1.0
    return rho


def geyer_tau(rho, n_draws):
    T = rho.shape[0]
    sums = []
    k = 0
    while 2 * k + 1 < T:
        p = rho[2 * k] + rho[2 * k + 1]
        if not p > 0.0:
            break
        sums.append(p)
        k += 1
    for i in range(1, len(sums)):
        sums[i] = min(sums[i], sums[i - 1])
    return max(-1.0 + 2.0 * float(np.sum(sums)), 1.0 / np.log10(n_draws))


def ess(x):
    """x (M, T) one parameter -> ESS."""
    M, T = np.shape(x)
    return M * T / geyer_tau(rho_hat(x), M * T)


def min_ess(samples):
    """samples (T, M, d) -> (min ESS over parameters, per-parameter ESS)."""
    s = np.asarray(samples)
    per = np.array([ess(s[:, :, i].T) for i in range(s.shape[2])])
    return float(per.min()), per

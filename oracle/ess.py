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

Two degenerate cases are reported instead of being turned into a number:
  * FROZEN: W = 0, every chain constant over the window (nothing was accepted, or the
    chains never left their start).  The autocorrelations are undefined (0/0 when the
    chains also share one value; rho_t = 1 at every lag otherwise), so there is no
    estimate: ESS = 0 with this flag.  "W = 0" is taken as W <= (1e-10 s)^2 with s the
    largest |chain mean|, so that the rounding of the chain means of constant FP64 chains
    (relative 1e-16 per step) does not count as movement; a float32 record that moves by one
    unit in the last place is far above it.
  * UNTRUNCATED: the pair sums stay positive up to the last lag the window allows, so the
    Geyer sequence was cut by the window length, not by the autocorrelation; tau is then
    a lower bound and the ESS an upper bound (a window shorter than the chains'
    autocorrelation time).  The value is returned with this flag.
The autocovariances are computed here with numpy's FFT (zero-padded to avoid wrap-around).
"""
from __future__ import annotations

import numpy as np

FLAG_OK = 0
FLAG_UNTRUNCATED = 1
FLAG_FROZEN = 2


def autocov_fft(x):
    """x (M, T) -> gamma (M, T) with 1/T normalisation, centred per chain."""
    x = np.asarray(x, dtype=np.float64)
    M, T = x.shape
    y = x - x.mean(1, keepdims=True)
    nfft = 1 << int(np.ceil(np.log2(2 * T)))
    f = np.fft.rfft(y, n=nfft, axis=1)
    ac = np.fft.irfft(f * np.conj(f), n=nfft, axis=1)[:, :T]
    return ac / T


def within_variance(x):
    """W = mean over chains of the unbiased within-chain variance."""
    return float(np.mean(np.var(np.asarray(x, dtype=np.float64), axis=1, ddof=1)))


def rho_hat(x):
    x = np.asarray(x, dtype=np.float64)
    M, T = x.shape
    means = x.mean(1)
    W = within_variance(x)
    b_over_t = means.var(ddof=1) if M > 1 else 0.0
    var_plus = (T - 1) / T * W + b_over_t
    gam = autocov_fft(x).mean(0)
    rho = 1.0 - (W - gam) / var_plus
    rho[0] = 1.0
    return rho


def geyer_tau(rho, n_draws):
    """(tau, truncated): truncated is False when every pair sum the window holds is
    positive (the sequence ran into the end of the window)."""
    T = rho.shape[0]
    sums = []
    k = 0
    truncated = False
    while 2 * k + 1 < T:
        p = rho[2 * k] + rho[2 * k + 1]
        if not p > 0.0:
            truncated = True
            break
        sums.append(p)
        k += 1
    for i in range(1, len(sums)):
        sums[i] = min(sums[i], sums[i - 1])
    tau = max(-1.0 + 2.0 * float(np.sum(sums)), 1.0 / np.log10(n_draws))
    return tau, truncated


FROZEN_REL = 1e-10


def is_frozen(x):
    """W <= (FROZEN_REL * max_m |xbar_m|)^2 (every chain constant up to rounding)."""
    x = np.asarray(x, dtype=np.float64)
    scale = float(np.max(np.abs(x.mean(1))))
    return not within_variance(x) > (FROZEN_REL * scale) ** 2


def ess_flagged(x):
    """x (M, T) one parameter -> (ESS, flag)."""
    M, T = np.shape(x)
    if is_frozen(x):
        return 0.0, FLAG_FROZEN
    tau, truncated = geyer_tau(rho_hat(x), M * T)
    return M * T / tau, (FLAG_OK if truncated else FLAG_UNTRUNCATED)


def ess(x):
    """x (M, T) one parameter -> ESS (0 for frozen chains; see ess_flagged)."""
    return ess_flagged(x)[0]


def min_ess(samples):
    """samples (T, M, d) -> (min ESS over parameters, per-parameter ESS, per-parameter
    flags)."""
    s = np.asarray(samples)
    res = [ess_flagged(s[:, :, i].T) for i in range(s.shape[2])]
    per = np.array([r[0] for r in res])
    flags = np.array([r[1] for r in res], dtype=np.int32)
    return float(per.min()), per, flags

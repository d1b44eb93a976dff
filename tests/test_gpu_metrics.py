"""GPU convergence metrics (Sec. 4.1) against the FP64 oracle (oracle/metrics.py) on the
same float32 records.

Tolerances: R - 1 to 1e-9 relative (FP64 sums of the same floats in another order, then
d x d algebra); credible limits to 1e-12 relative plus 1e-12 absolute (the same sorted
values and the same interpolation rule; whitening by forward substitution on the device,
by a general solve in the oracle); sliced Wasserstein to 1e-9 relative (FP64 projections in
another summation order, the same directions from the same Philox counters)."""
import numpy as np
import pytest
import torch

import paper_2606_04895_amd as B
from oracle import metrics as OM
from workloads import small_problem, walsh_chains

pytestmark = pytest.mark.gpu


def _ctx(d, n=16):
    prob = small_problem(d=d, width=128, n_hidden=2, seed=3)
    return B.best_init(prob, n_chains=n, precision="fp32", seed=1)


def _rec(rng, T, d, N, spread=0.3, corr=True):
    A = rng.normal(size=(d, d)) * 0.4 + np.eye(d) if corr else np.eye(d)
    z = rng.normal(size=(T, d, N))
    x = np.einsum("ij,tjn->tin", A, z) + spread * rng.normal(size=(1, d, N)) + 2.0
    return np.ascontiguousarray(x, dtype=np.float32)


@pytest.mark.parametrize("T,d,N", [(50, 3, 17), (300, 6, 64), (7, 27, 129), (2, 1, 2)])
def test_rhat_matches_oracle(T, d, N):
    rng = np.random.default_rng(T + d + N)
    rec = _rec(rng, T, d, N)
    ctx = _ctx(d)
    got = B.best_rhat(ctx, torch.tensor(rec, device="cuda"))
    ref = OM.rhat_minus_one(rec.astype(np.float64))
    assert got == pytest.approx(ref, rel=1e-9)


def test_rhat_sign_pattern_closed_form():
    deltas = [0.3, 1.7, 0.9]
    rec = walsh_chains(deltas, n_chains=16).astype(np.float32)
    ctx = _ctx(3)
    got = B.best_rhat(ctx, torch.tensor(rec, device="cuda"))
    n = rec.shape[2]
    assert got == pytest.approx(max(x * x for x in deltas) * n / (n - 1), rel=1e-6)


def test_rhat_rejects_identical_chain_means():
    rec = np.tile(np.random.default_rng(0).normal(size=(40, 2, 1)), (1, 1, 8)).astype(np.float32)
    ctx = _ctx(2)
    with pytest.raises(B.BestError) as e:
        B.best_rhat(ctx, torch.tensor(rec, device="cuda"))
    assert e.value.code == 1


@pytest.mark.parametrize("alpha", [0.68, 0.95])
@pytest.mark.parametrize("T,d,N,whiten", [(100, 4, 33, False), (100, 4, 33, True),
                                          (1, 5, 1, False), (3000, 27, 70, True)])
def test_credible_limits_and_metric_match_oracle(alpha, T, d, N, whiten):
    rng = np.random.default_rng(int(alpha * 100) + T + d)
    rec = _rec(rng, T, d, N)
    ctx = _ctx(d)
    W = None
    if whiten:
        mu = rng.normal(size=d)
        L = np.linalg.cholesky(np.cov(rec.transpose(0, 2, 1).reshape(-1, d).T.astype(np.float64))
                               + 0.1 * np.eye(d))
        W = (mu, L)
    lo0 = rng.normal(size=d) - 1.0
    hi0 = lo0 + 2.0 + rng.uniform(size=d)
    lo, hi, m = B.best_credible(ctx, torch.tensor(rec, device="cuda"), alpha, whitening=W,
                                ref=(lo0, hi0))
    kw = dict(mu=W[0], L=W[1]) if whiten else {}
    m_or, lo_or, hi_or = OM.credible_metric(rec.astype(np.float64), alpha, lo0, hi0, **kw)
    np.testing.assert_allclose(lo, lo_or, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(hi, hi_or, rtol=1e-12, atol=1e-12)
    assert m == pytest.approx(m_or, rel=1e-10, abs=1e-12)


@pytest.mark.parametrize("na,nb,d,K,whiten", [((40, 25), (30, 20), 4, 500, False),
                                              ((40, 25), (30, 20), 4, 37, True),
                                              ((1, 1), (1, 3), 2, 20, False),
                                              ((200, 64), (150, 64), 27, 64, True)])
def test_sliced_wasserstein_matches_oracle(na, nb, d, K, whiten):
    rng = np.random.default_rng(na[0] + nb[1] + d + K)
    a = _rec(rng, na[0], d, na[1])
    b = _rec(rng, nb[0], d, nb[1], spread=0.5)
    ctx = _ctx(d)
    W = None
    kw = {}
    if whiten:
        L = np.linalg.cholesky(np.cov(a.transpose(0, 2, 1).reshape(-1, d).T.astype(np.float64))
                               + 0.1 * np.eye(d))
        W = (rng.normal(size=d), L)
        kw = dict(mu=W[0], L=W[1])
    seed = 0xABCDEF12345
    got = B.best_sliced_wasserstein(ctx, torch.tensor(a, device="cuda"),
                                    torch.tensor(b, device="cuda"), K, seed, whitening=W)
    ref = OM.sliced_wasserstein(a.astype(np.float64), b.astype(np.float64), K, seed, **kw)
    assert got == pytest.approx(ref, rel=1e-9)


def test_sliced_wasserstein_shift_closed_form_and_zero():
    rng = np.random.default_rng(9)
    d, K, seed = 5, 200, 4242
    a = rng.normal(size=(60, d, 30)).astype(np.float32)
    u = np.array([1.0, -0.5, 0.25, 2.0, 0.0])
    s = 0.5  # exact in float32 together with a grid of draws
    a = np.round(a * 64) / 64
    b = (a + (s * u)[None, :, None]).astype(np.float32)
    ctx = _ctx(d)
    ta, tb = torch.tensor(a, device="cuda"), torch.tensor(b, device="cuda")
    assert B.best_sliced_wasserstein(ctx, ta, ta, K, seed) == 0.0
    w = OM.directions(d, K, seed)
    got = B.best_sliced_wasserstein(ctx, ta, tb, K, seed)
    assert got == pytest.approx(s * np.mean(np.abs(w @ u)), rel=1e-9)

"""Seeded synthetic problem definitions standing in for the paper's cosmology emulators.

The paper samples neural-network likelihood emulators of Planck+BAO (27 parameters for
LambdaCDM, 29 with the sterile-neutrino pair; Sec. 4) whose trained weights and data are not
public inputs here.  These generators build targets of the same dimensionality and shape:

  c1  6 params, Gaussian (cond 1e3) + 0.5*MLP(6->128->128->1), random-walk MH, FP64
  c2  6 params, same form, MLP 6->512x4->1, MALA and HMC (L=10) at 4096 chains
  c3  12 params: 10-d Gaussian + a twisted (banana) pair standing in for (N_eff, m_s),
      MLP 12->1024x4->1, HMC at 16384 chains
  c4  6 params, plain forward model (2500-bin spectrum from 8 damped cosines, chi^2 against
      seeded noisy data); an MLP 6->512x4->1 emulator is trained on it
  c5  27 params (6 "cosmological" + 21 linear nuisance), Gaussian + MLP 27->1024x5->1,
      AIES vs MALA at 65536 walkers

Only numpy's seeded generator is used; nothing here evaluates a log-density or a gradient.
The c4 data vector is simulated by a forward model written here for data generation only.
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 0xBE570000

CONFIGS = {
    "c1": dict(cid=1, d=6, width=128, n_hidden=2, n_chains=64, n_steps=2000, burn=500),
    "c2": dict(cid=2, d=6, width=512, n_hidden=4, n_chains=4096, n_steps=5000, burn=1000),
    "c3": dict(cid=3, d=12, width=1024, n_hidden=4, n_chains=16384, n_steps=3000, burn=1000),
    "c4": dict(cid=4, d=6, width=512, n_hidden=4, n_chains=4096, n_steps=5000, burn=1000),
    "c5": dict(cid=5, d=27, width=1024, n_hidden=5, n_chains=65536, n_steps=5000, burn=1000),
}


# ----------------------------------------------------------------------------------------
# Flat MLP parameter layout (shared convention, data only)
#   [W1 (H x d, row-major), b1 (H), W2 (H x H), b2 (H), ..., W_nh (H x H), b_nh (H),
#    w_out (H), b_out (1)]
# ----------------------------------------------------------------------------------------
def mlp_nparams(d: int, width: int, n_hidden: int) -> int:
    return width * d + width + (n_hidden - 1) * (width * width + width) + width + 1


def mlp_layout(d: int, width: int, n_hidden: int):
    """Offsets of each block in the flat vector: list of (name, offset, shape)."""
    out, off = [], 0
    fan_in = d
    for l in range(n_hidden):
        out.append((f"W{l + 1}", off, (width, fan_in)))
        off += width * fan_in
        out.append((f"b{l + 1}", off, (width,)))
        off += width
        fan_in = width
    out.append(("w_out", off, (width,)))
    off += width
    out.append(("b_out", off, (1,)))
    off += 1
    assert off == mlp_nparams(d, width, n_hidden)
    return out


def xavier_mlp(rng: np.random.Generator, d: int, width: int, n_hidden: int) -> np.ndarray:
    """Glorot & Bengio (2010) normal init: W ~ N(0, 2/(fan_in+fan_out)), biases zero."""
    theta = np.zeros(mlp_nparams(d, width, n_hidden))
    for name, off, shape in mlp_layout(d, width, n_hidden):
        if name.startswith("W"):
            fo, fi = shape
            theta[off:off + fo * fi] = rng.normal(0.0, np.sqrt(2.0 / (fi + fo)), size=fo * fi)
        elif name == "w_out":
            theta[off:off + width] = rng.normal(0.0, np.sqrt(2.0 / (width + 1)), size=width)
    return theta


# ----------------------------------------------------------------------------------------
# Covariances
# ----------------------------------------------------------------------------------------
def spd_with_condition(rng: np.random.Generator, d: int, cond: float = 1e3):
    """S = Q diag(lam) Q^T with Q from a sign-fixed QR of a Gaussian matrix and
    lam_k = cond^{k/(d-1)}, so cond(S) = cond exactly (up to rounding).
    Returns (S, Q, lam)."""
    g = rng.normal(size=(d, d))
    q, r = np.linalg.qr(g)
    q = q * np.sign(np.diag(r))[None, :]
    lam = cond ** (np.arange(d) / max(d - 1, 1))
    s = (q * lam[None, :]) @ q.T
    s = 0.5 * (s + s.T)
    return s, q, lam


def _gauss_mlp_problem(name, cfg, rng, with_mlp=True):
    d = cfg["d"]
    mu = rng.normal(size=d)
    if name in ("c1", "c2"):
        s, q, lam = spd_with_condition(rng, d, 1e3)
        prec = (q / lam[None, :]) @ q.T
        prec = 0.5 * (prec + prec.T)
        twist = None
        cov_closed = s.copy()
        half = 10.0 * np.sqrt(np.diag(s))
    elif name == "c3":
        # indices 0..5 "cosmological", 6 = N_eff-like, 7 = m_s-like, 8..11 nuisance
        gidx = np.array([0, 1, 2, 3, 4, 5, 8, 9, 10, 11])
        s10, q, lam = spd_with_condition(rng, 10, 1e3)
        p10 = (q / lam[None, :]) @ q.T
        sig_u, sig_w, b_lat = 0.8, 0.3, 0.1
        beta = 100.0 * b_lat * sig_w / sig_u ** 2
        s = np.zeros((d, d))
        prec = np.zeros((d, d))
        s[np.ix_(gidx, gidx)] = s10
        prec[np.ix_(gidx, gidx)] = 0.5 * (p10 + p10.T)
        prec[6, 6] = 1.0 / sig_u ** 2
        prec[7, 7] = 1.0 / sig_w ** 2
        cov_closed = s.copy()
        cov_closed[6, 6] = sig_u ** 2
        # Var(x_v) = sig_w^2 + beta^2 Var((x_u - m_u)^2) = sig_w^2 + 2 beta^2 sig_u^4
        cov_closed[7, 7] = sig_w ** 2 + 2.0 * beta ** 2 * sig_u ** 4
        twist = dict(u=6, v=7, beta=beta, center=float(mu[6]), kappa=sig_u ** 2)
        half = 10.0 * np.sqrt(np.diag(cov_closed))
        half[6] = 20.0 * sig_u
        half[7] = 20.0 * np.sqrt(cov_closed[7, 7])
        s = cov_closed  # the Gaussian-equivalent covariance used for scales / whitening
    elif name == "c5":
        s6, _, _ = spd_with_condition(rng, 6, 1e3)
        lc = np.linalg.cholesky(s6)
        tau = 10.0 ** rng.uniform(-1.0, 1.0, size=d - 6)
        c = rng.normal(0.0, 0.3, size=(d - 6, 6))
        a = np.zeros((d, d))
        a[:6, :6] = lc
        a[6:, :6] = c
        a[6:, 6:] = np.diag(tau)
        s = a @ a.T
        ainv = np.linalg.inv(a)
        prec = ainv.T @ ainv
        prec = 0.5 * (prec + prec.T)
        cov_closed = s.copy()
        twist = None
        half = 10.0 * np.sqrt(np.diag(s))
    else:
        raise ValueError(name)

    sd = np.sqrt(np.diag(cov_closed))
    width, nh = cfg["width"], cfg["n_hidden"]
    params = xavier_mlp(rng, d, width, nh)
    prob = dict(
        name=name, d=d,
        lower=mu - half, upper=mu + half,
        gauss_coef=1.0, gauss_mean=mu.copy(), gauss_prec=prec, gauss_cov=s,
        twist=twist,
        width=width, n_hidden=nh, mlp_params=params,
        in_center=mu.copy(), in_invscale=1.0 / sd,
        mlp_coef=0.5 if with_mlp else 0.0, offset=0.0,
        plain=None, plain_mode=0, train_lo=None, train_hi=None,
        closed_mean=mu.copy(), closed_cov=cov_closed,
    )
    return prob


# ----------------------------------------------------------------------------------------
# c4: plain forward model data (simulated here only to produce the observed data vector)
# ----------------------------------------------------------------------------------------
def _simulate_spectrum(theta_hat, xg, a, g, p, k, gamma0):
    amp = np.exp(a @ theta_hat)
    gam = gamma0 * np.exp(g @ theta_hat)
    phs = np.pi * np.tanh(p @ theta_hat)
    return (amp[:, None] * np.exp(-gam[:, None] * xg[None, :])
            * np.cos(2.0 * np.pi * k[:, None] * xg[None, :] + phs[:, None])).sum(0)


def _plain_problem(cfg, rng, train_halfwidth=0.02):
    d = cfg["d"]
    n_bins, n_terms = 2500, 8
    c = rng.normal(size=d)
    w = rng.uniform(0.5, 2.0, size=d)
    xg = np.arange(n_bins) / (n_bins - 1.0)
    m = np.arange(1, n_terms + 1, dtype=np.float64)
    k = 3.0 * m
    gamma0 = 0.5 * m
    a = rng.normal(0.0, 0.3, size=(n_terms, d))
    g = rng.normal(0.0, 0.3, size=(n_terms, d))
    p = rng.normal(0.0, 0.3, size=(n_terms, d))
    th_star = rng.uniform(-0.5, 0.5, size=d)
    sigma = 0.05 * (1.0 + xg)
    noise = rng.normal(size=n_bins)
    data = _simulate_spectrum(th_star, xg, a, g, p, k, gamma0) + sigma * noise
    plain = dict(n_bins=n_bins, n_terms=n_terms, xgrid=xg, data=data,
                 inv_sigma2=1.0 / sigma ** 2, a=a, g=g, p=p, k=k, gamma0=gamma0,
                 center=c.copy(), invscale=1.0 / w, theta_star=c + w * th_star)
    lower, upper = c - w, c + w
    tlo = np.clip(th_star - train_halfwidth, -1.0, 1.0)
    thi = np.clip(th_star + train_halfwidth, -1.0, 1.0)
    train_lo, train_hi = c + w * tlo, c + w * thi
    width, nh = cfg["width"], cfg["n_hidden"]
    prob = dict(
        name="c4", d=d, lower=lower, upper=upper,
        gauss_coef=0.0, gauss_mean=np.zeros(d), gauss_prec=np.zeros((d, d)),
        gauss_cov=np.diag((0.5 * (train_hi - train_lo)) ** 2), twist=None,
        width=width, n_hidden=nh, mlp_params=xavier_mlp(rng, d, width, nh),
        in_center=0.5 * (train_lo + train_hi), in_invscale=2.0 / (train_hi - train_lo),
        mlp_coef=1.0, offset=0.0,
        plain=plain, plain_mode=2, train_lo=train_lo, train_hi=train_hi,
        closed_mean=None, closed_cov=None,
    )
    return prob


def make_problem(name: str, seed: int | None = None, with_mlp: bool = True, **kw) -> dict:
    """Build the problem dict for config `name` (c1..c5).  Seed defaults to 0xBE570000 + id."""
    cfg = CONFIGS[name]
    rng = np.random.default_rng(SEED_BASE + cfg["cid"] if seed is None else seed)
    if name == "c4":
        prob = _plain_problem(cfg, rng, **kw)
    else:
        prob = _gauss_mlp_problem(name, cfg, rng, with_mlp=with_mlp)
    prob["config"] = dict(cfg)
    prob["seed"] = int(SEED_BASE + cfg["cid"] if seed is None else seed)
    return prob


def small_problem(d=5, width=64, n_hidden=3, seed=7, twist=False, with_mlp=True):
    """A small Gaussian+MLP problem for quick parity tests (several MFMA tiles, ragged
    chain counts are chosen by the caller)."""
    rng = np.random.default_rng(seed)
    mu = rng.normal(size=d)
    s, q, lam = spd_with_condition(rng, d, 1e2)
    prec = (q / lam[None, :]) @ q.T
    prec = 0.5 * (prec + prec.T)
    cov = s.copy()
    tw = None
    if twist and d >= 2:
        # replace the last two coordinates' block by an independent twisted pair
        u, v = d - 2, d - 1
        sig_u, sig_w, b_lat = 1.0, 0.5, 0.1
        prec[[u, v], :] = 0.0
        prec[:, [u, v]] = 0.0
        cov[[u, v], :] = 0.0
        cov[:, [u, v]] = 0.0
        prec[u, u] = 1.0 / sig_u ** 2
        prec[v, v] = 1.0 / sig_w ** 2
        beta = 100.0 * b_lat * sig_w / sig_u ** 2
        # the Gaussian block's covariance is the inverse of its (kept) precision block
        g = [i for i in range(d) if i not in (u, v)]
        cov[np.ix_(g, g)] = np.linalg.inv(prec[np.ix_(g, g)])
        cov[u, u] = sig_u ** 2
        cov[v, v] = sig_w ** 2 + 2.0 * beta ** 2 * sig_u ** 4
        tw = dict(u=u, v=v, beta=beta, center=float(mu[u]), kappa=sig_u ** 2)
    sd = np.sqrt(np.diag(cov))
    half = 10.0 * sd
    return dict(
        name="small", d=d, lower=mu - half, upper=mu + half,
        gauss_coef=1.0, gauss_mean=mu.copy(), gauss_prec=prec, gauss_cov=cov, twist=tw,
        width=width, n_hidden=n_hidden, mlp_params=xavier_mlp(rng, d, width, n_hidden),
        in_center=mu.copy(), in_invscale=1.0 / sd, mlp_coef=0.5 if with_mlp else 0.0,
        offset=0.0, plain=None, plain_mode=0, train_lo=None, train_hi=None,
        closed_mean=mu.copy(), closed_cov=cov, config=dict(d=d, width=width, n_hidden=n_hidden),
        seed=seed,
    )


# ----------------------------------------------------------------------------------------
# Designs and test series
# ----------------------------------------------------------------------------------------
def latin_hypercube(rng: np.random.Generator, n: int, d: int) -> np.ndarray:
    """McKay, Beckman & Conover (1979): per dimension an independent random permutation of
    the n strata plus a uniform jitter inside each stratum.  Returns points in [0, 1)^d."""
    out = np.empty((n, d))
    for j in range(d):
        out[:, j] = (rng.permutation(n) + rng.uniform(size=n)) / n
    return out


def minibatch_permutations(rng: np.random.Generator, n: int, n_epochs: int) -> np.ndarray:
    return np.stack([rng.permutation(n) for _ in range(n_epochs)]).astype(np.int32)


def ar1_chains(rng: np.random.Generator, rho: float, n_chains: int, n_steps: int) -> np.ndarray:
    """Stationary AR(1) series x_t = rho x_{t-1} + sqrt(1-rho^2) e_t, shape (n_chains, n_steps)."""
    x = np.empty((n_chains, n_steps))
    x[:, 0] = rng.normal(size=n_chains)
    e = rng.normal(size=(n_chains, n_steps)) * np.sqrt(1.0 - rho * rho)
    for t in range(1, n_steps):
        x[:, t] = rho * x[:, t - 1] + e[:, t]
    return x


def walsh_chains(deltas, n_chains=8) -> np.ndarray:
    """Record (T, d, N) of chains x_tc = m_c + y_t with T = 2d: the rows y_t = +-a e_k
    (a^2 = (T - 1)/2) give every chain the unbiased covariance I exactly, and the chain means
    m_c = (delta_i s_i[c]) use orthogonal zero-mean sign vectors s_i (Hadamard columns), so
    the unbiased covariance of the means is diag(delta_i^2 N / (N - 1)).  n_chains is a
    power of two above d."""
    from scipy.linalg import hadamard
    d = len(deltas)
    T = 2 * d
    a = np.sqrt((T - 1) / 2.0)
    y = np.concatenate([a * np.eye(d), -a * np.eye(d)])
    hm = hadamard(n_chains)[:, 1:d + 1].astype(np.float64)
    m = hm * np.asarray(deltas, dtype=np.float64)[None, :]
    return np.ascontiguousarray(y[:, :, None] + m.T[None, :, :])

"""No-U-Turn sampler (Hoffman & Gelman 2014, efficient slice version with progressive
sampling), float64, one chain at a time.  Test infrastructure only: the library's HIP
path never imports this module.

The paper lists NUTS among its samplers (Sec. 2.1 and Table 1) and names it as the
sampler whose per-transition gradient cost grows with the tree depth.  This oracle follows
Hoffman & Gelman's efficient algorithm in the whitened space of Sec. 2.2 (identity mass):

  q ~ N(0, I); H(z, q) = -log pi_z(z) + |q|^2 / 2; slice log u* = log u - H(z0, q0);
  the trajectory doubles (depth j = 0, 1, ...): a direction v = +-1 is drawn, and a
  balanced subtree of 2^j leapfrog steps (step v eps) is built from the tree end on that
  side.  A leaf counts as a valid point when log u* <= -H(leaf) and is divergent when
  log u* >= -H(leaf) + 1000.  Two sibling subtrees merge into their parent: the parent's
  candidate is the second sibling's with probability n2 / (n1 + n2) (n = valid points),
  and the parent stops the trajectory if either sibling stopped or its end points make a
  U-turn: continue only while (z+ - z-) . q- >= 0 and (z+ - z-) . q+ >= 0.  At the top
  level a finished subtree that did not stop replaces the tree's candidate with
  probability min(1, n' / n); the tree then stops on a U-turn of its whole span, or at
  the maximum depth.

Readings where the algorithm leaves a choice (also used by the HIP path):
  * the prior box: a leaf outside it has log pi = -inf (never a valid point, and it stops
    the trajectory as a divergence); the leapfrog dynamics use the unbounded density, as
    in the HMC transition; with the smooth box penalty the penalised density is used
    everywhere;
  * the acceptance statistic for step-size adaptation is the mean over every leaf of the
    transition of min(1, exp(H(z0, q0) - H(leaf)));
  * random numbers (Philox counters, step t):
      momentum       normals(stream 1, sub 0)                       (as HMC)
      slice u        stream 2, sub 0, block 0, first uniform       (as the accept uniform)
      doubling j     stream 5, sub j, block 0: first uniform < 0.5 -> v = -1, else +1;
                     second uniform u: the finished subtree's candidate is taken iff
                     u < n' / n
      merge          stream 5, sub 16 + j, block 8 k + l, first uniform: merging two
                     siblings into a subtree of 2^l leaves whose last leaf is leaf k
                     (0-based) of doubling j takes the second sibling's candidate iff
                     u < n2 / (n1 + n2).
"""
from __future__ import annotations

import numpy as np

from . import philox as ph
from .target import hard_box, whitened

STREAM_NUTS = 5
DELTA_MAX = 1000.0


def _u(seed, chain, t, sub, blk):
    ua, ub = ph.uniforms2(seed, np.array([chain], dtype=np.uint64), t, STREAM_NUTS, sub, blk)
    return float(ua[0]), float(ub[0])


class _Leaf:
    __slots__ = ("z", "q", "g", "lp")

    def __init__(self, z, q, g, lp):
        self.z, self.q, self.g, self.lp = z, q, g, lp


def _uturn_ok(zm, qm, zp, qp):
    dz = zp - zm
    return bool(np.dot(dz, qm) >= 0.0 and np.dot(dz, qp) >= 0.0)


def nuts_step(prob, W, st, t, seed, eps, max_depth=8, chains=None, params=None):
    """One NUTS transition for every chain of st (dict z, lp, g).  Returns (new state,
    info with accept_stat (mean over leaves), n_leaves, depth)."""
    z0s, lp0s, g0s = st["z"], st["lp"], st["g"]
    n, d = z0s.shape
    ids = np.arange(n, dtype=np.uint64) if chains is None else np.asarray(chains, np.uint64)
    q0s = ph.normals(seed, ids, t, ph.STREAM_NORMAL, 0, d)
    log_us = np.log(ph.accept_uniform(seed, ids, t))
    out_z, out_lp, out_g = z0s.copy(), lp0s.copy(), g0s.copy()
    stats, leaves, depths = np.zeros(n), np.zeros(n, dtype=np.int64), np.zeros(n, dtype=np.int64)
    mu, L = W["mu"], W["L"]

    for c in range(n):
        ch = int(ids[c])
        z0, q0, g0, lp0 = z0s[c], q0s[c], g0s[c], lp0s[c]
        h0 = -lp0 + 0.5 * q0 @ q0
        log_slice = log_us[c] - h0
        counters = dict(leaves=0, stat=0.0)

        def leapfrog(leaf, v):
            qh = leaf.q + 0.5 * v * eps * leaf.g
            z = leaf.z + v * eps * qh
            lpu, g, x = whitened(prob, mu, L, z[None, :], params, with_box=False)
            inside = bool(np.all((x[0] >= prob["lower"]) & (x[0] <= prob["upper"]))) or \
                not hard_box(prob)
            q = qh + 0.5 * v * eps * g[0]
            return _Leaf(z, q, g[0], float(lpu[0]) if inside else -np.inf)

        def build(start, v, j, depth_j, k0):
            """Subtree of 2^j leaves continuing from `start` in direction v; its leaves are
            leaves k0 .. k0 + 2^j - 1 of doubling depth_j.  Returns (first, last,
            candidate, n_valid, keep_going)."""
            if j == 0:
                leaf = leapfrog(start, v)
                h = -leaf.lp + 0.5 * leaf.q @ leaf.q
                counters["leaves"] += 1
                with np.errstate(over="ignore", invalid="ignore"):
                    a = np.exp(min(0.0, h0 - h)) if np.isfinite(h) else 0.0
                counters["stat"] += a
                valid = 1 if log_slice <= -h else 0
                go = bool(log_slice < -h + DELTA_MAX)
                return leaf, leaf, leaf, valid, go
            first, mid, cand, n1, go1 = build(start, v, j - 1, depth_j, k0)
            if not go1:
                return first, mid, cand, n1, False
            mid2, last, cand2, n2, go2 = build(mid, v, j - 1, depth_j, k0 + (1 << (j - 1)))
            k_last = k0 + (1 << j) - 1
            u, _ = _u(seed, ch, t, 16 + depth_j, 8 * k_last + j)
            if n1 + n2 > 0 and u < n2 / (n1 + n2):
                cand = cand2
            if v > 0:
                ok = _uturn_ok(first.z, first.q, last.z, last.q)
            else:
                ok = _uturn_ok(last.z, last.q, first.z, first.q)
            return first, last, cand, n1 + n2, bool(go2 and ok)

        start = _Leaf(z0, q0, g0, lp0)
        minus, plus, cand = start, start, start
        n_valid, depth = 1, 0
        for j in range(max_depth):
            ua, ub = _u(seed, ch, t, j, 0)
            v = -1 if ua < 0.5 else 1
            first, last, c_new, n_new, go = build(minus if v < 0 else plus, v, j, j, 0)
            depth = j + 1
            if v < 0:
                minus = last
            else:
                plus = last
            if not go:
                break
            if ub < n_new / n_valid:
                cand = c_new
            n_valid += n_new
            if not _uturn_ok(minus.z, minus.q, plus.z, plus.q):
                break
        if cand is not start:
            lpb, gb, _ = whitened(prob, mu, L, cand.z[None, :], params, with_box=True)
            out_z[c], out_lp[c], out_g[c] = cand.z, float(lpb[0]), gb[0]
        leaves[c] = counters["leaves"]
        stats[c] = counters["stat"] / max(1, counters["leaves"])
        depths[c] = depth
    new = dict(z=out_z, lp=out_lp, g=out_g)
    return new, dict(accept_stat=stats, n_leaves=leaves, depth=depths, momentum=q0s,
                     log_u=log_us)

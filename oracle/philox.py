"""Philox4x32-10 counter-based generator and the uniform / normal maps built on it.

Generator: Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as easy as 1, 2, 3"
(SC'11).  A 128-bit counter (c0..c3) and 64-bit key (k0, k1) go through 10 rounds; each
round multiplies c0 and c2 by fixed 32-bit constants, splits the 64-bit products into
high/low halves and mixes them with c1, c3 and the key; the key is bumped by the Weyl
constants between rounds.

Counter layout used by every sampler (both implementations follow it independently):
    c0 = chain index, c1 = step index (low 32 bits), c2 = (stream << 24) | substep,
    c3 = block index;  key = (seed low 32 bits, seed high 32 bits)
Streams: 1 proposal / momentum normals, 2 accept uniform, 3 AIES partner + stretch,
         4 walker initialisation, 5 NUTS tree decisions, 6 sliced-Wasserstein directions,
         7 differential-evolution partners and gamma noise.

Uniform map: two 32-bit words (ra, rb) -> n = (ra >> 6) * 2^26 + (rb >> 6)  (52 bits)
             u = (n + 0.5) * 2^-52, exactly representable, strictly inside (0, 1).
Normals: Box-Muller on the block's two uniforms (u1 from words 0,1; u2 from words 2,3):
             r = sqrt(-2 ln u1);  n0 = r cos(2 pi u2),  n1 = r sin(2 pi u2).
Dimension i of a d-vector of normals uses block i // 2 and member i % 2.
"""
from __future__ import annotations

import numpy as np

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
_MASK = np.uint64(0xFFFFFFFF)

STREAM_NORMAL = 1
STREAM_ACCEPT = 2
STREAM_AIES = 3
STREAM_INIT = 4


def philox4x32_10(c0, c1, c2, c3, k0: int, k1: int):
    """Vectorised Philox4x32 with 10 rounds.  Counters are array-likes of uint32 values
    (broadcast together); returns four uint32 arrays."""
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) & _MASK for c in (c0, c1, c2, c3))
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    k0 = np.uint64(k0 & 0xFFFFFFFF)
    k1 = np.uint64(k1 & 0xFFFFFFFF)
    m0, m1 = np.uint64(M0), np.uint64(M1)
    for _ in range(10):
        p0 = m0 * c0            # < 2^64, exact in uint64
        p1 = m1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        k0 = (k0 + np.uint64(W0)) & _MASK
        k1 = (k1 + np.uint64(W1)) & _MASK
    return (c0.astype(np.uint32), c1.astype(np.uint32),
            c2.astype(np.uint32), c3.astype(np.uint32))


def seed_key(seed: int):
    return seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF


def u52(ra, rb):
    n = ((np.asarray(ra, dtype=np.uint64) >> np.uint64(6)) << np.uint64(26)) | (
        np.asarray(rb, dtype=np.uint64) >> np.uint64(6))
    return (n.astype(np.float64) + 0.5) * 2.0 ** -52


def block(seed, chain, step, stream, sub, blk):
    k0, k1 = seed_key(seed)
    c2 = (np.asarray(stream, dtype=np.uint64) << np.uint64(24)) | np.asarray(sub, dtype=np.uint64)
    return philox4x32_10(chain, np.asarray(step, dtype=np.uint64) & _MASK, c2, blk, k0, k1)


def uniforms2(seed, chain, step, stream, sub, blk):
    """The two uniforms of one block: (u from words 0,1 ; u from words 2,3)."""
    r0, r1, r2, r3 = block(seed, chain, step, stream, sub, blk)
    return u52(r0, r1), u52(r2, r3)


def normals(seed, chains, step, stream, sub, d):
    """Standard normals, shape (len(chains), d); dim i from block i//2, member i%2."""
    chains = np.asarray(chains)
    nb = (d + 1) // 2
    out = np.empty((chains.shape[0], 2 * nb))
    for b in range(nb):
        ua, ub = uniforms2(seed, chains, step, stream, sub, b)
        r = np.sqrt(-2.0 * np.log(ua))
        out[:, 2 * b] = r * np.cos(2.0 * np.pi * ub)
        out[:, 2 * b + 1] = r * np.sin(2.0 * np.pi * ub)
    return out[:, :d]


def accept_uniform(seed, chains, step, sub=0):
    ua, _ = uniforms2(seed, np.asarray(chains), step, STREAM_ACCEPT, sub, 0)
    return ua


def init_uniforms(seed, chains, d, step=0):
    """Uniforms for walker initialisation: dim i from block i//2, member i%2 (step 0 at
    the start, the current step counter when the walkers are re-initialised)."""
    chains = np.asarray(chains)
    nb = (d + 1) // 2
    out = np.empty((chains.shape[0], 2 * nb))
    for b in range(nb):
        ua, ub = uniforms2(seed, chains, step, STREAM_INIT, 0, b)
        out[:, 2 * b] = ua
        out[:, 2 * b + 1] = ub
    return out[:, :d]


def init_normals(seed, chains, d, step=0):
    return normals(seed, chains, step, STREAM_INIT, 1, d)


def init_hypersphere(seed, chains, d, step=0):
    """Points uniform in the unit d-ball for the hypersphere-based initialisation (Sec. 3.2):
    u = xi / |xi| with xi the d normals of the init stream's sub 2 (uniform on the sphere,
    Muller 1959), radius U^(1/d) with U the first uniform of block 0 of sub 3 (the ball's
    volume below radius r is r^d).  Returns (len(chains), d)."""
    xi = normals(seed, chains, step, STREAM_INIT, 2, d)
    u, _ = uniforms2(seed, np.asarray(chains), step, STREAM_INIT, 3, 0)
    r = u ** (1.0 / d)
    return xi / np.sqrt(np.sum(xi * xi, axis=1))[:, None] * r[:, None]

"""Pins for the oracle's Philox4x32-10 generator and its uniform / normal maps."""
import os

import numpy as np
import pytest
from scipy import stats

from oracle import philox as ph


def _kat(golden_dir):
    rows = []
    with open(os.path.join(golden_dir, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            rows.append([int(v, 16) for v in line.split()])
    return rows


def test_philox_known_answers(golden_dir):
    rows = _kat(golden_dir)
    assert len(rows) == 3
    for r in rows:
        out = ph.philox4x32_10(*[np.uint32(v) for v in r[:4]], r[4], r[5])
        assert [int(v) for v in out] == r[6:10]


def test_philox_vectorised_matches_scalar():
    c0 = np.arange(100, dtype=np.uint64)
    vec = ph.philox4x32_10(c0, 7, 3 << 24, 2, 11, 13)
    for i in (0, 17, 99):
        sc = ph.philox4x32_10(np.uint32(i), np.uint32(7), np.uint32(3 << 24), np.uint32(2), 11, 13)
        assert [int(v[i]) for v in vec] == [int(v) for v in sc]


def test_u52_exact_and_open_interval():
    assert ph.u52(0, 0) == 0.5 * 2.0 ** -52
    top = ph.u52(np.uint32(0xFFFFFFFF), np.uint32(0xFFFFFFFF))
    assert top == 1.0 - 0.5 * 2.0 ** -52
    assert 0.0 < ph.u52(0, 0) < top < 1.0


def test_uniform_distribution():
    ids = np.arange(200000, dtype=np.uint64)
    ua, ub = ph.uniforms2(1234, ids, 5, ph.STREAM_ACCEPT, 0, 0)
    for u in (ua, ub):
        assert stats.kstest(u, "uniform").pvalue > 1e-4
        assert abs(u.mean() - 0.5) < 5 * np.sqrt(1 / 12 / u.size)
    assert abs(np.corrcoef(ua, ub)[0, 1]) < 5 / np.sqrt(ua.size)


def test_normals_distribution_and_layout():
    ids = np.arange(100000, dtype=np.uint64)
    z = ph.normals(99, ids, 3, ph.STREAM_NORMAL, 0, 5)
    assert z.shape == (100000, 5)
    for i in range(5):
        assert stats.kstest(z[:, i], "norm").pvalue > 1e-4
        assert abs(z[:, i].mean()) < 5 / np.sqrt(ids.size)
        assert abs(z[:, i].var() - 1.0) < 5 * np.sqrt(2.0 / ids.size)
    # dims 2i and 2i+1 come from the same block: the Box-Muller pair
    ua, ub = ph.uniforms2(99, ids[:10], 3, ph.STREAM_NORMAL, 0, 1)
    r = np.sqrt(-2 * np.log(ua))
    np.testing.assert_allclose(z[:10, 2], r * np.cos(2 * np.pi * ub), rtol=0, atol=0)
    np.testing.assert_allclose(z[:10, 3], r * np.sin(2 * np.pi * ub), rtol=0, atol=0)


def test_streams_are_distinct():
    ids = np.arange(1000, dtype=np.uint64)
    a = ph.block(5, ids, 0, 1, 0, 0)[0]
    b = ph.block(5, ids, 0, 2, 0, 0)[0]
    c = ph.block(5, ids, 1, 1, 0, 0)[0]
    assert np.mean(a == b) < 0.01 and np.mean(a == c) < 0.01


@pytest.mark.parametrize("d", [1, 2, 6, 27])
def test_hypersphere_points_are_uniform_in_the_unit_ball(d):
    """Uniform in the d-ball: |u| <= 1, P(|u| <= r) = r^d (KS), mean 0 and covariance
    I / (d + 2) (E|u|^2 = d / (d + 2)) within 5 Monte-Carlo standard errors."""
    n = 40000
    u = ph.init_hypersphere(123, np.arange(n), d, step=4)
    r = np.sqrt(np.sum(u * u, axis=1))
    assert u.shape == (n, d) and np.all(r <= 1.0)
    assert stats.kstest(r, lambda t: np.clip(t, 0, 1) ** d).pvalue > 1e-4
    se = np.sqrt(1.0 / (d + 2) / n)
    assert np.all(np.abs(u.mean(0)) < 5 * se)
    cov = u.T @ u / n
    # Var(u_i^2) <= E u_i^4 <= 1; off-diagonal and diagonal entries within 5 SE
    assert np.all(np.abs(cov - np.eye(d) / (d + 2)) < 5 * np.sqrt(1.0 / n))
    if d == 2:  # a disk: a quarter of the points inside radius 1/2
        assert abs(np.mean(r < 0.5) - 0.25) < 5 * np.sqrt(0.25 * 0.75 / n)


def test_hypersphere_direction_and_radius_use_their_own_substreams():
    # the direction comes from the init stream's normals of sub 2, the radius from sub 3
    u = ph.init_hypersphere(9, np.arange(5), 4, step=2)
    xi = ph.normals(9, np.arange(5), 2, ph.STREAM_INIT, 2, 4)
    ua, _ = ph.uniforms2(9, np.arange(5), 2, ph.STREAM_INIT, 3, 0)
    np.testing.assert_allclose(u, xi / np.linalg.norm(xi, axis=1)[:, None] * ua[:, None] ** 0.25,
                               rtol=1e-14)

"""Pins for the smooth boundary penalty of Sec. 3.1 (box_penalty = 1): zero inside the box,
a closed form on a flat target, gradients equal to central finite differences outside,
value and slope continuous across a face, and the hard box unchanged when it is off."""
import numpy as np
import pytest

from oracle import target
from workloads import small_problem


def _prob(**kw):
    prob = small_problem(d=4, width=64, n_hidden=2, seed=5)
    return dict(prob, box_penalty=1, penalty_width=0.02, **kw)


def test_zero_inside_and_hard_box_unchanged():
    prob = _prob()
    rng = np.random.default_rng(1)
    x = prob["lower"] + rng.uniform(size=(50, 4)) * (prob["upper"] - prob["lower"])
    a, ga = target.log_target(prob, x)
    b, gb = target.log_target(dict(prob, box_penalty=0), x)
    assert np.array_equal(a, b) and np.array_equal(ga, gb)
    out = prob["upper"] + 0.1
    assert target.log_target(dict(prob, box_penalty=0), out[None, :])[0][0] == -np.inf


def test_closed_form_on_a_flat_target():
    prob = _prob(gauss_coef=0.0, mlp_coef=0.0, offset=0.0)
    width = prob["upper"] - prob["lower"]
    w = 0.02
    x = prob["upper"].copy()
    x[1] += w * width[1]  # one width w outside the upper face: r = w
    x[3] = prob["lower"][3] - 2 * w * width[3]  # two widths below the lower face
    lp, g = target.log_target(prob, x[None, :])
    assert lp[0] == pytest.approx(-((np.e - 2.0) + (np.e ** 2 - 3.0)), rel=1e-13)
    assert g[0, 1] == pytest.approx(-(np.e - 1.0) / (w * width[1]), rel=1e-13)
    assert g[0, 3] == pytest.approx((np.e ** 2 - 1.0) / (w * width[3]), rel=1e-13)
    assert g[0, 0] == 0.0 and g[0, 2] == 0.0


def test_gradient_matches_central_differences_outside():
    prob = _prob()
    width = prob["upper"] - prob["lower"]
    rng = np.random.default_rng(2)
    x = prob["upper"] + rng.uniform(0.001, 0.05, size=(6, 4)) * width
    x[:, 0] = prob["lower"][0] - 0.03 * width[0]
    _, g = target.log_target(prob, x)
    for i in range(4):
        h = 1e-6 * width[i]
        e = np.zeros(4)
        e[i] = h
        fd = (target.log_target(prob, x + e)[0] - target.log_target(prob, x - e)[0]) / (2 * h)
        np.testing.assert_allclose(g[:, i], fd, rtol=1e-6, atol=1e-6)


def test_value_and_slope_continuous_across_a_face():
    """Just outside a face (r = distance / width) the penalty is (r/w)^2 / 2 to leading order
    and its slope (r/w) / (w width): both vanish at the face, so the penalised density and
    its gradient join the unbounded ones continuously."""
    prob = _prob()
    w = prob["penalty_width"]
    x_in = 0.5 * (prob["lower"] + prob["upper"])
    x_in[2] = prob["upper"][2]
    width = prob["upper"][2] - prob["lower"][2]
    free = dict(prob, box_penalty=0)
    for r in (1e-4, 1e-6):
        x_out = x_in.copy()
        x_out[2] += r * width
        p, dp = target.box_penalty(prob, x_out[None, :])
        assert p[0] == pytest.approx(0.5 * (r / w) ** 2, rel=0.02)
        assert dp[0, 2] == pytest.approx((r / w) / (w * width), rel=0.02)
        a, ga = target.log_target(prob, x_out[None, :])
        b, gb = target.log_target(free, x_out[None, :], with_box=False)
        assert a[0] == pytest.approx(b[0] - p[0], abs=1e-12)
        np.testing.assert_allclose(ga, gb - dp, atol=1e-12)

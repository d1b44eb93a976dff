"""Weight gradients of the target through the emulator (best_logL_param_grad) and the
autograd wrapper EmulatorFn, against the FP64 oracle's reverse mode (oracle.mlp.param_grad,
itself pinned to central differences) and against central differences of the GPU path.

Tolerance: the weight-gradient GEMMs sum n products of FP32-exported activations and deltas
on FP32 matrix cores, so every component is compared on the scale of the largest one:
|g - g_ref| <= tol * max|g_ref|, tol = 2e-5 for FP32 networks and 2^-7 for BF16 (the
deltas carry the 16-bit rounding of the layer inputs, 2^-8 relative, through the layers)."""
import numpy as np
import pytest
import torch

import paper_2606_04895_amd as B
from oracle import mlp as OM, target as OT
from workloads import make_problem, small_problem

pytestmark = pytest.mark.gpu

TOL = {"fp32": 2e-5, "bf16": 2.0 ** -7}


def _points(prob, n, seed, spread=1.5):
    rng = np.random.default_rng(seed)
    if prob.get("closed_cov") is not None:
        sd = np.sqrt(np.diag(prob["closed_cov"]))
        return prob["gauss_mean"] + spread * rng.normal(size=(n, prob["d"])) * sd
    return prob["lower"] + rng.uniform(size=(n, prob["d"])) * (prob["upper"] - prob["lower"])


def _oracle(prob, x, w):
    """sum_c w_c d log pi(x_c) / d theta in FP64: the MLP term only, where log pi uses it."""
    use = np.ones(len(x), bool)
    if prob.get("plain_mode", 0) == 1:
        use = OT.in_box(prob["train_lo"], prob["train_hi"], x)
    up = prob["mlp_coef"] * w * use
    g, _ = OM.param_grad(prob["mlp_params"], OT.normalise(prob, x), up, prob["d"],
                         prob["width"], prob["n_hidden"])
    return g


def _check(prob, prec, n, seed):
    print(f"param grad: {prob['name']} {prec} n={n}", flush=True)
    ctx = B.best_init(prob, n_chains=64, precision=prec, seed=1)
    x = _points(prob, n, seed)
    w = np.random.default_rng(seed + 1).normal(size=n)
    g = B.best_logL_param_grad(ctx, torch.tensor(x.T.copy(), device="cuda"),
                               torch.tensor(w, device="cuda")).cpu().numpy()
    ref = _oracle(prob, x, w)
    err = np.abs(g - ref).max() / np.abs(ref).max()
    assert np.all(np.isfinite(g)) and err < TOL[prec], (prob["name"], prec, n, err)
    return err


@pytest.mark.parametrize("n", [1, 37, 333])
def test_param_grad_small_problem_fp32(n):
    _check(small_problem(d=5, width=128, n_hidden=3, twist=True), "fp32", n, seed=n)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_param_grad_c2_full_batch(prec):
    """C2's network at its 4096 chains (every weight-gradient GEMM tile and the full
    vector of 790,017 parameters)."""
    _check(make_problem("c2"), prec, 4096, seed=5)


def test_param_grad_single_hidden_layer_and_ragged():
    _check(small_problem(d=3, width=128, n_hidden=1), "fp32", 50, seed=2)


def test_param_grad_learned_emulator_counts_only_points_in_the_training_box():
    prob = dict(make_problem("c4"), plain_mode=1)
    rng = np.random.default_rng(3)
    lo, hi = prob["train_lo"], prob["train_hi"]
    inside = lo + rng.uniform(size=(150, 6)) * (hi - lo)
    outside = prob["lower"] + rng.uniform(size=(50, 6)) * (prob["upper"] - prob["lower"])
    x = np.concatenate([inside, outside])
    assert (~OT.in_box(lo, hi, outside)).sum() > 40
    ctx = B.best_init(prob, n_chains=64, precision="fp32", seed=1)
    w = rng.normal(size=len(x))
    g = B.best_logL_param_grad(ctx, torch.tensor(x.T.copy(), device="cuda"),
                               torch.tensor(w, device="cuda")).cpu().numpy()
    ref = _oracle(prob, x, w)
    assert np.abs(g - ref).max() / np.abs(ref).max() < TOL["fp32"]
    # the plain model alone has no emulator parameters to differentiate
    ctx2 = B.best_init(dict(prob, plain_mode=2), n_chains=64, precision="fp32", seed=1)
    g2 = B.best_logL_param_grad(ctx2, torch.tensor(x.T.copy(), device="cuda"))
    assert torch.count_nonzero(g2).item() == 0


def test_emulator_fn_backward_matches_oracle_for_points_and_weights():
    prob = small_problem(d=5, width=128, n_hidden=3, twist=True)
    ctx = B.best_init(prob, n_chains=64, precision="fp32", seed=1)
    x_np = _points(prob, 200, 9)
    w_np = np.random.default_rng(4).normal(size=200)
    params = torch.tensor(prob["mlp_params"] * 1.1, device="cuda", requires_grad=True)
    x = torch.tensor(x_np.T.copy(), device="cuda", requires_grad=True)
    lp = B.EmulatorFn.apply(ctx, x, params)
    (lp * torch.tensor(w_np, device="cuda")).sum().backward()
    p2 = dict(prob, mlp_params=prob["mlp_params"] * 1.1)
    lo, go = OT.log_target(p2, x_np)
    np.testing.assert_allclose(lp.detach().cpu().numpy(), lo, atol=2e-5 * (1 + np.abs(lo).max()))
    gx = x.grad.cpu().numpy().T
    assert np.abs(gx - w_np[:, None] * go).max() < 2e-4 * (1 + np.abs(w_np[:, None] * go).max())
    ref = _oracle(p2, x_np, w_np)
    gp = params.grad.cpu().numpy()
    assert np.abs(gp - ref).max() / np.abs(ref).max() < TOL["fp32"]


def test_emulator_fn_weight_gradient_matches_central_differences_of_the_gpu_path():
    """d/d theta_k of sum_c log pi(x_c), from EmulatorFn's backward and from central
    differences of the GPU evaluation itself (FP32 network, step h = 1e-3 relative)."""
    prob = small_problem(d=4, width=128, n_hidden=2)
    ctx = B.best_init(prob, n_chains=64, precision="fp32", seed=1)
    x = torch.tensor(_points(prob, 512, 3).T.copy(), device="cuda")
    p0 = torch.tensor(prob["mlp_params"], device="cuda", requires_grad=True)
    B.EmulatorFn.apply(ctx, x, p0).sum().backward()
    g = p0.grad.cpu().numpy()
    # one parameter of each block: W1, b1, W2, b2, w_out, b_out
    d, H = 4, 128
    ks = [3, H * d + 7, H * d + H + 5 * H + 11, H * d + H + H * H + 17,
          H * d + 2 * H + H * H + 23, H * d + 3 * H + H * H]
    for k in ks:
        hk = 1e-3 * max(1.0, abs(float(prob["mlp_params"][k])))
        vals = []
        for sgn in (1.0, -1.0):
            p = prob["mlp_params"].copy()
            p[k] += sgn * hk
            with torch.no_grad():
                vals.append(float(B.EmulatorFn.apply(ctx, x, torch.tensor(p)).sum()))
        fd = (vals[0] - vals[1]) / (2 * hk)
        assert abs(fd - g[k]) < 2e-3 * max(1.0, abs(g[k])), (k, fd, g[k])

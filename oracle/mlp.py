"""The tanh multilayer-perceptron likelihood emulator, in float64.

The paper's emulators (CLiENT, Sec. 1 and Sec. 4) are dense networks mapping parameters to
a log-likelihood, evaluated in batches (Fig. scaling) and differentiated automatically
(Sec. 2.1 needs grad log pi).  Definition used here, for input theta_hat (n, d):

    h_0 = theta_hat,   h_l = tanh(W_l h_{l-1} + b_l)  (l = 1..L),   out = w_out . h_L + b_out

Reverse mode for the input gradient:
    delta_L = w_out * (1 - h_L^2);  delta_{l-1} = (W_l^T delta_l) * (1 - h_{l-1}^2);
    d out / d theta_hat = W_1^T delta_1
Weight gradients of sum_c up_c * out_c (used by training):
    dW_l = sum_c delta_l[c] h_{l-1}[c]^T,  db_l = sum_c delta_l[c],
    dw_out = sum_c up_c h_L[c],  db_out = sum_c up_c     (delta scaled by up_c)

Flat parameter layout: [W1 (H x d), b1, W2 (H x H), b2, ..., W_L, b_L, w_out (H), b_out].
"""
from __future__ import annotations

import numpy as np


def unpack(params, d, width, n_hidden):
    params = np.asarray(params, dtype=np.float64)
    Ws, bs, off, fan_in = [], [], 0, d
    for _ in range(n_hidden):
        Ws.append(params[off:off + width * fan_in].reshape(width, fan_in))
        off += width * fan_in
        bs.append(params[off:off + width])
        off += width
        fan_in = width
    w_out = params[off:off + width]
    off += width
    b_out = params[off]
    off += 1
    assert off == params.size, "parameter vector length does not match the layout"
    return Ws, bs, w_out, b_out


def pack(Ws, bs, w_out, b_out):
    parts = []
    for W, b in zip(Ws, bs):
        parts += [np.ravel(W), np.ravel(b)]
    parts += [np.ravel(w_out), np.atleast_1d(b_out)]
    return np.concatenate(parts).astype(np.float64)


def forward(params, theta_hat, d, width, n_hidden, activation=np.tanh):
    """Returns (out (n,), hs list of (n, H) activations h_1..h_L)."""
    Ws, bs, w_out, b_out = unpack(params, d, width, n_hidden)
    h = np.asarray(theta_hat, dtype=np.float64)
    hs = []
    for W, b in zip(Ws, bs):
        h = activation(h @ W.T + b)
        hs.append(h)
    return h @ w_out + b_out, hs


def value_and_input_grad(params, theta_hat, d, width, n_hidden):
    """MLP value (n,) and d out / d theta_hat (n, d) by reverse mode."""
    Ws, _, w_out, _ = unpack(params, d, width, n_hidden)
    out, hs = forward(params, theta_hat, d, width, n_hidden)
    delta = w_out[None, :] * (1.0 - hs[-1] ** 2)
    for l in range(n_hidden - 1, 0, -1):
        delta = (delta @ Ws[l]) * (1.0 - hs[l - 1] ** 2)
    return out, delta @ Ws[0]


def param_grad(params, theta_hat, upstream, d, width, n_hidden):
    """Gradient of sum_c upstream[c] * out[c] with respect to every parameter (flat)."""
    Ws, bs, w_out, _ = unpack(params, d, width, n_hidden)
    theta_hat = np.asarray(theta_hat, dtype=np.float64)
    up = np.asarray(upstream, dtype=np.float64)
    out, hs = forward(params, theta_hat, d, width, n_hidden)
    dWs, dbs = [None] * n_hidden, [None] * n_hidden
    dw_out = up @ hs[-1]
    db_out = up.sum()
    delta = up[:, None] * w_out[None, :] * (1.0 - hs[-1] ** 2)
    for l in range(n_hidden - 1, -1, -1):
        h_prev = hs[l - 1] if l > 0 else theta_hat
        dWs[l] = delta.T @ h_prev
        dbs[l] = delta.sum(0)
        if l > 0:
            delta = (delta @ Ws[l]) * (1.0 - hs[l - 1] ** 2)
    return pack(dWs, dbs, dw_out, db_out), out

"""One training step of the adaptive observables and the linear reconstruction on cached
Pauli features (oracle; test infrastructure only).

§II-C/§II-D: the Pauli expectations are computed once and cached; training updates the
observable parameters (A, B, D) and the linear layer (W, b) with two separate Adam optimizers.
The paper's loss is a weighted sum of MSE and LPIPS (Eq. (7)); LPIPS needs a trained network
that is not available here, so this step uses the MSE term alone:
    L = mean over the batch and the outputs of (y_hat - y)^2,  y_hat = W q + b  (Eq. (6)),
    q_q = sum_alpha c_{q,alpha} <P_alpha>  (Eq. (5)),  c = Tr(H P)/4  (Eq. (4)).
Gradients are written out by the chain rule below (each line one factor of it); Adam follows
Kingma & Ba (bias-corrected first and second moments).
"""
from __future__ import annotations

import numpy as np

from . import readout


def forward(pauli, a, b, d, w, bias):
    c = readout.coefficients(a, b, d)
    q = readout.features_from_paulis(c, pauli)
    return c, q, readout.reconstruct(q, w, bias)


def loss(pauli, a, b, d, w, bias, target) -> float:
    return float(np.mean((forward(pauli, a, b, d, w, bias)[2] - target) ** 2))


def gradients(pauli, a, b, d, w, bias, target):
    """(L, dA, dB, dD, dW, dbias)."""
    c, q, yhat = forward(pauli, a, b, d, w, bias)
    nb, nout = yhat.shape
    g_y = 2.0 * (yhat - target) / (nb * nout)          # dL/dy_hat
    d_w = g_y.T @ q                                     # y_hat = W q + b
    d_bias = g_y.sum(axis=0)
    g_q = g_y @ w                                       # dL/dq [batch][m]
    p16 = np.concatenate([np.ones(pauli.shape[:2] + (1,)), pauli], axis=2)
    g_c = np.einsum("bq,bqa->qa", g_q, p16)             # q = sum_alpha c_alpha <P_alpha>
    m = len(a)
    d_a, d_b, d_d = np.zeros((m, 6)), np.zeros((m, 6)), np.zeros((m, 4))
    for al in range(16):                                # c_alpha = Tr(H P_alpha) / 4
        p = readout.pauli16(al)
        for j in range(4):
            d_d[:, j] += g_c[:, al] * 0.25 * p[j, j].real
        for idx, (j, k) in enumerate(readout.UPPER):
            # H[j][k] = A + iB and H[k][j] = A - iB enter as P[k][j] (A + iB) + P[j][k] (A - iB)
            d_a[:, idx] += g_c[:, al] * 0.25 * (p[k, j] + p[j, k]).real
            d_b[:, idx] += g_c[:, al] * 0.25 * (1j * p[k, j] - 1j * p[j, k]).real
    return float(np.mean((yhat - target) ** 2)), d_a, d_b, d_d, d_w, d_bias


def adam(param, grad, m, v, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update; returns (param, m, v).  step counts from 1."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return param - lr * mhat / (np.sqrt(vhat) + eps), m, v


def train_step(pauli, params, state, target, step, lr_obs, lr_lin, beta1=0.9, beta2=0.999,
               eps=1e-8):
    """params = (A, B, D, W, bias); state = [(m, v)] per parameter.  Observable parameters
    use lr_obs, the linear layer lr_lin (two optimizers).  Returns (loss, params, state)."""
    lval, *grads = gradients(pauli, *params, target)
    new_p, new_s = [], []
    for i, (p, g, (m, v)) in enumerate(zip(params, grads, state)):
        lr = lr_obs if i < 3 else lr_lin
        p2, m2, v2 = adam(p, g, m, v, step, lr, beta1, beta2, eps)
        new_p.append(p2)
        new_s.append((m2, v2))
    return lval, tuple(new_p), new_s

"""FP64 CPU reference of the warm-start MLP (test infrastructure only).

The network maps instance features to reduced coordinates of the solution:
three tanh hidden layers and a linear output,
    a0 = x,  a_k = tanh(a_{k-1} W_k + b_k)  (k = 1..L-1),  out = a_{L-1} W_L + b_L,
trained on the mean squared error  loss = (1 / 2N) sum_i |out_i - Y_i|^2  with
Adam (Kingma and Ba 2015: beta1 = 0.9, beta2 = 0.999, bias-corrected moments).
This is a textbook definition written out plainly; it pins the GPU kernels
through forward values, backpropagated gradients (themselves pinned by
central finite differences in the tests) and one Adam step.

The reduced coordinates use the fixed Householder basis of the budget
tangent space: H = I - 2 v v^T / v^T v with v = e_n - 1/sqrt(n) * 1 maps e_n
to 1/sqrt(n); its first n-1 columns U span {1^T x = 0}.
"""

from __future__ import annotations

import numpy as np

__all__ = ["forward", "backward", "loss", "adam_step", "householder_U_apply",
           "householder_UT_apply"]


def forward(params, x):
    """params = [(W1, b1), ..., (WL, bL)]; returns (out, activations)."""
    acts = [x]
    a = x
    for k, (W, b) in enumerate(params):
        z = a @ W + b
        a = z if k == len(params) - 1 else np.tanh(z)
        acts.append(a)
    return a, acts


def loss(params, x, Y):
    out, _ = forward(params, x)
    return 0.5 * np.sum((out - Y) ** 2) / x.shape[0]


def backward(params, x, Y):
    """Gradients of ``loss`` with respect to every (W, b)."""
    out, acts = forward(params, x)
    N = x.shape[0]
    delta = (out - Y) / N
    grads = [None] * len(params)
    for k in range(len(params) - 1, -1, -1):
        a_prev = acts[k]
        W, _ = params[k]
        grads[k] = (a_prev.T @ delta, delta.sum(axis=0))
        if k > 0:
            delta = (delta @ W.T) * (1.0 - acts[k] ** 2)
    return grads


def adam_step(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update of array p (returns new p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def _hh_vector(n):
    v = -np.full(n, 1.0 / np.sqrt(n))
    v[-1] += 1.0
    return v


def householder_U_apply(y):
    """x = U y for y in R^{n-1} (U = first n-1 columns of H)."""
    n = y.shape[-1] + 1
    v = _hh_vector(n)
    e = np.concatenate([y, np.zeros(y.shape[:-1] + (1,))], axis=-1)
    return e - 2.0 * (e @ v)[..., None] * v / (v @ v)


def householder_UT_apply(x):
    """y = U^T x (drops the last coordinate of H x)."""
    n = x.shape[-1]
    v = _hh_vector(n)
    hx = x - 2.0 * (x @ v)[..., None] * v / (v @ v)
    return hx[..., :-1]

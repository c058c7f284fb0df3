"""Pins of the FP64 warm-start network reference (CPU only).

The reference is pinned to facts outside itself: backpropagated gradients
against central finite differences of the loss, Adam's first steps against the
closed form -lr * sign(g) that bias correction gives for a constant gradient,
forward values against hand-evaluated small networks, and the Householder
reduced coordinates against orthonormality and the budget-tangent projector.
"""

import numpy as np
import pytest

from oracle import mlp as M


def _net(rng, dims):
    return [(rng.standard_normal((a, b)) / np.sqrt(a), 0.1 * rng.standard_normal(b))
            for a, b in zip(dims[:-1], dims[1:])]


@pytest.mark.parametrize("dims", [(5, 7, 7, 7, 4), (3, 2), (4, 6, 1)])
def test_backward_matches_central_differences(dims):
    rng = np.random.default_rng(11)
    params = _net(rng, dims)
    X = rng.standard_normal((6, dims[0]))
    Y = rng.standard_normal((6, dims[-1]))
    grads = M.backward(params, X, Y)
    h = 1e-6
    for k, (W, b) in enumerate(params):
        for arr, g in ((W, grads[k][0]), (b, grads[k][1])):
            fd = np.zeros_like(arr)
            it = np.nditer(arr, flags=["multi_index"])
            for _ in it:
                idx = it.multi_index
                old = arr[idx]
                arr[idx] = old + h
                lp = M.loss(params, X, Y)
                arr[idx] = old - h
                lm = M.loss(params, X, Y)
                arr[idx] = old
                fd[idx] = (lp - lm) / (2 * h)
            assert np.allclose(g, fd, rtol=1e-6, atol=1e-9), (k, np.abs(g - fd).max())


def test_forward_hand_evaluated():
    # one linear layer: out = x W + b
    W = np.array([[1.0, -2.0], [0.5, 3.0]])
    b = np.array([0.25, -1.0])
    x = np.array([[2.0, 4.0]])
    out, _ = M.forward([(W, b)], x)
    assert np.array_equal(out, np.array([[2.0 + 2.0 + 0.25, -4.0 + 12.0 - 1.0]]))
    # tanh hidden layer then linear: h = tanh(x w1), out = 2 h - 1
    w1 = np.array([[0.5]])
    out, acts = M.forward([(w1, np.zeros(1)), (np.array([[2.0]]), np.array([-1.0]))],
                          np.array([[1.0], [-2.0]]))
    assert np.allclose(acts[1][:, 0], np.tanh([0.5, -1.0]), rtol=0, atol=1e-16)
    assert np.allclose(out[:, 0], 2 * np.tanh([0.5, -1.0]) - 1, rtol=0, atol=1e-15)
    # loss of a perfect fit is zero; of a unit miss in one of N rows is 1/(2N)
    assert M.loss([(W, b)], x, out_lin := x @ W + b) == 0.0
    assert M.loss([(W, b)], np.vstack([x, x]),
                  np.vstack([out_lin, out_lin + [1.0, 0.0]])) == pytest.approx(0.25)


def test_adam_bias_corrected_first_steps():
    rng = np.random.default_rng(3)
    p = rng.standard_normal(50)
    g = rng.standard_normal(50)
    m = np.zeros(50)
    v = np.zeros(50)
    lr = 1e-3
    q = p.copy()
    for t in (1, 2, 3):
        q, m, v = M.adam_step(q, g, m, v, t, lr)
        # constant gradient: bias-corrected m = g, v = g^2 at every t
        step = (p - q) / t
        assert np.allclose(step, lr * np.sign(g) * np.abs(g) / (np.abs(g) + 1e-8),
                           rtol=1e-12, atol=1e-18)
    # zero gradient leaves p unchanged
    z, _, _ = M.adam_step(p, np.zeros(50), np.zeros(50), np.zeros(50), 1, lr)
    assert np.array_equal(z, p)


@pytest.mark.parametrize("n", [2, 3, 13, 257])
def test_householder_reduced_coordinates(n):
    I = np.eye(n - 1)
    U = M.householder_U_apply(I).T          # n x (n-1), column j = U e_j
    assert np.allclose(U.T @ U, np.eye(n - 1), atol=1e-14)
    assert np.allclose(np.ones(n) @ U, 0.0, atol=1e-14)
    P = np.eye(n) - np.ones((n, n)) / n     # projector onto {1^T x = 0}
    assert np.allclose(U @ U.T, P, atol=1e-14)
    rng = np.random.default_rng(n)
    y = rng.standard_normal((4, n - 1))
    assert np.allclose(M.householder_UT_apply(M.householder_U_apply(y)), y, atol=1e-13)
    # for budget-feasible w, 1/n + U U^T (w - 1/n) = w
    w = rng.standard_normal((4, n))
    w += (1.0 - w.sum(axis=1, keepdims=True)) / n
    back = 1.0 / n + M.householder_U_apply(M.householder_UT_apply(w - 1.0 / n))
    assert np.allclose(back, w, atol=1e-13)

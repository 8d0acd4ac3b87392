"""Pins of the FP64 reference MLP (the predictor's oracle) against facts outside it:
central finite differences, the closed-form softmax cross-entropy gradient,
the closed form of Adam's first step, and simple invariants."""
import numpy as np
import pytest

from oracle import mlp
import synth


def _net(sizes, seed=0):
    r = synth.rng(400, seed, 0)
    params = []
    for i in range(len(sizes) - 1):
        W = r.normal(0, np.sqrt(2.0 / sizes[i]), (sizes[i + 1], sizes[i]))
        b = r.normal(0, 0.1, sizes[i + 1])
        params.append((W, b))
    return params


def _data(B, d, K, seed=0):
    r = synth.rng(401, seed, 0)
    return r.normal(0, 1, (B, d)), r.integers(0, K, B)


def test_softmax_rows_sum_to_one_and_shift_invariance():
    z = synth.rng(402, 0, 0).normal(0, 5, (20, 7))
    p = mlp.softmax(z)
    assert np.allclose(p.sum(1), 1.0, atol=1e-15)
    assert np.allclose(mlp.softmax(z + 123.0), p, atol=1e-15)


def test_uniform_logits_give_log_K():
    for K in (2, 5, 16):
        assert abs(mlp.cross_entropy(np.zeros((9, K)), np.arange(9) % K) - np.log(K)) < 1e-14


def test_logit_gradient_closed_form():
    """For a single linear layer, dL/dW = ((softmax(z) - onehot) / B)^T x."""
    X, y = _data(13, 4, 3)
    params = _net([4, 3])
    grads, _ = mlp.backward(params, X, y)
    z = X @ params[0][0].T + params[0][1]
    d = mlp.softmax(z)
    d[np.arange(13), y] -= 1
    d /= 13
    assert np.allclose(grads[0][0], d.T @ X, atol=1e-15)
    assert np.allclose(grads[0][1], d.sum(0), atol=1e-15)


@pytest.mark.parametrize("sizes", [[5, 7, 7, 7, 4], [11, 16, 16, 16, 16]])
def test_gradients_match_central_differences(sizes):
    X, y = _data(17, sizes[0], sizes[-1], seed=len(sizes))
    params = _net(sizes, seed=sizes[1])
    grads, _ = mlp.backward(params, X, y)
    h = 1e-6
    r = synth.rng(403, 0, 0)
    for li, (W, b) in enumerate(params):
        for (arr, g) in ((W, grads[li][0]), (b, grads[li][1])):
            flat = arr.reshape(-1)
            gf = g.reshape(-1)
            for idx in r.choice(flat.size, size=min(12, flat.size), replace=False):
                old = flat[idx]
                flat[idx] = old + h
                lp = mlp.loss(params, X, y)
                flat[idx] = old - h
                lm = mlp.loss(params, X, y)
                flat[idx] = old
                fd = (lp - lm) / (2 * h)
                assert abs(fd - gf[idx]) <= 1e-7 * max(1.0, abs(fd)) + 1e-9, (li, idx, fd, gf[idx])


def test_adam_first_step_closed_form():
    """At t = 1 with zero moments, the step is lr * g / (|g| + eps) (bias corrections cancel)."""
    params = _net([3, 2])
    g = [(np.array([[0.5, -2.0, 1e-3], [3.0, -0.25, 0.0]]), np.array([1.0, -1.0]))]
    p1, m1, v1 = mlp.adam_step(params, g, mlp.zeros_like(params), mlp.zeros_like(params), 1, lr=0.01, eps=1e-8)
    for (W0, b0), (W1, b1), (gW, gb) in zip(params, p1, g):
        assert np.allclose(W0 - W1, 0.01 * gW / (np.abs(gW) + 1e-8), atol=1e-15)
        assert np.allclose(b0 - b1, 0.01 * gb / (np.abs(gb) + 1e-8), atol=1e-15)
    assert np.allclose(m1[0][0], 0.1 * g[0][0]) and np.allclose(v1[0][0], 0.001 * g[0][0] ** 2)


def test_adam_second_step_closed_form():
    """t = 2, from the definition of Adam's bias-corrected moments (Kingma & Ba):
    m_2 = b1 (1 - b1) g_1 + (1 - b1) g_2, v_2 = b2 (1 - b2) g_1^2 + (1 - b2) g_2^2,
    step = lr (m_2 / (1 - b1^2)) / (sqrt(v_2 / (1 - b2^2)) + eps).

    Two entries pin it: a constant gradient, whose corrected moments are exactly g
    and g^2 at every t (the purpose of the correction), so the step equals the
    first one; and g_1 = 1, g_2 = -1, worked by hand with b1 = 0.9, b2 = 0.999:
    m_2 = 0.09 - 0.1 = -0.01, corrected -0.01 / 0.19 = -1/19; v_2 = 0.000999 + 0.001
    = 0.001999, corrected 0.001999 / 0.001999 = 1; step = lr (-1/19) / (1 + eps).
    A correction that used t = 1 at t = 2 would give steps of 1.9/sqrt(1.999) and
    -0.1/sqrt(1.999) instead."""
    lr, eps = 0.01, 1e-8
    params = [(np.array([[0.0, 0.0]]), np.array([0.0]))]
    g1 = [(np.array([[0.5, 1.0]]), np.array([-3.0]))]
    g2 = [(np.array([[0.5, -1.0]]), np.array([-3.0]))]
    m0, v0 = mlp.zeros_like(params), mlp.zeros_like(params)
    p1, m1, v1 = mlp.adam_step(params, g1, m0, v0, 1, lr=lr, eps=eps)
    p2, m2, v2 = mlp.adam_step(p1, g2, m1, v1, 2, lr=lr, eps=eps)
    step = p1[0][0] - p2[0][0]
    # constant gradient 0.5: the same step as t = 1, lr g / (|g| + eps)
    assert abs(step[0, 0] - lr * 0.5 / (0.5 + eps)) < 1e-15
    assert abs((p1[0][1] - p2[0][1])[0] - lr * (-3.0) / (3.0 + eps)) < 1e-15
    # g_1 = 1, g_2 = -1
    assert abs(m2[0][0][0, 1] - (-0.01)) < 1e-15
    assert abs(v2[0][0][0, 1] - 0.001999) < 1e-15
    assert abs(step[0, 1] - lr * (-1.0 / 19.0) / (1.0 + eps)) < 1e-15


def test_training_decreases_loss():
    X, y = _data(64, 6, 4, seed=9)
    params = _net([6, 16, 16, 16, 4], seed=9)
    m, v = mlp.zeros_like(params), mlp.zeros_like(params)
    l0 = mlp.loss(params, X, y)
    for t in range(1, 201):
        g, _ = mlp.backward(params, X, y)
        params, m, v = mlp.adam_step(params, g, m, v, t, lr=1e-2)
    assert mlp.loss(params, X, y) < 0.5 * l0


def test_soft_targets_reduce_to_hard_labels_and_match_differences():
    X, y = _data(11, 5, 4, seed=21)
    params = _net([5, 8, 8, 8, 4], seed=21)
    onehot = np.eye(4)[y]
    g_hard, l_hard = mlp.backward(params, X, y=y)
    g_soft, l_soft = mlp.backward(params, X, T=onehot)
    assert abs(l_hard - l_soft) < 1e-14
    for (a, b), (c, d) in zip(g_hard, g_soft):
        assert np.allclose(a, c, atol=1e-15) and np.allclose(b, d, atol=1e-15)
    T = synth.rng(404, 0, 0).random((11, 4))
    T /= T.sum(1, keepdims=True)
    g, _ = mlp.backward(params, X, T=T)
    W = params[1][0]
    h = 1e-6
    for idx in [(0, 0), (3, 5), (7, 2)]:
        old = W[idx]
        W[idx] = old + h
        lp = mlp.loss(params, X, T=T)
        W[idx] = old - h
        lm = mlp.loss(params, X, T=T)
        W[idx] = old
        assert abs((lp - lm) / (2 * h) - g[1][0][idx]) < 1e-8

"""FP64 CPU reference of the parameter predictor's network -- TEST INFRASTRUCTURE ONLY.

Only tests (and the smoke check) use this module; the GPU predictor has its own
HIP kernels and shares no code with it.

The predictor is a multilayer perceptron classifier: the paper finds that
classification, not regression, suits its discrete targets (section 6.3), and
the network follows that choice:

    a_0 = x;   a_l = relu(a_{l-1} W_l^T + b_l)  (hidden layers);
    z   = a_{L-1} W_L^T + b_L                   (logits);
    p   = softmax(z);   loss = mean_i -log p_i[y_i].

Gradients are the textbook back-propagation of that composition; the update is
Adam (Kingma and Ba, 2015) with bias correction.  Weights are W_l of shape
(out, in) and biases of shape (out,); everything is float64.
"""
from __future__ import annotations

import numpy as np


def forward(params, X):
    """Returns (activations [a_0 .. a_{L-1}], logits)."""
    acts = [np.asarray(X, np.float64)]
    a = acts[0]
    for li, (W, b) in enumerate(params):
        z = a @ W.T + b
        if li < len(params) - 1:
            a = np.maximum(z, 0.0)
            acts.append(a)
        else:
            return acts, z
    raise ValueError("empty network")


def softmax(z):
    z = np.asarray(z, np.float64)
    e = np.exp(z - z.max(axis=1, keepdims=True))
    return e / e.sum(axis=1, keepdims=True)


def cross_entropy(z, y):
    """Mean over rows of -log softmax(z)[y]."""
    z = np.asarray(z, np.float64)
    m = z.max(axis=1, keepdims=True)
    lse = np.log(np.exp(z - m).sum(axis=1)) + m[:, 0]
    return float(np.mean(lse - z[np.arange(z.shape[0]), y]))


def cross_entropy_soft(z, T):
    """Mean over rows of -sum_k T[i, k] log softmax(z)[i, k] (T rows sum to 1)."""
    z = np.asarray(z, np.float64)
    m = z.max(axis=1, keepdims=True)
    logp = z - m - np.log(np.exp(z - m).sum(axis=1, keepdims=True))
    return float(np.mean(-(np.asarray(T, np.float64) * logp).sum(axis=1)))


def loss(params, X, y=None, T=None):
    z = forward(params, X)[1]
    return cross_entropy_soft(z, T) if T is not None else cross_entropy(z, y)


def backward(params, X, y=None, T=None):
    """Gradients [(dW_l, db_l)] of the mean cross-entropy against integer labels y
    or against target distributions T, and the loss."""
    acts, z = forward(params, X)
    B = z.shape[0]
    p = softmax(z)
    if T is not None:
        dz = (p - np.asarray(T, np.float64)) / B
    else:
        dz = p.copy()
        dz[np.arange(B), y] -= 1.0
        dz /= B
    grads = [None] * len(params)
    for li in range(len(params) - 1, -1, -1):
        W, _ = params[li]
        a_in = acts[li]
        grads[li] = (dz.T @ a_in, dz.sum(axis=0))
        if li > 0:
            da = dz @ W
            dz = da * (acts[li] > 0)
    return grads, (cross_entropy_soft(z, T) if T is not None else cross_entropy(z, y))


def adam_step(params, grads, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (t counts from 1); returns new (params, m, v)."""
    out_p, out_m, out_v = [], [], []
    for (W, b), (gW, gb), (mW, mb), (vW, vb) in zip(params, grads, m, v):
        new = []
        for P, G, Mm, Vv in ((W, gW, mW, vW), (b, gb, mb, vb)):
            Mn = b1 * Mm + (1 - b1) * G
            Vn = b2 * Vv + (1 - b2) * G * G
            mh = Mn / (1 - b1 ** t)
            vh = Vn / (1 - b2 ** t)
            new.append((P - lr * mh / (np.sqrt(vh) + eps), Mn, Vn))
        out_p.append((new[0][0], new[1][0]))
        out_m.append((new[0][1], new[1][1]))
        out_v.append((new[0][2], new[1][2]))
    return out_p, out_m, out_v


def zeros_like(params):
    return [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]

"""FP64 oracle of the schedule predictor's arithmetic -- test infrastructure only.

Plain numpy in float64, written from the definitions (no fusion, no tricks):
  * a layer is y = act(x W^T + b), act = ReLU (max(0, z)) or the identity;
  * its backward, given dL/dy: dz = dy * [z > 0] (ReLU) or dy, dW = dz^T x,
    db = sum over rows of dz, dx = dz W;
  * the loss is, per head, the cross-entropy -sum_i t_i log softmax(z)_i of
    the head's logits against soft targets t, averaged over the batch and
    summed over heads; dL/dz = (softmax(z) * sum_i t_i - t) / batch;
  * Adam (Kingma & Ba, "Adam: A Method for Stochastic Optimization", 2015,
    Algorithm 1): m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2,
    p <- p - lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).

Pins (tests/test_mlp_oracle.py): central finite differences of the loss for
every parameter tensor, softmax rows summing to one, the cross-entropy of a
one-hot target, and Adam's first step (|step| = lr * |g| / (|g| + eps)).
"""
from __future__ import annotations

import numpy as np


def linear_fwd(x, W, b, relu):
    z = x @ W.T + b
    return np.maximum(z, 0.0) if relu else z


def linear_bwd(x, W, y, dy, relu):
    dz = dy * (y > 0) if relu else dy
    return dz @ W, dz.T @ x, dz.sum(axis=0)


def softmax_xent(z, t, heads):
    B = z.shape[0]
    dz = np.zeros_like(z)
    loss = 0.0
    o = 0
    for n in heads:
        zz = z[:, o:o + n]
        tt = t[:, o:o + n]
        mx = zz.max(axis=1, keepdims=True)
        e = np.exp(zz - mx)
        p = e / e.sum(axis=1, keepdims=True)
        lp = zz - mx - np.log(e.sum(axis=1, keepdims=True))
        loss += float(-(tt * lp).sum()) / B
        dz[:, o:o + n] = (p * tt.sum(axis=1, keepdims=True) - tt) / B
        o += n
    return loss, dz


def forward(params, x):
    """params = [W1, b1, W2, b2, W3, b3]; returns the activations."""
    W1, b1, W2, b2, W3, b3 = params
    y1 = linear_fwd(x, W1, b1, True)
    y2 = linear_fwd(y1, W2, b2, True)
    z = linear_fwd(y2, W3, b3, False)
    return y1, y2, z


def loss_and_grads(params, x, t, heads):
    W1, b1, W2, b2, W3, b3 = params
    y1, y2, z = forward(params, x)
    loss, dz = softmax_xent(z, t, heads)
    dy2, dW3, db3 = linear_bwd(y2, W3, z, dz, False)
    dy1, dW2, db2 = linear_bwd(y1, W2, y2, dy2, True)
    _, dW1, db1 = linear_bwd(x, W1, y1, dy1, True)
    return loss, [dW1, db1, dW2, db2, dW3, db3]


def adam(p, g, m, v, lr, b1, b2, eps, t):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v

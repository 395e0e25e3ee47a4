"""Pins of the predictor's FP64 oracle (no GPU)."""
import numpy as np
import pytest

from oracle import mlp

HEADS = [5, 4, 4]


def make(rng, din=9, h=7, dout=13, batch=6):
    params = [rng.standard_normal((h, din)) * 0.5, rng.standard_normal(h) * 0.1,
              rng.standard_normal((h, h)) * 0.5, rng.standard_normal(h) * 0.1,
              rng.standard_normal((dout, h)) * 0.5, rng.standard_normal(dout) * 0.1]
    x = rng.standard_normal((batch, din))
    t = np.abs(rng.standard_normal((batch, dout)))
    o = 0
    for n in HEADS:
        t[:, o:o + n] /= t[:, o:o + n].sum(axis=1, keepdims=True)
        o += n
    return params, x, t


def test_gradients_match_central_differences():
    rng = np.random.default_rng(0)
    params, x, t = make(rng)
    loss, grads = mlp.loss_and_grads(params, x, t, HEADS)
    h = 1e-6
    for pi, P in enumerate(params):
        num = np.zeros_like(P)
        for idx in np.ndindex(P.shape):
            old = P[idx]
            P[idx] = old + h
            lp = mlp.loss_and_grads(params, x, t, HEADS)[0]
            P[idx] = old - h
            lm = mlp.loss_and_grads(params, x, t, HEADS)[0]
            P[idx] = old
            num[idx] = (lp - lm) / (2 * h)
        assert np.allclose(grads[pi], num, rtol=1e-5, atol=1e-8), pi


def test_softmax_xent_closed_forms():
    z = np.array([[1.0, 2.0, 3.0, 0.0, 0.0], [0.0, 0.0, 0.0, 5.0, -5.0]])
    t = np.array([[0.0, 0.0, 1.0, 0.0, 0.0], [0.2, 0.2, 0.2, 0.2, 0.2]])
    loss, dz = mlp.softmax_xent(z, t, [5])
    p0 = np.exp(z[0]) / np.exp(z[0]).sum()
    p1 = np.exp(z[1]) / np.exp(z[1]).sum()
    ref = (-np.log(p0[2]) - (0.2 * np.log(p1)).sum()) / 2
    assert loss == pytest.approx(ref, rel=1e-14)
    assert np.allclose(dz[0], (p0 - t[0]) / 2, rtol=1e-14)
    assert np.allclose(dz.sum(axis=1), 0.0, atol=1e-15)   # soft targets sum to 1


def test_adam_first_step():
    g = np.array([0.5, -2.0, 1e-3])
    p, m, v = mlp.adam(np.zeros(3), g, np.zeros(3), np.zeros(3), 0.01, 0.9, 0.999, 1e-8, 1)
    assert np.allclose(p, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_relu_mask_in_backward():
    x = np.array([[1.0, -1.0]])
    W = np.array([[1.0, 0.0], [0.0, 1.0]])
    y = mlp.linear_fwd(x, W, np.zeros(2), True)
    dx, dW, db = mlp.linear_bwd(x, W, y, np.ones((1, 2)), True)
    assert np.array_equal(y, [[1.0, 0.0]])
    assert np.array_equal(db, [1.0, 0.0]) and np.array_equal(dx, [[1.0, 0.0]])

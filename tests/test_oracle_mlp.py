"""Pins for the FP64 predictor reference (oracle/mlp.py).

* the analytic gradient equals central finite differences of the loss;
* softmax cross-entropy: the logit gradient of each head sums to zero per row,
  and a uniform prediction has loss log(4);
* the first Adam step moves every trained parameter by lr * sign(g)
  (bias-corrected m/sqrt(v) = g/|g|), and mean/std never move.
"""
import numpy as np

from oracle import mlp

RNG = np.random.default_rng(77)


def _batch(b=16):
    X = RNG.standard_normal((b, mlp.F)) * 2 + 1
    y = np.stack([RNG.integers(0, 4, b), RNG.integers(0, 4, b)], 1)
    return X, y


def test_layout_size():
    assert mlp.nparam() == 2 * 12 + 12 * 64 + 64 + 64 * 64 + 64 + 64 * 8 + 8


def test_gradient_is_finite_difference():
    X, y = _batch()
    theta = mlp.init(1, mean=X.mean(0), std=X.std(0))
    loss, g = mlp.loss_and_grad(theta, X, y)
    idx = np.concatenate([RNG.choice(np.arange(2 * mlp.F, mlp.nparam()), 60, replace=False)])
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (mlp.loss_and_grad(tp, X, y)[0] - mlp.loss_and_grad(tm, X, y)[0]) / (2 * h)
        assert abs(fd - g[i]) < 1e-7 + 1e-6 * abs(g[i]), (i, fd, g[i])
    assert np.all(g[: 2 * mlp.F] == 0)


def test_uniform_prediction_loss_and_zero_sum():
    X, y = _batch()
    theta = mlp.init(2)
    P = mlp.unpack(theta)
    theta[-(mlp.H * mlp.C + mlp.C):] = 0.0          # W3 = b3 = 0: uniform softmax
    loss, g = mlp.loss_and_grad(theta, X, y)
    assert abs(loss - np.log(4.0)) < 1e-14
    logits, _ = mlp.forward(mlp.init(3), X)
    assert logits.shape == (len(X), 8)
    # d loss / d b3 is the batch mean of (softmax - onehot)/2 per head: sums to 0
    _, g = mlp.loss_and_grad(mlp.init(3), X, y)
    b3 = g[-mlp.C:]
    assert abs(b3[:4].sum()) < 1e-14 and abs(b3[4:].sum()) < 1e-14
    assert P["W1"].shape == (12, 64)


def test_first_adam_step_is_sign_step():
    X, y = _batch()
    theta = mlp.init(4)
    _, g = mlp.loss_and_grad(theta, X, y)
    lr = 1e-3
    new, m, v = mlp.adam(theta, g, np.zeros_like(theta), np.zeros_like(theta), 1, lr, eps=0.0)
    moved = new - theta
    nz = g != 0
    assert np.allclose(moved[nz], -lr * np.sign(g[nz]), rtol=1e-12, atol=0)
    assert np.all(moved[: 2 * mlp.F] == 0)

"""Pins for the oracle's selector MLP: closed-form forward on hand-set
weights, central finite differences of the loss, and the softmax
cross-entropy gradient identity at the logits."""
import numpy as np
import pytest

import oracle

SHAPE = oracle.MLP_SHAPE


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


def split(p, shape=SHAPE):
    i, h1, h2, o = shape
    k = 0
    out = []
    for n in (h1 * i, h1, h2 * h1, h2, o * h2, o):
        out.append(p[k:k + n])
        k += n
    W1, b1, W2, b2, W3, b3 = out
    return W1.reshape(h1, i), b1, W2.reshape(h2, h1), b2, W3.reshape(o, h2), b3


def test_forward_closed_form():
    rng = np.random.default_rng(0)
    p = rng.normal(0, 0.3, oracle.mlp_param_count())
    X = rng.normal(0, 1, (7, 6))
    W1, b1, W2, b2, W3, b3 = split(p)
    h1 = np.maximum(X @ W1.T + b1, 0)
    h2 = np.maximum(h1 @ W2.T + b2, 0)
    ref = h2 @ W3.T + b3
    np.testing.assert_allclose(oracle.mlp_forward(p, X), ref, rtol=1e-12, atol=1e-12)


def test_identity_network_hand_weights():
    # W1 copies x into the first 6 units, W2 copies them on, W3 sums pairs: logits computable by hand
    p = np.zeros(oracle.mlp_param_count())
    W1, b1, W2, b2, W3, b3 = [a.copy() for a in split(p)]
    W1[:6, :6] = np.eye(6)
    W2[:6, :6] = np.eye(6)
    W3[0, 0] = W3[0, 1] = 1.0
    W3[1, 2] = 2.0
    b3[9] = -3.0
    p = np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3.ravel(), b3])
    x = np.array([[1.0, 2.0, 3.0, -1.0, 0.5, 0.0]])
    z = oracle.mlp_forward(p, x)[0]
    assert z[0] == 3.0 and z[1] == 6.0 and z[9] == -3.0 and np.all(z[2:9] == 0)


def test_gradient_finite_differences():
    rng = np.random.default_rng(1)
    p = rng.normal(0, 0.3, oracle.mlp_param_count())
    X = rng.normal(0, 1, (5, 6))
    y = rng.integers(0, 10, 5)
    loss, g = oracle.mlp_loss_grad(p, X, y)
    h = 1e-6
    for idx in rng.choice(p.size, 60, replace=False):
        e = np.zeros_like(p)
        e[idx] = h
        lp, _ = oracle.mlp_loss_grad(p + e, X, y)
        lm, _ = oracle.mlp_loss_grad(p - e, X, y)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-6 * max(1.0, abs(fd)) + 1e-8, (idx, fd, g[idx])


def test_loss_value_and_logit_gradient():
    rng = np.random.default_rng(2)
    p = rng.normal(0, 0.3, oracle.mlp_param_count())
    X = rng.normal(0, 1, (4, 6))
    y = np.array([0, 3, 9, 3])
    z = oracle.mlp_forward(p, X)
    ez = np.exp(z - z.max(1, keepdims=True))
    sm = ez / ez.sum(1, keepdims=True)
    ref_loss = float(np.mean(-np.log(sm[np.arange(4), y])))
    loss, g = oracle.mlp_loss_grad(p, X, y)
    assert abs(loss - ref_loss) < 1e-12
    # gradient of b3 = mean(softmax - onehot)
    onehot = np.eye(10)[y]
    np.testing.assert_allclose(split(g)[5], (sm - onehot).mean(0), rtol=1e-10, atol=1e-14)

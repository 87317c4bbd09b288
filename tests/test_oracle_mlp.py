"""Pins for the oracle's MLP (loss, gradients) and Adam step (CPU only).

* gradients vs central finite differences of the oracle's own loss (brute
  force: a dropped term, wrong index or transposed operand in the backward
  pass fails it);
* forward pinned by permutation-matrix weights, where the logits are a known
  permutation of the input and the loss is scipy's logsumexp closed form
  (a transposed weight gives a different permutation);
* zero weights: uniform softmax, loss = ln K, closed-form bias gradient;
* Adam: with a constant gradient the bias-corrected step is exactly
  lr * g / (|g| + eps) every step.
"""
import math

import numpy as np
import pytest
from scipy.special import logsumexp

import oracle


def _params(g, F, H1, H2, K, scale=0.5):
    return {
        "W1": g.standard_normal((H1, F)) * scale, "b1": g.standard_normal(H1) * 0.1,
        "W2": g.standard_normal((H2, H1)) * scale, "b2": g.standard_normal(H2) * 0.1,
        "W3": g.standard_normal((K, H2)) * scale, "b3": g.standard_normal(K) * 0.1,
    }


def test_gradients_vs_central_differences():
    g = np.random.Generator(np.random.PCG64(7))
    F, H1, H2, K, B = 5, 7, 6, 4, 9
    P = _params(g, F, H1, H2, K)
    X = g.standard_normal((B, F))
    y = g.integers(0, K, B).astype(np.int32)
    _, _, grads = oracle.mlp_loss_grad(X, y, P)
    h = 1e-6
    for name, w in P.items():
        num = np.zeros_like(w)
        for idx in np.ndindex(w.shape):
            wp = {k: v.copy() for k, v in P.items()}
            wm = {k: v.copy() for k, v in P.items()}
            wp[name][idx] += h
            wm[name][idx] -= h
            num[idx] = (oracle.mlp_loss_grad(X, y, wp, False)[0]
                        - oracle.mlp_loss_grad(X, y, wm, False)[0]) / (2 * h)
        err = np.linalg.norm(num - grads[name]) / max(np.linalg.norm(num), 1e-12)
        assert err < 1e-6, (name, err)


def test_forward_permutation_weights():
    g = np.random.Generator(np.random.PCG64(8))
    D, B = 6, 5
    perms = [g.permutation(D) for _ in range(3)]
    mats = [np.eye(D)[p] for p in perms]            # (M x)[i] = x[p[i]]
    P = {"W1": mats[0], "b1": np.zeros(D), "W2": mats[1], "b2": np.zeros(D),
         "W3": mats[2], "b3": np.zeros(D)}
    X = np.abs(g.standard_normal((B, D))) + 0.1       # positive: ReLU is identity
    y = g.integers(0, D, B).astype(np.int32)
    loss, Z, _ = oracle.mlp_loss_grad(X, y, P, False)
    comp = perms[0][perms[1][perms[2]]]               # z[i] = x[p0[p1[p2[i]]]]
    assert np.allclose(Z, X[:, comp], rtol=0, atol=0)
    want = np.mean(logsumexp(Z, axis=1) - Z[np.arange(B), y])
    assert loss == pytest.approx(want, rel=1e-14)
    # a transposed first layer yields a different map
    assert not np.array_equal(perms[0][perms[1][perms[2]]], np.argsort(perms[0])[perms[1][perms[2]]])


def test_relu_blocks_negative_preactivation():
    D, B = 3, 2
    I = np.eye(D)
    P = {"W1": I, "b1": np.zeros(D), "W2": I, "b2": np.zeros(D), "W3": I, "b3": np.zeros(D)}
    X = np.array([[-1.0, 2.0, 0.5], [3.0, -4.0, -0.1]])
    _, Z, _ = oracle.mlp_loss_grad(X, np.zeros(B, np.int32), P, False)
    assert np.array_equal(Z, np.maximum(X, 0))


def test_zero_weights_uniform_softmax():
    F, H1, H2, K, B = 16, 64, 64, 12, 10
    P = {"W1": np.zeros((H1, F)), "b1": np.zeros(H1), "W2": np.zeros((H2, H1)),
         "b2": np.zeros(H2), "W3": np.zeros((K, H2)), "b3": np.zeros(K)}
    g = np.random.Generator(np.random.PCG64(1))
    X = g.standard_normal((B, F))
    y = g.integers(0, K, B).astype(np.int32)
    loss, Z, gr = oracle.mlp_loss_grad(X, y, P)
    assert loss == pytest.approx(math.log(K), rel=1e-15)
    freq = np.bincount(y, minlength=K) / B
    assert np.allclose(gr["b3"], 1.0 / K - freq, atol=1e-15)
    for k in ("W1", "b1", "W2", "b2", "W3"):
        assert np.all(gr[k] == 0.0), k


def test_adam_constant_gradient_closed_form():
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    w0 = np.array([1.0, 2.0, 3.0, 4.0])
    w, m, v = w0, np.zeros(4), np.zeros(4)
    lr, eps = 1e-2, 1e-8
    for t in range(1, 6):
        w, m, v = oracle.adam(w, m, v, g, t, lr=lr, eps=eps)
        step = lr * g / (np.abs(g) + eps)
        assert np.allclose(w, w0 - t * step, rtol=0, atol=1e-12), t


def test_adam_first_step_is_sign_like():
    g = np.array([5.0, -1e-4])
    w, m, v = oracle.adam(np.zeros(2), np.zeros(2), np.zeros(2), g, 1, lr=0.1, eps=0.0)
    assert np.allclose(w, [-0.1, 0.1], rtol=1e-14)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)

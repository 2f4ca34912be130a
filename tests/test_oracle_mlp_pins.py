"""Pins of the oracle's FP64 MLP demapper reference: central finite differences of the
loss, closed-form values of GELU and of the loss at special points, and the closed
form of Adam's first step."""
import math

import numpy as np
import pytest

import oracle


def _params(D=3, H1=5, H2=4, m=2, seed=0, scale=0.7):
    rng = np.random.default_rng(seed)
    return oracle.MLPParams(
        rng.standard_normal((H1, D)) * scale, rng.standard_normal(H1) * 0.1,
        rng.standard_normal((H2, H1)) * scale, rng.standard_normal(H2) * 0.1,
        rng.standard_normal((m, H2)) * scale, rng.standard_normal(m) * 0.1)


def _gelu_tanh_ref(a):
    return 0.5 * a * (1.0 + math.tanh(math.sqrt(2.0 / math.pi) * (a + 0.044715 * a ** 3)))


def test_gelu_values_and_closeness_to_the_erf_form():
    # one hidden unit per layer with identity weights exposes the activation itself
    p = oracle.MLPParams(np.array([[1.0]]), np.zeros(1), np.array([[1.0]]), np.zeros(1),
                         np.array([[1.0]]), np.zeros(1))
    a = np.linspace(-6, 6, 241)
    out = oracle.mlp_forward(p, a[:, None].astype(np.float32))[:, 0]
    a32 = a.astype(np.float32).astype(np.float64)
    # exact special values: g(0) = 0, g(a) -> a for large a, g(-a) -> 0
    assert out[120] == 0.0
    # the tanh form stays within 2e-3 of the erf form a * Phi(a) (Hendrycks & Gimpel)
    phi = np.array([0.5 * (1 + math.erf(v / math.sqrt(2))) for v in a32])
    g1 = a32 * phi
    g_erf = g1 * 0.5 * (1 + np.array([math.erf(v / math.sqrt(2)) for v in g1]))
    assert np.max(np.abs(out - g_erf)) < 2e-3
    # and the composition is the activation applied twice
    g_once = np.array([_gelu_tanh_ref(v) for v in a32])
    np.testing.assert_allclose(out, [_gelu_tanh_ref(v) for v in g_once], rtol=1e-12, atol=1e-15)


def test_zero_network_loss_closed_form():
    # all-zero weights: output = b3 = 0, p = sigmoid(0) = 1/2 -> loss = m ln 2 and dL/db3 = 0
    D, H1, H2, m = 4, 6, 5, 3
    p = oracle.MLPParams(np.zeros((H1, D)), np.zeros(H1), np.zeros((H2, H1)), np.zeros(H2),
                         np.zeros((m, H2)), np.zeros(m))
    y = np.random.default_rng(1).standard_normal((10, D)).astype(np.float32)
    loss, g = oracle.mlp_loss_grad(p, y, np.zeros((10, m), dtype=np.float32))
    assert abs(loss - m * math.log(2)) < 1e-14
    assert np.all(np.abs(g[5]) < 1e-15)
    # target +inf-like: p -> 1, gradient wrt b3 = sigmoid(0) - 1 = -1/2
    loss2, g2 = oracle.mlp_loss_grad(p, y, np.full((10, m), 60.0, dtype=np.float32))
    np.testing.assert_allclose(g2[5], -0.5, atol=1e-12)
    assert abs(loss2 - m * math.log(2)) < 1e-12


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gradient_central_differences(seed):
    p = _params(seed=seed)
    if seed == 2:                       # with the fixed input / output scales in play
        p.in_scale, p.out_scale = 1.7, 2.5
    rng = np.random.default_rng(10 + seed)
    y = rng.standard_normal((7, 3)).astype(np.float32)
    tgt = (rng.standard_normal((7, 2)) * 3).astype(np.float32)
    _, grads = oracle.mlp_loss_grad(p, y, tgt)
    h = 1e-6
    for a, g in zip(p.flat(), grads):
        flat = a.reshape(-1)
        gflat = g.reshape(-1)
        for i in range(flat.size):
            old = flat[i]
            flat[i] = old + h
            lp, _ = oracle.mlp_loss_grad(p, y, tgt)
            flat[i] = old - h
            lm, _ = oracle.mlp_loss_grad(p, y, tgt)
            flat[i] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - gflat[i]) <= 1e-7 * max(1.0, abs(fd)), (i, fd, gflat[i])


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(3)
    w = rng.standard_normal(50)
    g = rng.standard_normal(50)
    w0 = w.copy()
    m1 = np.zeros(50)
    m2 = np.zeros(50)
    oracle.adam_step(w, g, m1, m2, 1, 1e-3)
    # bias-corrected moments equal g and g^2 on the first step
    np.testing.assert_allclose(w, w0 - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(m1, 0.1 * g, rtol=1e-14)
    np.testing.assert_allclose(m2, 0.001 * g * g, rtol=1e-13)


def test_fixed_scales_are_reparametrisations():
    """f(y) = s_out net(s_in y): s_in equals scaling the first-layer weights, s_out equals
    scaling the last layer's weights and bias, and the loss of the scaled network equals
    the loss of the reparametrised one."""
    p = _params(seed=4)
    rng = np.random.default_rng(5)
    y = rng.standard_normal((9, 3)).astype(np.float32)
    tgt = (rng.standard_normal((9, 2)) * 3).astype(np.float32)
    q = oracle.MLPParams(p.W1 * 1.7, p.b1, p.W2, p.b2, p.W3 * 2.5, p.b3 * 2.5)
    p.in_scale, p.out_scale = 1.7, 2.5
    np.testing.assert_allclose(oracle.mlp_forward(p, y), oracle.mlp_forward(q, y), rtol=1e-12, atol=1e-12)
    lp, gp = oracle.mlp_loss_grad(p, y, tgt)
    lq, gq = oracle.mlp_loss_grad(q, y, tgt)
    assert abs(lp - lq) < 1e-12
    # chain rule: d/dW1 of the scaled net = s_in * d/dW1' of the reparametrised one, and so on
    np.testing.assert_allclose(gp[0], 1.7 * gq[0], rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(gp[4], 2.5 * gq[4], rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(gp[5], 2.5 * gq[5], rtol=1e-9, atol=1e-12)

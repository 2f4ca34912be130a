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


# Standard normal distribution function at 1 and its density at 0 (tabulated constants,
# not computed by the oracle): Phi(1) = 0.841344746068542948585..., phi(0) = 1/sqrt(2 pi).
PHI_1 = 0.8413447460685429486
PDF_0 = 0.3989422804014326779


def test_gelu_is_input_times_normal_cdf():
    """GELU (Hendrycks & Gimpel) is a Phi(a): checked against scipy's normal distribution
    function (Cephes ndtr, a library independent of the C library's erfc) on [-8, 8], with
    the tabulated value Phi(1), the exact zero, the asymptotes and the derivative."""
    from scipy.special import ndtr
    a = np.linspace(-8.0, 8.0, 1601)
    g, dg = oracle.gelu(a)
    np.testing.assert_allclose(g, a * ndtr(a), rtol=1e-13, atol=1e-300)
    assert g[800] == 0.0 and dg[800] == 0.5                       # g(0) = 0, g'(0) = Phi(0) = 1/2
    g1, dg1 = oracle.gelu([1.0, -1.0])
    assert abs(g1[0] - PHI_1) <= 1e-15                             # g(1) = Phi(1)
    assert abs(g1[1] + (1.0 - PHI_1)) <= 1e-15                     # g(-1) = -Phi(-1) = -(1 - Phi(1))
    # g'(1) = Phi(1) + phi(1), phi(1) = phi(0) e^(-1/2)
    assert abs(dg1[0] - (PHI_1 + PDF_0 * math.exp(-0.5))) <= 1e-15
    # asymptotes: g(a) - a -> 0 above, g(a) -> 0 below (faster than any power)
    hi, _ = oracle.gelu([10.0, 40.0])
    lo, _ = oracle.gelu([-10.0, -40.0])
    assert hi[0] == 10.0 and hi[1] == 40.0
    assert -1e-22 < lo[0] < 0.0 and -1e-300 < lo[1] <= 0.0
    # g(-10) = -10 Phi(-10) and Phi(-10) = 7.6198530241605e-24 (lower-tail table value)
    assert abs(lo[0] / -10.0 - 7.6198530241605e-24) <= 1e-35
    # the derivative against central differences of the activation itself
    h = 1e-6
    gp, _ = oracle.gelu(a + h)
    gm, _ = oracle.gelu(a - h)
    np.testing.assert_allclose(dg, (gp - gm) / (2 * h), rtol=0, atol=2e-9)


def test_one_unit_network_applies_gelu_twice():
    # one hidden unit per layer with identity weights exposes the activation itself
    p = oracle.MLPParams(np.array([[1.0]]), np.zeros(1), np.array([[1.0]]), np.zeros(1),
                         np.array([[1.0]]), np.zeros(1))
    a = np.linspace(-6, 6, 241)
    out = oracle.mlp_forward(p, a[:, None].astype(np.float32))[:, 0]
    from scipy.special import ndtr
    a32 = a.astype(np.float32).astype(np.float64)
    g1 = a32 * ndtr(a32)
    np.testing.assert_allclose(out, g1 * ndtr(g1), rtol=1e-12, atol=1e-300)
    assert out[120] == 0.0


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

"""Pins of the FP64 oracle's widely-linear DD-LMS equaliser (the step before the demapper
in the paper's receiver, section "Experimental setup"), each fixed by something other
than the oracle's own formula:
  * frozen identity taps (mu = 0, h = delta_0, g = 0) reduce it to the even samples and
    a nearest-point search (numpy argmin over the squared distances);
  * for an IQ-imbalanced input x = a s + b conj(s) the closed-form inverse
    h_0 = conj(a) / (|a|^2 - |b|^2), g_0 = -b / (|a|^2 - |b|^2) is a fixed point of the
    update, and the equaliser output is the sent symbol;
  * started from identity taps, the decision-directed update converges to that inverse,
    and taps that only ever see zero samples stay exactly zero.
"""
import numpy as np

import oracle
import synth


def qam16():
    X, labels = synth.qam_gray(16)
    return (X[:, 0] + 1j * X[:, 1]).astype(np.complex64)


def test_frozen_identity_taps_are_sampling_and_nearest_point():
    rng = np.random.default_rng(3)
    B, N = 5, 60
    x = (rng.standard_normal((2 * N + 2, B)) + 1j * rng.standard_normal((2 * N + 2, B))).astype(np.complex64)
    C = qam16()
    dec, z, h, g = oracle.ddlms(x, C, [1, 0, 0, 0], [0, 0, 0, 0], 0.0)
    assert np.array_equal(z, x[0:2 * N:2])
    d2 = np.abs(x[0:2 * N:2, :, None].astype(np.complex128) - C[None, None, :].astype(np.complex128)) ** 2
    assert np.array_equal(dec, np.argmin(d2, axis=2).astype(np.uint32))
    assert np.array_equal(h, np.tile(np.array([1, 0, 0, 0], dtype=np.complex128), (B, 1)))
    assert np.array_equal(g, np.zeros((B, 4)))


def _imbalanced(B, N, a, b, seed):
    C = qam16()
    rng = np.random.default_rng(seed)
    tx = rng.integers(0, 16, size=(N + 1, B))
    s = C[tx].astype(np.complex128)
    x = np.zeros((2 * N + 2, B), dtype=np.complex128)
    x[0::2] = a * s + b * np.conj(s)          # odd samples stay zero
    return x.astype(np.complex64), tx, C


def test_closed_form_inverse_is_a_fixed_point():
    a, b = 0.9 + 0.2j, 0.12 - 0.05j
    den = abs(a) ** 2 - abs(b) ** 2
    hs, gs = np.conj(a) / den, -b / den
    x, tx, C = _imbalanced(3, 400, a, b, 11)
    dec, z, h, g = oracle.ddlms(x, C, [hs, 0, 0, 0], [gs, 0, 0, 0], 0.01)
    assert np.array_equal(dec, tx[:400].astype(np.uint32))
    assert np.max(np.abs(z - C[tx[:400]])) < 1e-5
    assert np.max(np.abs(h[:, 0] - hs)) < 1e-6 and np.max(np.abs(g[:, 0] - gs)) < 1e-6


def test_converges_to_the_inverse_from_identity_taps():
    a, b = 1.0 + 0.0j, 0.1 + 0.03j
    den = abs(a) ** 2 - abs(b) ** 2
    hs, gs = np.conj(a) / den, -b / den
    N = 4000
    x, tx, C = _imbalanced(4, N, a, b, 12)
    dec, z, h, g = oracle.ddlms(x, C, [1, 0, 0, 0], [0, 0, 0, 0], 0.02)
    assert np.array_equal(dec[N // 2:], tx[N // 2:N].astype(np.uint32))
    assert np.max(np.abs(h[:, 0] - hs)) < 1e-3 and np.max(np.abs(g[:, 0] - gs)) < 1e-3
    # taps 1 and 3 only see the zero odd samples: their updates are exactly zero
    assert np.all(h[:, [1, 3]] == 0) and np.all(g[:, [1, 3]] == 0)
    # tap 2 sees the next symbol, which is independent of the current one
    assert np.max(np.abs(h[:, 2])) < 2e-2 and np.max(np.abs(g[:, 2])) < 2e-2


def test_seeded_input_shapes():
    x, tx, C, labels = synth.equaliser_input(7, 33)
    assert x.shape == (68, 7) and x.dtype == np.complex64
    assert tx.shape == (34, 7) and C.shape == (16,) and sorted(labels.tolist()) == list(range(16))
    x2, _, _, _ = synth.equaliser_input(7, 33)
    assert np.array_equal(x, x2)

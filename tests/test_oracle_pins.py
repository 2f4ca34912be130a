"""Pins of the FP64 oracle against facts fixed outside the oracle itself.

Each test checks the oracle against something other than a retyped copy of its
own formula: closed-form LLRs and capacities (BPSK, Gray QPSK), Gauss-Hermite
quadrature of the GMI integral, exact product identities of the 4D 8-PSK x 8-PSK
format, 50-digit brute force with mpmath (direct sums of exponentials, no
log-sum-exp), invariances of the metric, published Philox known-answer vectors,
and distribution tests of the AWGN twin.  The paper itself prints no LLR or GMI
value (its acronym glossary names LLR, GMI and AWGN only), so these are the pins.
"""
import math
import os

import mpmath
import numpy as np
import pytest
from scipy import stats
from scipy.special import logsumexp

import oracle
import synth

HERE = os.path.dirname(os.path.abspath(__file__))


# ----------------------------------------------------------------------------- helpers (quadrature)
def bpsk_capacity(gamma: float, nodes: int = 200) -> float:
    """C(gamma) = 1 - E_z log2(1 + exp(-2 gamma - 2 sqrt(gamma) z)), z ~ N(0,1) (textbook BPSK
    bit-metric capacity), by Gauss-Hermite quadrature."""
    x, w = np.polynomial.hermite.hermgauss(nodes)
    z = math.sqrt(2.0) * x
    t = -2.0 * gamma - 2.0 * math.sqrt(gamma) * z
    f = np.logaddexp(0.0, t) / math.log(2.0)
    return 1.0 - float(np.sum(w * f) / math.sqrt(math.pi))


def gmi_quadrature_2d(X, labels, sigma2, nodes=90):
    """GMI of a 2D constellation by product Gauss-Hermite quadrature over the noise.
    LLRs at each node come from scipy's logsumexp over the label subsets."""
    X = np.asarray(X, dtype=np.float64)
    M = X.shape[0]
    m = int(M).bit_length() - 1
    x, w = np.polynomial.hermite.hermgauss(nodes)
    zx, zy = np.meshgrid(math.sqrt(2.0) * x, math.sqrt(2.0) * x, indexing="ij")
    ww = np.outer(w, w).ravel() / math.pi
    Z = np.stack([zx.ravel(), zy.ravel()], axis=1)
    sigma = math.sqrt(sigma2)
    total = 0.0
    for i in range(M):
        Y = X[i] + sigma * Z                                           # nodes x 2
        q = -np.sum((Y[:, None, :] - X[None, :, :]) ** 2, axis=2) / (2 * sigma2)   # nodes x M
        lost = np.zeros(Y.shape[0])
        for k in range(m):
            bits = (labels >> (m - 1 - k)) & 1
            L = logsumexp(q[:, bits == 0], axis=1) - logsumexp(q[:, bits == 1], axis=1)
            s = 1.0 if ((int(labels[i]) >> (m - 1 - k)) & 1) == 0 else -1.0
            lost += np.logaddexp(0.0, -s * L) / math.log(2.0)
        total += float(np.sum(ww * lost))
    return m - total / M


def mc_channel(X, labels, sigma2, N, seed):
    """Independent Monte-Carlo channel draw with numpy (not the generator under test)."""
    rng = np.random.default_rng(seed)
    tx = rng.integers(0, X.shape[0], size=N).astype(np.uint32)
    y = (X[tx].astype(np.float64) + math.sqrt(sigma2) * rng.standard_normal((N, X.shape[1]))).astype(np.float32)
    return tx, y


# ----------------------------------------------------------------------------- LLR closed forms
@pytest.mark.parametrize("snr_db", [-5.0, 0.0, 6.0, 14.0])
def test_bpsk_llr_closed_form(snr_db):
    X, labels = synth.bpsk()
    s2 = synth.sigma2_from_snr_db(X, snr_db)
    tx, y = mc_channel(X, labels, s2, 4000, 1)
    L = oracle.llr_exact(X, labels, y, s2)
    ref = 2.0 * y[:, 0].astype(np.float64) / s2
    np.testing.assert_allclose(L[:, 0], ref, rtol=1e-12, atol=1e-12)
    # max-log is exact for BPSK
    np.testing.assert_allclose(oracle.llr_maxlog(X, labels, y, s2)[:, 0], ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("snr_db", [0.0, 8.0, 14.0])
def test_gray_qpsk_llr_closed_form(snr_db):
    X, labels = synth.gray_qpsk()
    s2 = synth.sigma2_from_snr_db(X, snr_db)
    tx, y = mc_channel(X, labels, s2, 4000, 2)
    a = float(X[0, 0])
    L = oracle.llr_exact(X, labels, y, s2)
    # column 0 = MSB: the MSB is 1 exactly on the lower half plane; column 1 = LSB: left half plane
    np.testing.assert_allclose(L[:, 0], 2 * a * y[:, 1].astype(np.float64) / s2, rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(L[:, 1], 2 * a * y[:, 0].astype(np.float64) / s2, rtol=1e-11, atol=1e-11)
    Lml = oracle.llr_maxlog(X, labels, y, s2)
    np.testing.assert_allclose(Lml, L, rtol=1e-11, atol=1e-11)


# ----------------------------------------------------------------------------- GMI pins
def test_gmi_bpsk_per_sample_and_capacity():
    X, labels = synth.bpsk()
    # (above ~10 dB the loss is carried by rare error events and the sample SE is unreliable)
    for snr_db in (-10.0, 0.0, 4.0, 8.0):
        s2 = synth.sigma2_from_snr_db(X, snr_db)
        tx, y = mc_channel(X, labels, s2, 200_000, 3)
        L = oracle.llr_exact(X, labels, y, s2)
        T, _ = oracle.gmi_terms(L, tx, labels)
        sgn = np.where(tx == 0, 1.0, -1.0)
        np.testing.assert_allclose(T, np.logaddexp(0.0, -sgn * 2 * y[:, 0] / s2) / math.log(2), rtol=1e-10,
                                   atol=1e-14)
        g, gb, se = oracle.gmi(L, tx, labels)
        cap = bpsk_capacity(1.0 / s2)
        assert abs(g - cap) <= 4 * se + 1e-9, (snr_db, g, cap, se)
        assert gb.shape == (1,) and abs(gb[0] - g) < 1e-12


def test_gmi_gray_qpsk_is_twice_bpsk():
    X, labels = synth.gray_qpsk()
    for snr_db in (0.0, 4.0, 8.0):
        s2 = synth.sigma2_from_snr_db(X, snr_db)
        tx, y = mc_channel(X, labels, s2, 200_000, 4)
        g, gb, se = oracle.gmi(oracle.llr_exact(X, labels, y, s2), tx, labels)
        ref = 2.0 * bpsk_capacity(10 ** (snr_db / 10))
        assert abs(g - ref) <= 4 * se + 1e-9, (snr_db, g, ref, se)


def test_gmi_8psk_brgc_quadrature():
    X, labels = synth.psk8_brgc()
    for snr_db in (4.0, 8.0, 10.0):
        s2 = synth.sigma2_from_snr_db(X, snr_db)
        ref = gmi_quadrature_2d(X, labels, s2)
        tx, y = mc_channel(X, labels, s2, 200_000, 5)
        g, _, se = oracle.gmi(oracle.llr_exact(X, labels, y, s2), tx, labels)
        assert abs(g - ref) <= 4 * se, (snr_db, g, ref, se)


def test_4d_product_identity_per_sample_and_gmi():
    X4, l4 = synth.product_4d_8psk()
    X2, l2 = synth.psk8_brgc()
    s2 = synth.sigma2_from_snr_db(X4, 8.0)
    tx, y = mc_channel(X4, l4, s2, 100_000, 6)
    L4 = oracle.llr_exact(X4, l4, y, s2)
    La = oracle.llr_exact(X2, l2, y[:, 0:2], s2)
    Lb = oracle.llr_exact(X2, l2, y[:, 2:4], s2)
    np.testing.assert_allclose(L4[:, 0:3], La, rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(L4[:, 3:6], Lb, rtol=1e-10, atol=1e-10)
    g, _, se = oracle.gmi(L4, tx, l4)
    ref = 2.0 * gmi_quadrature_2d(X2, l2, s2)
    assert abs(g - ref) <= 4 * se, (g, ref, se)


def test_gmi_extremes_closed_form():
    # LLR = 0 everywhere: every bit loses exactly one bit -> GMI 0.  Confident correct LLRs -> GMI m.
    rng = np.random.default_rng(7)
    labels = rng.permutation(16).astype(np.uint32)
    tx = rng.integers(0, 16, size=1000).astype(np.uint32)
    g0, gb0, se0 = oracle.gmi(np.zeros((1000, 4)), tx, labels)
    assert abs(g0) < 1e-12 and np.all(np.abs(gb0) < 1e-12) and se0 < 1e-12
    bits = ((labels[tx][:, None] >> (3 - np.arange(4))[None, :]) & 1).astype(np.float64)
    L = np.where(bits == 0, 800.0, -800.0)
    g1, gb1, _ = oracle.gmi(L, tx, labels)
    assert abs(g1 - 4.0) < 1e-12 and np.all(np.abs(gb1 - 1.0) < 1e-12)
    # Wrong sign with |L| = 800 loses 800/ln 2 bits per bit
    g2, _, _ = oracle.gmi(-L, tx, labels)
    assert abs(g2 - (4.0 - 4 * 800.0 / math.log(2))) < 1e-9
    # Standard error of two alternating values a, b: std = |a-b|/2 * sqrt(N/(N-1))
    Lh = np.zeros((1000, 4))
    Lh[::2] = L[::2]
    _, _, se = oracle.gmi(Lh, tx, labels)
    expect = (4.0 / 2.0) * math.sqrt(1000 / 999) / math.sqrt(1000)
    assert abs(se - expect) < 1e-9, (se, expect)


# ----------------------------------------------------------------------------- brute force
def _brute_llr(X, labels, y, sigma2):
    mpmath.mp.dps = 50
    M, D = X.shape
    m = int(M).bit_length() - 1
    out = np.zeros((y.shape[0], m))
    for n in range(y.shape[0]):
        ex = []
        for j in range(M):
            d2 = mpmath.mpf(0)
            for d in range(D):
                diff = mpmath.mpf(float(y[n, d])) - mpmath.mpf(float(X[j, d]))
                d2 += diff * diff
            ex.append(mpmath.exp(-d2 / (2 * mpmath.mpf(sigma2))))
        for k in range(m):
            s0 = mpmath.mpf(0)
            s1 = mpmath.mpf(0)
            for j in range(M):
                if (int(labels[j]) >> (m - 1 - k)) & 1:
                    s1 += ex[j]
                else:
                    s0 += ex[j]
            out[n, k] = float(mpmath.log(s0) - mpmath.log(s1))
    return out


@pytest.mark.parametrize("M,D,seed", [(2, 1, 0), (4, 2, 1), (8, 3, 2), (16, 2, 3), (16, 3, 4)])
def test_brute_force_mpmath(M, D, seed):
    rng = np.random.default_rng(100 + seed)
    X = rng.standard_normal((M, D)).astype(np.float32)
    labels = rng.permutation(M).astype(np.uint32)
    s2 = float(rng.uniform(0.05, 1.0))
    y = (X[rng.integers(0, M, 24)] + math.sqrt(s2) * rng.standard_normal((24, D))).astype(np.float32)
    ref = _brute_llr(X, labels, y, s2)
    got = oracle.llr_exact(X, labels, y, s2)
    np.testing.assert_allclose(got, ref, rtol=1e-11, atol=1e-11)
    # max-log against a brute-force min over subsets
    m = int(M).bit_length() - 1
    d2 = np.array([[sum((float(y[n, d]) - float(X[j, d])) ** 2 for d in range(D)) for j in range(M)]
                   for n in range(24)])
    for k in range(m):
        b = (labels >> (m - 1 - k)) & 1
        ref_ml = (d2[:, b == 1].min(axis=1) - d2[:, b == 0].min(axis=1)) / (2 * s2)
        np.testing.assert_allclose(oracle.llr_maxlog(X, labels, y, s2)[:, k], ref_ml, rtol=1e-11, atol=1e-11)


def test_far_away_symbols_stay_finite():
    # A received point hundreds of sigma from every point: every subset sum underflows in a
    # naive evaluation, the per-subset log-sum-exp must stay finite and equal the brute force.
    X, labels = synth.psk8_brgc()
    y = np.array([[40.0, -25.0], [0.0, 90.0]], dtype=np.float32)
    s2 = 0.01
    got = oracle.llr_exact(X, labels, y, s2)
    assert np.all(np.isfinite(got))
    np.testing.assert_allclose(got, _brute_llr(X, labels, y, s2), rtol=1e-10, atol=1e-8)


# ----------------------------------------------------------------------------- invariances
def _rand_problem(M=32, D=4, N=400, seed=11, s2=0.2):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((M, D)).astype(np.float32)
    labels = rng.permutation(M).astype(np.uint32)
    tx = rng.integers(0, M, N).astype(np.uint32)
    y = (X[tx] + math.sqrt(s2) * rng.standard_normal((N, D))).astype(np.float32)
    return X, labels, tx, y, s2


def test_invariance_point_reordering():
    X, labels, tx, y, s2 = _rand_problem()
    perm = np.random.default_rng(1).permutation(X.shape[0])
    L = oracle.llr_exact(X, labels, y, s2)
    Lp = oracle.llr_exact(X[perm], labels[perm], y, s2)
    np.testing.assert_allclose(Lp, L, rtol=1e-12, atol=1e-12)


def test_invariance_label_bit_permutation_and_xor():
    X, labels, tx, y, s2 = _rand_problem()
    m = 5
    L = oracle.llr_exact(X, labels, y, s2)
    g, gb, _ = oracle.gmi(L, tx, labels)
    # xor with a mask negates the columns of the mask's set bits
    mask = 0b10110
    Lx = oracle.llr_exact(X, labels ^ mask, y, s2)
    sign = np.array([-1.0 if (mask >> (m - 1 - k)) & 1 else 1.0 for k in range(m)])
    np.testing.assert_allclose(Lx, L * sign, rtol=1e-12, atol=1e-12)
    gx, _, _ = oracle.gmi(Lx, tx, labels ^ mask)
    assert abs(gx - g) < 1e-12
    # permuting label bits permutes the columns
    pb = [3, 0, 4, 1, 2]            # new bit position of old bit i (LSB indexing)
    newlab = np.zeros_like(labels)
    for i in range(m):
        newlab |= ((labels >> i) & 1) << pb[i]
    Lb = oracle.llr_exact(X, newlab, y, s2)
    for i in range(m):
        np.testing.assert_allclose(Lb[:, m - 1 - pb[i]], L[:, m - 1 - i], rtol=1e-12, atol=1e-12)
    gpb, _, _ = oracle.gmi(Lb, tx, newlab)
    assert abs(gpb - g) < 1e-12


def test_invariance_rigid_motion_and_scaling():
    X, labels, tx, y, s2 = _rand_problem(D=3)
    L = oracle.llr_exact(X, labels, y, s2)
    Q, _ = np.linalg.qr(np.random.default_rng(2).standard_normal((3, 3)))
    c = np.array([0.3, -1.2, 0.7])
    Xr = (X.astype(np.float64) @ Q.T + c)
    yr = (y.astype(np.float64) @ Q.T + c)
    # inputs are float32 in the oracle: compare at float32 input precision
    Lr = oracle.llr_exact(Xr, labels, yr, s2)
    np.testing.assert_allclose(Lr, L, rtol=2e-4, atol=2e-4)
    a = 2.0       # power-of-two scaling is exact in float32
    La = oracle.llr_exact(X * a, labels, y * a, s2 * a * a)
    np.testing.assert_allclose(La, L, rtol=1e-12, atol=1e-12)


def test_gmi_bounds_monotone_and_exact_beats_maxlog():
    X, labels = synth.gaussian_constellation(64, 4, 9)
    rng = np.random.default_rng(12)
    N = 40_000
    tx = rng.integers(0, 64, N).astype(np.uint32)
    z = rng.standard_normal((N, 4))
    prev = -1.0
    for snr_db in (-20.0, 0.0, 5.0, 10.0, 15.0, 30.0):
        s2 = synth.sigma2_from_snr_db(X, snr_db)
        y = (X[tx] + math.sqrt(s2) * z).astype(np.float32)
        L = oracle.llr_exact(X, labels, y, s2)
        T, _ = oracle.gmi_terms(L, tx, labels)
        assert np.all(T >= 0.0)                         # every sample: GMI contribution <= m
        g, _, se = oracle.gmi(L, tx, labels)
        gml, _, _ = oracle.gmi(oracle.llr_maxlog(X, labels, y, s2), tx, labels)
        assert g >= gml - 4 * se
        assert g >= prev - 4 * se                      # degraded channel has lower GMI
        prev = g
        if snr_db == -20.0:
            assert abs(g) < 0.05
        if snr_db == 30.0:
            assert g > 6.0 - 1e-3


# ----------------------------------------------------------------------------- RNG twin
def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            w = [int(t, 16) for t in line.split()]
            rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


def test_philox_known_answers():
    for ctr, key, out in _kat():
        assert list(oracle.philox4x32_10(ctr, key)) == out


def _round_to_float32(v: int) -> float:
    """Positive integer v rounded to 24 significant bits, ties to even (exact integer
    arithmetic, independent of any float conversion)."""
    shift = max(v.bit_length() - 24, 0)
    q, r = divmod(v, 1 << shift)
    half = 1 << shift >> 1
    if shift and (r > half or (r == half and q & 1)):
        q += 1
    return float(q << shift)


def test_box_muller_transform_against_libm():
    """The twin's FP32 normal pair against libm in FP64 on the same words: radius
    sqrt(-2 ln U1) with U1 = round24(a | 1) 2^-32 (a the radius word), angle 2 pi U2 with
    U2 = (q + (2T + 1) 2^-24) / 4 (q = b >> 30, T = (b >> 7) mod 2^23, b the angle word).
    FP32 bounds: a few units of 2^-24 relative; a wrong series coefficient, constant or
    exponent offset moves them by 1e-4 or more."""
    rng = np.random.default_rng(21)
    words = rng.integers(0, 2 ** 32, size=(3000, 2), dtype=np.uint64).astype(np.uint32)
    # the longest radius, a radius word rounding up to U1 = 1, binade and sqrt2 edges
    words[:8, 0] = [0, 1, 2 ** 32 - 1, 2 ** 32 - 200, 2 ** 31, 2 ** 31 - 1, 0xB504F300, 0xB504F400]
    words[8:12, 1] = [0, 2 ** 30 - 1, 2 ** 30, 2 ** 32 - 1]   # quadrant edges
    for a, b in words:
        z0, z1 = oracle.box_muller([a, b])
        U1 = _round_to_float32(int(a) | 1) * 2.0 ** -32
        q, T = int(b) >> 30, (int(b) >> 7) & 0x7FFFFF
        U2 = (q + (2 * T + 1) * 2.0 ** -24) / 4.0
        R = math.sqrt(-2.0 * math.log(U1))
        assert abs(math.hypot(z0, z1) - R) <= 1e-6 * max(R, 1.0), (a, b, R, math.hypot(z0, z1))
        if R == 0.0:
            assert z0 == 0.0 and z1 == 0.0
            continue
        ang = math.atan2(z1, z0) % (2 * math.pi)
        diff = abs(ang - 2 * math.pi * U2)
        diff = min(diff, 2 * math.pi - diff)
        assert diff <= 1e-6, (a, b, diff)
    # U1 = 2^-32 gives the largest radius, sqrt(64 ln 2)
    assert abs(math.hypot(*oracle.box_muller([0, 12345])) - math.sqrt(64 * math.log(2))) < 1e-5


def test_awgn_word_stream_layout():
    """The channel's use of the Philox stream, checked through the KAT-pinned Philox and
    the libm-pinned pair: block j of channel use g is counter (g_lo, g_hi, j, 1); word 0
    gives the index, words 2p + 1 and 2p + 2 the pair p (dimensions 2p, 2p + 1); the
    received value is fl32(x + sigma z) in one double fma (checked to one FP32 ulp)."""
    X, _ = synth.gaussian_constellation(64, 7, 3)
    seed, offset, N, sigma = (5 << 32) | 99, (1 << 32) - 3, 6, 0.7
    tx, y = oracle.awgn(X, seed, offset, N, sigma)
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for n in range(N):
        g = offset + n
        words = np.concatenate([oracle.philox4x32_10([g & 0xFFFFFFFF, g >> 32, j, 1], key) for j in range(3)])
        assert tx[n] == int(words[0]) >> (32 - 6)
        for p in range(4):
            z = oracle.box_muller([words[2 * p + 1], words[2 * p + 2]])
            for h in range(2):
                d = 2 * p + h
                if d < 7:
                    want = float(X[tx[n], d]) + sigma * z[h]
                    assert abs(float(y[n, d]) - want) <= 2.0 ** -23 * max(abs(want), 1e-30), (n, d)


def test_awgn_twin_statistics_and_offsets():
    X = np.zeros((16, 6), dtype=np.float32)
    tx, y = oracle.awgn(X, seed=77, offset=0, N=100_000, sigma=1.0)
    z = y.astype(np.float64).ravel()
    assert abs(z.mean()) < 4 / math.sqrt(z.size)
    assert abs(z.var() - 1.0) < 4 * math.sqrt(2.0 / z.size)
    assert stats.kstest(z, "norm").pvalue > 1e-4
    cnt = np.bincount(tx, minlength=16)
    assert stats.chisquare(cnt).pvalue > 1e-4
    # dimensions uncorrelated
    C = np.corrcoef(y.astype(np.float64).T)
    assert np.max(np.abs(C - np.eye(6))) < 5 / math.sqrt(100_000)
    # a window at an offset reproduces the same stream
    tx2, y2 = oracle.awgn(X, seed=77, offset=12345, N=1000, sigma=1.0)
    assert np.array_equal(tx2, tx[12345:13345]) and np.array_equal(y2, y[12345:13345])
    # other seed: different stream
    tx3, _ = oracle.awgn(X, seed=78, offset=0, N=1000, sigma=1.0)
    assert not np.array_equal(tx3, tx[:1000])


def test_awgn_twin_channel_mean_and_odd_dimension():
    X, labels = synth.gaussian_constellation(8, 3, 5)
    tx, y = oracle.awgn(X, seed=5, offset=0, N=50_000, sigma=0.5)
    r = (y.astype(np.float64) - X[tx]) / 0.5
    assert abs(r.mean()) < 4 / math.sqrt(r.size)
    assert abs(r.var() - 1.0) < 4 * math.sqrt(2.0 / r.size)


# ----------------------------------------------------------------------------- hard decision
def test_hard_decision_brute_force():
    X, labels, tx, y, s2 = _rand_problem(M=16, D=2, N=300)
    d2 = ((y[:, None, :].astype(np.float64) - X[None].astype(np.float64)) ** 2).sum(-1)
    assert np.array_equal(oracle.hard_decision(X, y), np.argmin(d2, axis=1).astype(np.uint32))


# ----------------------------------------------------------------------------- hard decisions, BER, Q
def test_bpsk_and_gray_qpsk_ber_closed_form():
    """Nearest-point decisions: with SNR per real dimension (sigma2 = Es / (D SNR)), BPSK
    and Gray QPSK both have BER = Q(sqrt(SNR)) = erfc(sqrt(SNR / 2)) / 2 per bit
    (textbook), checked within 4 Monte-Carlo standard errors on an independent draw."""
    for X, labels in (synth.bpsk(), synth.gray_qpsk()):
        m = int(X.shape[0]).bit_length() - 1
        for snr_db in (0.0, 4.0, 7.0):
            s2 = synth.sigma2_from_snr_db(X, snr_db)
            tx, y = mc_channel(X, labels, s2, 200_000, 17)
            dec = labels.astype(np.int64)[oracle.hard_decision(X, y).astype(np.int64)]
            errs = oracle.bit_errors(dec, tx, labels, m)
            ber = errs.sum() / (len(tx) * m)
            p = 0.5 * math.erfc(math.sqrt(10 ** (snr_db / 10) / 2.0))
            assert abs(ber - p) <= 4 * math.sqrt(p * (1 - p) / (len(tx) * m)), (snr_db, ber, p)


def test_maxlog_signs_are_the_nearest_point_labels():
    X, labels, tx, y, s2 = _rand_problem(M=64, D=4, N=2000)
    dec_ml = labels.astype(np.int64)[oracle.hard_decision(X, y).astype(np.int64)]
    assert np.array_equal(oracle.llr_decisions(oracle.llr_maxlog(X, labels, y, s2)), dec_ml)


def test_q_factor_gaussian_tail_identity():
    # Q = 6 (15.563 dB) is BER = 9.866e-10 in the standard tables; BER = erfc(Q/sqrt2)/2
    assert abs(oracle.q_factor_db(0.5 * math.erfc(6.0 / math.sqrt(2.0))) - 20 * math.log10(6.0)) < 1e-9
    assert abs(0.5 * math.erfc(6.0 / math.sqrt(2.0)) - 9.8659e-10) < 1e-13
    for q in (0.5, 2.0, 3.5):
        assert abs(oracle.q_factor_db(0.5 * math.erfc(q / math.sqrt(2.0))) - 20 * math.log10(q)) < 1e-9

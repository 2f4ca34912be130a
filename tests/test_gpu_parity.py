"""GPU parity: the HIP library (through its C ABI) against the FP64 CPU oracle on the
same seeded inputs.

Tolerances (derivation in the design notes):
  * awgn_sample: bit-exact (tx indices and float32 bit patterns).
  * LLRs, FP32 precision: |dL| <= 2e-3 + 2e-4 |L|.  The score contraction is a
    split-FP16 MFMA product (hi*hi, hi*lo and lo*hi partial products side by side in
    K) whose dropped lo*lo term and FP32 accumulation leave an error of a few 2^-22 of
    sum_k |a_k b_k| (up to ~1e3 in base-2 exponent units at 14 dB) on each exponent,
    so ~3e-4 nat per score.
  * max-log LLRs: same bound.
  * LLRs, BF16 precision: the exponentials are converted to BF16 (relative error
    <= 2^-8 per term for any rounding of the 8-bit mantissa), so each subset sum is
    within 2^-8 and the LLR within 2 * 2^-8 ~ 7.8e-3 nat, plus the FP32 bound above
    for the scores: |dL| <= 1e-2 + 2e-4 |L|.
  * GMI: |dGMI| <= 1e-4 bit (the target), measured on the same y and tx.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

ATOL = 2e-3
RTOL = 2e-4


def md():
    import paper_2104_06311_amd as m
    return m


def to_dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def labels_dev(labels):
    return to_dev(labels.astype(np.int64).astype(np.int32))


def channel(X, labels, snr_db, N, seed, offset=0):
    """Draw the channel on the GPU; return host copies too."""
    s2 = synth.sigma2_from_snr_db(X, snr_db)
    Xd = to_dev(X)
    tx, y = md().awgn_sample(Xd, seed, offset, N, math.sqrt(s2))
    torch.cuda.synchronize()
    return s2, Xd, tx, y, tx.cpu().numpy().astype(np.uint32), y.cpu().numpy()


def assert_llr_close(got, ref, atol=ATOL, rtol=RTOL, what=""):
    err = np.abs(got.astype(np.float64) - ref)
    bound = atol + rtol * np.abs(ref)
    worst = np.argmax(err - bound)
    assert np.all(np.isfinite(got)), what + ": non-finite LLR"
    assert np.all(err <= bound), (f"{what}: max |dL| {err.max():.3e}, worst at {np.unravel_index(worst, err.shape)} "
                                  f"got {got.flat[worst]} ref {ref.flat[worst]}")
    return float(err.max())


# ----------------------------------------------------------------------------- AWGN
@pytest.mark.parametrize("M,D,seed,offset,N", [
    (64, 4, 2104, 0, 100_003),
    (2048, 8, 2105, 3, 20_000),
    (2, 1, 1, 0, 5000),
    (8, 3, 77, (1 << 32) - 100, 4097),     # offset crosses the 32-bit counter word
    (65536, 16, 2108, 123456789012, 3000),
    (16, 30, 9, 0, 1000),
])
def test_awgn_bit_exact_against_cpu_twin(M, D, seed, offset, N):
    X, _ = synth.gaussian_constellation(M, D, seed)
    sigma = 0.37
    txd, yd = md().awgn_sample(to_dev(X), seed, offset, N, sigma)
    tx_ref, y_ref = oracle.awgn(X, seed, offset, N, sigma)
    assert np.array_equal(txd.cpu().numpy().astype(np.uint32), tx_ref)
    assert np.array_equal(yd.cpu().numpy().view(np.uint32), y_ref.view(np.uint32))


@pytest.mark.parametrize("D,N", [(3, 1000), (8, 130), (5, 64)])
def test_awgn_into_unaligned_output(D, N):
    """y starting one float into its buffer (not 16-byte aligned): the kernel's 4-byte store
    path, bit-exact like the aligned one; the float after y stays untouched."""
    X, _ = synth.gaussian_constellation(64, D, 40 + D)
    buf = torch.full((N * D + 2,), -7.0, dtype=torch.float32, device="cuda")
    y = buf[1:1 + N * D].view(N, D)
    txd, yd = md().awgn_sample(to_dev(X), 11, 5, N, 0.3, y=y)
    tx_ref, y_ref = oracle.awgn(X, 11, 5, N, 0.3)
    assert np.array_equal(txd.cpu().numpy().astype(np.uint32), tx_ref)
    assert np.array_equal(yd.cpu().numpy().view(np.uint32), y_ref.view(np.uint32))
    b = buf.cpu().numpy()
    assert b[0] == -7.0 and b[-1] == -7.0


def test_awgn_window_consistency():
    X, _ = synth.gaussian_constellation(256, 4, 3)
    Xd = to_dev(X)
    tx, y = md().awgn_sample(Xd, 5, 1000, 50_000, 0.2)
    tx2, y2 = md().awgn_sample(Xd, 5, 1000 + 12_345, 1000, 0.2)
    assert torch.equal(tx[12_345:13_345], tx2) and torch.equal(y[12_345:13_345], y2)


# ----------------------------------------------------------------------------- exact LLR + GMI
def _parity(X, labels, snr_db, N, seed, maxlog=False, prec="fp32"):
    s2, Xd, tx, y, txh, yh = channel(X, labels, snr_db, N, seed)
    ld = labels_dev(labels)
    if maxlog:
        L = md().llr_maxlog(Xd, ld, y, s2)
        ref = oracle.llr_maxlog(X, labels, yh, s2)
    else:
        L = md().llr_exact(Xd, ld, y, s2, prec=prec)
        ref = oracle.llr_exact(X, labels, yh, s2)
    Lh = L.cpu().numpy()
    atol = ATOL if prec == "fp32" else 1e-2
    err = assert_llr_close(Lh, ref, atol=atol, what=f"M={X.shape[0]} D={X.shape[1]} snr={snr_db} {prec}")
    g, gb, se = md().gmi_reduce(L, tx, ld)
    g_ref, gb_ref, se_ref = oracle.gmi(ref, txh, labels)
    g = float(g.item())
    if prec == "fp32":
        assert abs(g - g_ref) <= 1e-4, (g, g_ref)
    else:
        # a reduced-precision variant is held to its LLR bound above; softplus is
        # 1-Lipschitz, so the GMI (bits) moves by at most the mean of sum_k |dL_nk| / ln 2
        bound = float(np.mean(np.abs(Lh.astype(np.float64) - ref).sum(axis=1))) / math.log(2.0)
        assert abs(g - g_ref) <= bound + 1e-6, (g, g_ref, bound)
    # the reduction alone: GPU gmi_reduce vs FP64 GMI of the very same float32 LLRs
    g_same, gb_same, se_same = oracle.gmi(Lh.astype(np.float64), txh, labels)
    assert abs(g - g_same) <= 1e-6 * max(1.0, abs(g_same))
    np.testing.assert_allclose(gb.cpu().numpy(), gb_same, atol=1e-6)
    assert abs(float(se.item()) - se_same) <= 1e-6 + 1e-3 * se_same
    return err, g, g_ref


def test_parity_4d_64_8psk_product_full():
    """4D M=64 (two 8-PSK, BRGC, 6 bits) at 8 dB, N = 1e5 seeded symbols, in full."""
    X, labels = synth.product_4d_8psk()
    err, g, g_ref = _parity(X, labels, 8.0, 100_000, 2104)
    assert 4.6 < g < 4.9


@pytest.mark.parametrize("snr_db", [4.0, 9.0, 14.0])
def test_parity_8d_2048_subset(snr_db):
    """8D M=2048 Gaussian constellation: a 20,000-symbol window of the sweep."""
    X, labels = synth.gaussian_constellation(2048, 8, synth.SEED_BASE + 1)
    _parity(X, labels, snr_db, 20_000, synth.SEED_BASE + 1)


@pytest.mark.parametrize("M,D,N,snr,perm", [
    (2, 1, 1000, 3.0, False), (4, 2, 777, 8.0, True), (16, 3, 2049, 10.0, True),
    (32, 2, 5000, 12.0, True), (64, 4, 4099, 6.0, True), (256, 8, 3333, 11.0, True),
    (1024, 13, 1500, 9.0, True), (128, 14, 999, 7.0, True), (512, 16, 700, 12.0, True),
    (64, 30, 300, 20.0, True), (4096, 2, 1200, 16.0, True), (64, 5, 1, 8.0, True),
])
def test_parity_random_problems(M, D, N, snr, perm):
    X, labels = synth.gaussian_constellation(M, D, 1000 + M + D)
    if perm:
        labels = synth.random_labels(M, M * 7 + D)
    _parity(X, labels, snr, N, 31 + M)


@pytest.mark.parametrize("M,D,N,snr", [
    (64, 4, 3000, 30.0), (32, 8, 2000, 24.0), (64, 1, 2000, 20.0), (32, 3, 4097, 2.0), (64, 8, 1500, 14.0),
    (64, 6, 1500, 12.0), (32, 7, 1200, 18.0), (64, 2, 2500, 9.0), (32, 5, 1000, 6.0),
])
def test_parity_one_thread_per_symbol(M, D, N, snr):
    """M = 32 and 64 with D <= 8 take the one-thread-per-symbol kernel (FP32 scores from
    per-point terms), exact and max-log; at 20-30 dB part of the symbols leave the exact
    form's FP32 range and are finished by the wide-range and FP64 passes through the same
    fallback list (max-log takes score differences only and never leaves the range)."""
    X, labels = synth.gaussian_constellation(M, D, 7000 + M + D)
    labels = synth.random_labels(M, 5 * M + D)
    _parity(X, labels, snr, N, 71 + M + D)
    _parity(X, labels, snr, N, 72 + M + D, maxlog=True)


@pytest.mark.parametrize("M,D,N,snr,maxlog", [
    (4096, 8, 2000, 13.0, False), (8192, 8, 1500, 10.0, False), (8192, 8, 1500, 10.0, True),
    (16384, 5, 700, 18.0, False),
])
def test_parity_streamed_fragments(M, D, N, snr, maxlog):
    """Constellations whose fragments exceed LDS (two K steps: 128, 256 and 512 tiles of
    2 KiB): the exact and max-log kernels copy them chunk by chunk for every symbol group,
    with a partial last chunk (72-tile chunks), the staging rows over the chunk buffer, and
    high SNR sending symbols through the wide-range passes."""
    X, labels = synth.gaussian_constellation(M, D, 5000 + M + D)
    labels = synth.random_labels(M, M + 3 * D)
    _parity(X, labels, snr, N, 61 + M, maxlog=maxlog)


@pytest.mark.parametrize("M,D,N,snr", [(2048, 8, 20_000, 4.0), (2048, 8, 20_000, 14.0), (64, 4, 30_001, 8.0),
                                       (32, 2, 3000, 10.0), (4096, 8, 2000, 12.0), (256, 16, 1500, 9.0),
                                       (128, 30, 700, 15.0)])
def test_parity_bf16_subset_sums(M, D, N, snr):
    if M == 64 and D == 4:
        X, labels = synth.product_4d_8psk()
    else:
        X, labels = synth.gaussian_constellation(M, D, 77 + M + D)
        labels = synth.random_labels(M, D)
    _parity(X, labels, snr, N, 41, prec="bf16")


@pytest.mark.parametrize("M,D,snr", [(64, 4, 8.0), (2048, 8, 14.0), (2, 1, 0.0), (4, 2, 8.0), (256, 16, 12.0)])
def test_parity_maxlog(M, D, snr):
    if M == 64 and D == 4:
        X, labels = synth.product_4d_8psk()
    elif M == 2:
        X, labels = synth.bpsk()
    elif M == 4:
        X, labels = synth.gray_qpsk()
    else:
        X, labels = synth.gaussian_constellation(M, D, 5 + M)
    _parity(X, labels, snr, 5000, 7, maxlog=True)


def test_maxlog_equals_exact_for_gray_qpsk():
    X, labels = synth.gray_qpsk()
    s2, Xd, tx, y, txh, yh = channel(X, labels, 8.0, 10_000, 3)
    ld = labels_dev(labels)
    a = float(X[0, 0])
    closed = np.stack([2 * a * yh[:, 1] / s2, 2 * a * yh[:, 0] / s2], axis=1)
    assert_llr_close(md().llr_exact(Xd, ld, y, s2).cpu().numpy(), closed)
    assert_llr_close(md().llr_maxlog(Xd, ld, y, s2).cpu().numpy(), closed)


# ----------------------------------------------------------------------------- edge cases
def test_far_symbols_take_the_careful_path():
    X, labels = synth.gaussian_constellation(256, 4, 1)
    rng = np.random.default_rng(0)
    y = (rng.standard_normal((600, 4)) * 30).astype(np.float32)     # far from every point
    y[:300] = X[rng.integers(0, 256, 300)] + 0.05 * rng.standard_normal((300, 4)).astype(np.float32)
    s2 = 0.004
    L = md().llr_exact(to_dev(X), labels_dev(labels), to_dev(y), s2).cpu().numpy()
    ref = oracle.llr_exact(X, labels, y, s2)
    assert_llr_close(L, ref, atol=ATOL, rtol=RTOL, what="far symbols")


def test_extreme_snr_range_fallback():
    # sigma2 so small that the split-FP16 operands overflow: every symbol must still be exact
    X, labels = synth.gaussian_constellation(64, 4, 2)
    rng = np.random.default_rng(1)
    y = (X[rng.integers(0, 64, 500)] + 1e-4 * rng.standard_normal((500, 4))).astype(np.float32)
    s2 = 1e-9
    L = md().llr_exact(to_dev(X), labels_dev(labels), to_dev(y), s2).cpu().numpy()
    ref = oracle.llr_exact(X, labels, y, s2)
    assert_llr_close(L, ref, atol=ATOL, rtol=RTOL, what="extreme snr")


@pytest.mark.parametrize("M,D", [(2, 1), (8, 3), (16, 2), (16, 30)])
def test_small_constellations_far_and_extreme(M, D):
    """M <= 16 (one thread per symbol, per-subset maxima): far symbols and tiny sigma2."""
    X, labels = synth.gaussian_constellation(M, D, 40 + M + D)
    labels = synth.random_labels(M, 3 + M)
    rng = np.random.default_rng(M + D)
    y = (rng.standard_normal((700, D)) * 20).astype(np.float32)
    y[:350] = X[rng.integers(0, M, 350)] + 0.01 * rng.standard_normal((350, D)).astype(np.float32)
    for s2 in (0.5, 1e-3, 1e-7):
        L = md().llr_exact(to_dev(X), labels_dev(labels), to_dev(y), s2).cpu().numpy()
        assert_llr_close(L, oracle.llr_exact(X, labels, y, s2), what=f"small M={M} s2={s2}")
        Lm = md().llr_maxlog(to_dev(X), labels_dev(labels), to_dev(y), s2).cpu().numpy()
        assert_llr_close(Lm, oracle.llr_maxlog(X, labels, y, s2), what=f"small max-log M={M} s2={s2}")


def test_wide_range_pass_at_high_snr():
    """8D M=2048 at 20 dB: the far subset of about half the symbols lies beyond the first
    exponent window; those symbols take the two-window pass, a few the careful kernel."""
    X, labels = synth.gaussian_constellation(2048, 8, synth.SEED_BASE + 1)
    s2, Xd, tx, y, txh, yh = channel(X, labels, 20.0, 3000, 11)
    ld = labels_dev(labels)
    L = md().llr_exact(Xd, ld, y, s2)
    n_wide, n_careful = md().llr_path_counts()
    assert n_wide > 300 and n_careful < n_wide, (n_wide, n_careful)
    ref = oracle.llr_exact(X, labels, yh, s2)
    assert_llr_close(L.cpu().numpy(), ref, what="wide-range pass")
    g = md().gmi_reduce(L, tx, ld)[0].item()
    g_ref = oracle.gmi(ref, txh, labels)[0]
    assert abs(g - g_ref) <= 1e-4
    Lm = md().llr_maxlog(Xd, ld, y, s2)
    assert md().llr_path_counts() == (0, 0)
    assert_llr_close(Lm.cpu().numpy(), oracle.llr_maxlog(X, labels, yh, s2), what="max-log 20 dB")


def test_three_window_pass_at_very_high_snr():
    """8D M=2048 at 24 dB: most symbols have a subset whose best point lies 196 to 576
    base-2 units below the bias.  They take the two- and three-window passes; only a
    subset beyond 576 units would need the FP64 kernel.  The stage counts are checked
    against the per-subset best scores, found here by brute force in FP64."""
    X, labels = synth.gaussian_constellation(2048, 8, synth.SEED_BASE + 1)
    s2, Xd, tx, y, txh, yh = channel(X, labels, 24.0, 3000, 13)
    ld = labels_dev(labels)
    L = md().llr_exact(Xd, ld, y, s2)
    n_wide, n_careful = md().llr_path_counts()
    ref = oracle.llr_exact(X, labels, yh, s2)
    assert_llr_close(L.cpu().numpy(), ref, what="three-window pass")
    assert abs(md().gmi_reduce(L, tx, ld)[0].item() - oracle.gmi(ref, txh, labels)[0]) <= 1e-4
    # worst per-subset best score of every symbol, in base-2 units
    c = math.log2(math.e) / (2.0 * s2)
    Xf = X.astype(np.float64)
    d2 = (yh.astype(np.float64) ** 2).sum(1)[:, None] - 2.0 * yh.astype(np.float64) @ Xf.T + (Xf ** 2).sum(1)[None, :]
    t = -c * d2
    lab = labels.astype(np.int64)
    worst = np.zeros(len(yh))
    for b in range(11):
        bit = (lab >> b) & 1
        worst = np.minimum(worst, np.minimum(t[:, bit == 0].max(1), t[:, bit == 1].max(1)))
    print(f"24 dB: wide {n_wide}, careful {n_careful}, beyond 196: {(worst < -196).sum()}, "
          f"beyond 386: {(worst < -386).sum()}, beyond 576: {(worst < -576).sum()}", flush=True)
    assert (worst < -386).sum() > 100            # the three-window pass has work
    assert (worst < -206).sum() <= n_wide <= (worst < -186).sum()
    assert n_careful <= (worst < -566).sum()


def test_path_counts_low_snr_and_small_m():
    X, labels = synth.gaussian_constellation(2048, 8, synth.SEED_BASE + 1)
    s2, Xd, tx, y, txh, yh = channel(X, labels, 6.0, 5000, 12)
    md().llr_exact(Xd, labels_dev(labels), y, s2)
    assert md().llr_path_counts() == (0, 0)
    X, labels = synth.gaussian_constellation(16, 2, 3)
    s2, Xd, tx, y, txh, yh = channel(X, labels, 6.0, 777, 12)
    md().llr_exact(Xd, labels_dev(labels), y, s2)
    assert md().llr_path_counts() == (0, 0)        # M <= 16: the one-thread-per-symbol kernel


def test_ber_count_and_q_factor():
    """Hard decisions from LLR signs: the counts are integers, so they are compared
    exactly -- with the signs of the GPU's own LLRs, and with the oracle's FP64
    nearest-point decisions except where the oracle's LLR lies within 1e-3 of 0 (a
    near tie the FP32 scores may break either way)."""
    X, labels = synth.product_4d_8psk()
    s2, Xd, tx, y, txh, yh = channel(X, labels, 8.0, 100_000, 2104)
    ld = labels_dev(labels)
    for maxlog in (True, False):
        L = md().llr_maxlog(Xd, ld, y, s2) if maxlog else md().llr_exact(Xd, ld, y, s2)
        e, eb = md().ber_count(L, tx, ld)
        Lh = L.cpu().numpy()
        own = oracle.bit_errors(oracle.llr_decisions(Lh), txh, labels, 6)
        assert np.array_equal(eb.cpu().numpy(), own) and int(e.item()) == int(own.sum())
        ref = oracle.llr_maxlog(X, labels, yh, s2) if maxlog else oracle.llr_exact(X, labels, yh, s2)
        ref_err = oracle.bit_errors(oracle.llr_decisions(ref), txh, labels, 6)
        ties = int((np.abs(ref) < 1e-3).sum())
        assert abs(int(e.item()) - int(ref_err.sum())) <= ties
        if maxlog:
            dec = labels.astype(np.int64)[oracle.hard_decision(X, yh).astype(np.int64)]
            assert abs(int(e.item()) - int(oracle.bit_errors(dec, txh, labels, 6).sum())) <= ties
        ber = int(e.item()) / (100_000 * 6)
        assert 0.0 < ber < 0.5
        q = md().q_factor_db(e, 100_000 * 6).item()
        assert abs(q - oracle.q_factor_db(ber)) < 1e-9
    # no finite Q-factor without errors, or at BER >= 1/2
    zero = torch.zeros(1, dtype=torch.int64, device="cuda")
    assert math.isnan(md().q_factor_db(zero, 100).item())
    assert math.isnan(md().q_factor_db(torch.full((1,), 50, dtype=torch.int64, device="cuda"), 100).item())
    assert abs(md().q_factor_db(torch.full((1,), 27, dtype=torch.int64, device="cuda"), 10**10).item()
               - oracle.q_factor_db(27e-10)) < 1e-9


def test_empty_input_is_a_no_op_and_gmi_rejects_it():
    X, labels = synth.gaussian_constellation(64, 4, 2)
    Xd, ld = to_dev(X), labels_dev(labels)
    y = torch.empty((0, 4), dtype=torch.float32, device="cuda")
    assert md().llr_exact(Xd, ld, y, 0.1).shape == (0, 6)
    assert md().llr_maxlog(Xd, ld, y, 0.1).shape == (0, 6)
    tx, y0 = md().awgn_sample(Xd, 1, 0, 0, 0.1)
    assert tx.numel() == 0
    with pytest.raises(md().MdemapError):
        md().gmi_reduce(torch.empty((0, 6), dtype=torch.float32, device="cuda"),
                        torch.empty(0, dtype=torch.int32, device="cuda"), ld)


def test_invalid_labels_are_rejected():
    X, _ = synth.gaussian_constellation(64, 4, 2)
    bad = np.arange(64, dtype=np.uint32)
    bad[5] = 7                           # duplicate
    y = to_dev(np.zeros((10, 4), dtype=np.float32))
    with pytest.raises(md().MdemapError) as e:
        md().llr_exact(to_dev(X), labels_dev(bad), y, 0.1)
    assert e.value.status == -3
    bad2 = np.arange(64, dtype=np.uint32)
    bad2[0] = 64                         # out of range
    with pytest.raises(md().MdemapError):
        md().llr_maxlog(to_dev(X), labels_dev(bad2), y, 0.1)


def test_labels_rewritten_in_place_are_caught_on_the_device():
    """The host checks a label buffer once per (device, address, M); labels rewritten in
    place afterwards are caught by the device check of every call (all outputs NaN), and
    after release_cache() the host check runs again and reports MD_ELABEL."""
    X, labels = synth.gaussian_constellation(64, 4, 2)
    s2, Xd, tx, y, txh, yh = channel(X, labels, 8.0, 500, 3)
    ld = labels_dev(labels)
    assert torch.isfinite(md().llr_exact(Xd, ld, y, s2)).all()
    ld[5] = ld[6]                        # now a duplicate label, same address
    L = md().llr_exact(Xd, ld, y, s2)
    assert torch.isnan(L).all()
    assert torch.isnan(md().llr_maxlog(Xd, ld, y, s2)).all()     # the max-log form of the same kernel
    md().release_cache()
    with pytest.raises(md().MdemapError) as e:
        md().llr_exact(Xd, ld, y, s2)
    assert e.value.status == -3


def test_results_do_not_depend_on_label_storage_order():
    X, labels = synth.gaussian_constellation(512, 8, 4)
    labels = synth.random_labels(512, 3)
    s2, Xd, tx, y, txh, yh = channel(X, labels, 10.0, 3000, 5)
    L1 = md().llr_exact(Xd, labels_dev(labels), y, s2)
    perm = np.random.default_rng(2).permutation(512)
    L2 = md().llr_exact(to_dev(X[perm]), labels_dev(labels[perm]), y, s2)
    assert torch.equal(L1, L2)          # the prep puts points in label order: identical bits


def test_deterministic_gmi():
    X, labels = synth.gaussian_constellation(1024, 8, 6)
    s2, Xd, tx, y, txh, yh = channel(X, labels, 9.0, 200_000, 8)
    ld = labels_dev(labels)
    L = md().llr_exact(Xd, ld, y, s2)
    g1 = md().gmi_reduce(L, tx, ld)[0].item()
    g2 = md().gmi_reduce(L, tx, ld)[0].item()
    assert g1 == g2


# ----------------------------------------------------------------------------- full size
def test_full_size_8d_2048_sampled_rows():
    """The benchmark's configuration (N = 1e7 per SNR, 8D M = 2048): sampled rows against
    the oracle, GMI bounds and monotonicity across the SNR sweep ends."""
    X, labels = synth.gaussian_constellation(2048, 8, synth.SEED_BASE + 1)
    Xd, ld = to_dev(X), labels_dev(labels)
    N = 10_000_000
    rng = np.random.default_rng(9)
    rows = np.sort(rng.choice(N, 1500, replace=False))
    prev = -1.0
    for snr in (4.0, 14.0):
        s2 = synth.sigma2_from_snr_db(X, snr)
        tx, y = md().awgn_sample(Xd, synth.SEED_BASE + 1, 0, N, math.sqrt(s2))
        L = md().llr_exact(Xd, ld, y, s2)
        g, _, se = md().gmi_reduce(L, tx, ld)
        g = g.item()
        assert 0.0 <= g <= 11.0 and g > prev
        prev = g
        idx = torch.from_numpy(rows).cuda()
        ys = y[idx].cpu().numpy()
        Ls = L[idx].cpu().numpy()
        assert_llr_close(Ls, oracle.llr_exact(X, labels, ys, s2), what=f"full-size rows snr={snr}")
        del tx, y, L
        torch.cuda.empty_cache()

"""Streaming receiver (rx_create / rx_run): buffers of a pinned host stream demapped on
several HIP streams with overlapping copies and kernels.

What must hold, at any buffer size and stream count:
  * decisions (hard mode) and LLRs (exact mode) equal llr_maxlog / llr_exact of the same
    symbols in one call (the demapping of a symbol does not depend on its buffer);
  * per-bin bit errors equal ber_count over the bin, and per-bin GMI equals gmi_reduce over
    the bin up to the FP64 combination of the buffers' pieces;
  * hard decisions equal the oracle's nearest point (FP64), ties aside;
  * a ring read several times (a looped capture) gives the same per-bin numbers as the
    stream written out in full.
"""
import ctypes
import math

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu


def md():
    import paper_2104_06311_amd
    return paper_2104_06311_amd


def channel(X, labels, snr_db, N, seed):
    s2 = synth.sigma2_from_snr_db(X, snr_db)
    Xd = torch.from_numpy(X).cuda()
    Ld = torch.from_numpy(labels.astype(np.int32)).cuda()
    tx, y = md().awgn_sample(Xd, seed, 0, N, math.sqrt(s2))
    return Xd, Ld, s2, tx, y


def decisions_from(llr):
    m = llr.shape[1]
    w = (1 << torch.arange(m - 1, -1, -1, device=llr.device, dtype=torch.int64))
    return ((llr < 0).to(torch.int64) * w).sum(1)


def bin_reference(llr, tx, Ld, bins):
    """(errors, gmi) per bin from single calls on the device over each bin's rows."""
    errs, gmis = [], []
    for rows in bins:
        e = md().ber_count(llr[rows], tx[rows], Ld, per_bit=False)[0]
        g = md().gmi_reduce(llr[rows], tx[rows], Ld, per_bit=False, se=False)[0]
        errs.append(int(e.item()))
        gmis.append(float(g.item()))
    return np.array(errs, dtype=np.uint64), np.array(gmis)


@pytest.mark.parametrize("n_streams,buf,binsz", [(3, 1 << 18, 600_000), (1, 100_003, 100_003), (8, 65_536, 1 << 20)])
def test_hard_mode_matches_single_calls_and_oracle(n_streams, buf, binsz):
    X, labels = synth.gaussian_constellation(256, 8, seed=31)
    N = 2_500_123
    Xd, Ld, s2, tx, y = channel(X, labels, 8.0, N, seed=77)
    rx = md().RxStream(Xd, Ld, s2, mode="hard", n_streams=n_streams, buf_symbols=buf, bin_symbols=binsz)
    y_h, tx_h = y.cpu().pin_memory(), tx.cpu().pin_memory()
    out = torch.empty(N, dtype=torch.int32).pin_memory()
    res = rx.run(y_h, tx_h, out=out)
    rx.close()
    L = md().llr_maxlog(Xd, Ld, y, s2)
    ref_dec = decisions_from(L).cpu().numpy()
    assert np.array_equal(out.numpy().astype(np.int64), ref_dec)
    nb = (N + binsz - 1) // binsz
    bins = [slice(b * binsz, min(N, (b + 1) * binsz)) for b in range(nb)]
    e_ref, g_ref = bin_reference(L, tx, Ld, bins)
    assert np.array_equal(res["bin_errors"], e_ref)
    assert np.max(np.abs(res["bin_gmi"] - g_ref)) <= 1e-6
    # the oracle's nearest point (FP64 distances) on a sample; a differing decision must be a near tie
    idx = np.arange(0, N, 997)
    yh = y.cpu().numpy()[idx]
    near = labels[oracle.hard_decision(X, yh).astype(np.int64)].astype(np.int64)
    own = out.numpy()[idx].astype(np.int64)
    diff = np.nonzero(near != own)[0]
    for i in diff:
        d_own = np.sum((X[own[i]].astype(np.float64) - yh[i]) ** 2)
        d_near = np.sum((X[near[i]].astype(np.float64) - yh[i]) ** 2)
        assert d_own - d_near <= 1e-5 * max(1.0, d_near), (i, d_own, d_near)
    assert len(diff) <= 2
    assert res["seconds"] > 0 and res["symbols_per_s"] > 0
    assert res["latency_ms_max"] >= res["latency_ms_mean"] > 0


def test_exact_mode_ring_read_several_times():
    X, labels = synth.product_4d_8psk()
    B = 100_000
    N = 4 * B
    total = 1_050_000                      # 2.6 passes over the ring, last buffer partial
    binsz = 250_000
    Xd, Ld, s2, tx, y = channel(X, labels, 8.0, N, seed=5)
    rx = md().RxStream(Xd, Ld, s2, mode="exact", n_streams=2, buf_symbols=B, bin_symbols=binsz)
    y_h, tx_h = y.cpu().pin_memory(), tx.cpu().pin_memory()
    out = torch.empty((N, 6), dtype=torch.float32).pin_memory()
    res = rx.run(y_h, tx_h, total=total, out=out)
    rx.close()
    L = md().llr_exact(Xd, Ld, y, s2)
    assert torch.equal(out, L.cpu())
    stream_rows = torch.arange(total, device="cuda") % N
    nb = (total + binsz - 1) // binsz
    bins = [stream_rows[b * binsz:min(total, (b + 1) * binsz)] for b in range(nb)]
    e_ref, g_ref = bin_reference(L, tx, Ld, bins)
    assert np.array_equal(res["bin_errors"], e_ref)
    assert np.max(np.abs(res["bin_gmi"] - g_ref)) <= 1e-6
    # and the GMI of the first bin against the FP64 oracle on the same LLR inputs
    rows = bins[0].cpu().numpy()
    ref = oracle.gmi(oracle.llr_exact(X, labels, y.cpu().numpy()[rows], s2), tx.cpu().numpy()[rows], labels)[0]
    assert abs(res["bin_gmi"][0] - ref) <= 1e-4


def test_qam16_hard_mode_and_no_statistics():
    X, labels = synth.qam_gray(16)
    N = 300_001
    Xd, Ld, s2, tx, y = channel(X, labels, 12.0, N, seed=9)
    rx = md().RxStream(Xd, Ld, s2, mode="hard", n_streams=4, buf_symbols=1 << 15, bin_symbols=1 << 17)
    y_h, tx_h = y.cpu().pin_memory(), tx.cpu().pin_memory()
    out = torch.empty(N, dtype=torch.int32).pin_memory()
    res = rx.run(y_h, tx_h, out=out)
    near = labels[oracle.hard_decision(X, y.cpu().numpy()).astype(np.int64)].astype(np.int64)
    assert np.mean(out.numpy().astype(np.int64) != near) <= 1e-5
    ber = res["bin_errors"].sum() / (N * 4)
    ref = oracle.bit_errors(near, tx.cpu().numpy(), labels, 4).sum() / (N * 4)
    assert abs(ber - ref) <= 2.0 / (N * 4)
    # without sent indices nothing is counted, decisions still come back
    out2 = torch.full((N,), -1, dtype=torch.int32).pin_memory()
    res2 = rx.run(y_h, None, out=out2)
    assert res2["bin_errors"] is None and torch.equal(out, out2)
    # zero symbols
    res3 = rx.run(y_h, tx_h, total=0)
    assert res3["bin_errors"].size == 0
    rx.close()


def test_exact_mode_small_constellation_many_streams():
    """M = 16 (the one-thread-per-symbol kernel) in exact mode, 8 streams, buffers of 4097
    symbols and bins of 3 buffers, LLRs checked element by element against one call."""
    X, labels = synth.gaussian_constellation(16, 3, seed=8)
    labels = synth.random_labels(16, 2)
    N = 100_000
    Xd, Ld, s2, tx, y = channel(X, labels, 5.0, N, seed=21)
    rx = md().RxStream(Xd, Ld, s2, mode="exact", n_streams=8, buf_symbols=4097, bin_symbols=3 * 4097)
    y_h, tx_h = y.cpu().pin_memory(), tx.cpu().pin_memory()
    out = torch.empty((N, 4), dtype=torch.float32).pin_memory()
    res = rx.run(y_h, tx_h, out=out)
    rx.close()
    L = md().llr_exact(Xd, Ld, y, s2)
    assert torch.equal(out, L.cpu())
    nb = (N + 3 * 4097 - 1) // (3 * 4097)
    bins = [slice(b * 3 * 4097, min(N, (b + 1) * 3 * 4097)) for b in range(nb)]
    e_ref, g_ref = bin_reference(L, tx, Ld, bins)
    assert np.array_equal(res["bin_errors"], e_ref)
    assert np.max(np.abs(res["bin_gmi"] - g_ref)) <= 1e-6


def test_rx_rejects_bad_arguments():
    X, labels = synth.qam_gray(16)
    Xd = torch.from_numpy(X).cuda()
    Ld = torch.from_numpy(labels.astype(np.int32)).cuda()
    with pytest.raises(md().MdemapError):
        md().RxStream(Xd, Ld, 0.1, buf_symbols=1000, bin_symbols=999)
    with pytest.raises(md().MdemapError):
        md().RxStream(Xd, Ld, 0.1, n_streams=9)
    with pytest.raises(md().MdemapError):
        md().RxStream(Xd, Ld, -0.1)
    rx = md().RxStream(Xd, Ld, 0.1, buf_symbols=1000, bin_symbols=4000)
    y = torch.zeros((2500, 2), dtype=torch.float32).pin_memory()
    tx = torch.zeros(2500, dtype=torch.int32).pin_memory()
    with pytest.raises(md().MdemapError):
        rx.run(y, tx, total=5000)          # a ring read twice must hold whole buffers
    with pytest.raises(ValueError):
        rx.run(torch.zeros((2500, 2), dtype=torch.float32), tx)     # not pinned
    # the C entry point checks the pinning itself
    from paper_2104_06311_amd._lib import lib
    pageable = np.zeros((2500, 2), dtype=np.float32)
    assert lib().rx_run(rx._h, pageable.ctypes.data, None, 2500, 2500, None, None, None, None) == -1
    assert b"pinned" in lib().last_error()
    err = np.zeros(3, dtype=np.uint64)
    assert lib().rx_run(rx._h, y.data_ptr(), None, 2500, 2500, None, err.ctypes.data, None, None) == -1
    rx.close()

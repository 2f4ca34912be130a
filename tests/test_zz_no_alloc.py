"""GPU check of the allocation-free entry point llr_exact_noalloc, called through the C
ABI: on the same inputs it gives llr_exact's LLRs bit for bit, on two calls in a row (the
second smaller, so that stale scratch contents of the first would show), across the
paths the exact demapper has (fast pass with the wide-range fallback at high SNR, the
M <= 16 kernel, a constellation streamed through LDS in chunks), it rejects sizes
beyond its limit before touching the device, and captured into a graph it replays like
the eager call."""
import ctypes
import math

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def lib():
    from paper_2104_06311_amd import _lib
    return _lib.lib()


def stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def case(X, labels, snr_db, N, seed):
    import paper_2104_06311_amd as md
    Xd = torch.from_numpy(X).cuda()
    ld = torch.from_numpy(labels.astype(np.int32)).cuda()
    s2 = synth.sigma2_from_snr_db(X, snr_db)
    tx, y = md.awgn_sample(Xd, seed, 0, N, math.sqrt(s2))
    return Xd, ld, y, s2


def both(Xd, ld, y, s2):
    M, D = Xd.shape
    N = y.shape[0]
    m = M.bit_length() - 1
    ref = torch.full((N, m), float("nan"), device="cuda")
    out = torch.full((N, m), float("nan"), device="cuda")
    L = lib()
    assert L.llr_exact(Xd.data_ptr(), ld.data_ptr(), M, D, y.data_ptr(), N, s2, 0, ref.data_ptr(), stream()) == 0
    assert L.llr_exact_noalloc(Xd.data_ptr(), ld.data_ptr(), M, D, y.data_ptr(), N, s2, 0, out.data_ptr(),
                               stream()) == 0, L.last_error()
    torch.cuda.synchronize()
    return ref, out


def test_noalloc_matches_llr_exact_on_two_calls_in_a_row():
    X8, l8 = synth.gaussian_constellation(2048, 8, 11)
    big = case(X8, l8, 14.0, 1 << 20, 5)          # fast pass + wide-range pass at 14 dB
    X4, l4 = synth.product_4d_8psk()
    small = case(X4, l4, 8.0, 5003, 6)            # smaller second call, ragged N
    import paper_2104_06311_amd as md
    for args in (big, small):
        ref, out = both(*args)
        assert torch.isfinite(ref).all()
        assert torch.equal(ref, out)
    md.llr_path_counts()
    # the wide-range pass ran on the first case (its symbols went through the scratch lists)
    ref, out = both(*big)
    assert torch.equal(ref, out)
    n_wide, _ = md.llr_path_counts()
    assert n_wide > 0


def test_noalloc_small_m_and_chunked_constellation():
    Xs, ls = synth.qam_gray(16)
    X16, l16 = synth.gaussian_constellation(65536, 16, 12)
    for args in (case(Xs, ls, 6.0, 777, 7), case(X16, l16, 10.0, 2000, 8), case(Xs, ls, 12.0, 100, 9)):
        ref, out = both(*args)
        assert torch.equal(ref, out)


def test_noalloc_limits_are_rejected_before_device_work():
    L = lib()
    fake = ctypes.c_void_p(0x1000)      # never dereferenced: validation fails first
    assert L.llr_exact_noalloc(fake, fake, 2048, 8, fake, (1 << 20) + 1, 0.1, 0, fake, None) == -1
    assert b"2^20" in L.last_error()
    assert L.llr_exact_noalloc(fake, fake, 48, 8, fake, 10, 0.1, 0, fake, None) == -2


@pytest.mark.parametrize("which", ["8d", "4d"])
def test_noalloc_in_a_captured_graph_replays_like_eager(which):
    """Captured into a graph (the callers it is for run under stream capture), the call
    replays several times, with other eager work and synchronisations between the
    replays, and every replay gives llr_exact's LLRs bit for bit: 8D M = 2048 through the
    matrix-core kernel with wide-range symbols at 14 dB, 4D M = 64 through the
    one-thread-per-symbol kernel."""
    import paper_2104_06311_amd as md
    if which == "8d":
        X, labels = synth.gaussian_constellation(2048, 8, synth.SEED_BASE + 1)
        snr, N = 14.0, 6000
    else:
        X, labels = synth.product_4d_8psk()
        snr, N = 8.0, 5000
    M, D = X.shape
    m = M.bit_length() - 1
    Xd = torch.from_numpy(X).cuda()
    ld = torch.from_numpy(labels.astype(np.int32)).cuda()
    s2 = synth.sigma2_from_snr_db(X, snr)
    tx, y = md.awgn_sample(Xd, 77, 0, N, math.sqrt(s2))
    ref = md.llr_exact(Xd, ld, y, s2)
    L = lib()
    out = torch.full((N, m), float("nan"), device="cuda")
    # one eager call first (the host label check and the scratch address lookup happen here)
    assert L.llr_exact_noalloc(Xd.data_ptr(), ld.data_ptr(), M, D, y.data_ptr(), N, s2, 0, out.data_ptr(),
                               stream()) == 0, L.last_error()
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    g = torch.cuda.CUDAGraph()
    cap = torch.cuda.Stream()
    with torch.cuda.stream(cap):
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=cap):
            rc = L.llr_exact_noalloc(Xd.data_ptr(), ld.data_ptr(), M, D, y.data_ptr(), N, s2, 0, out.data_ptr(),
                                     ctypes.c_void_p(cap.cuda_stream))
    assert rc == 0, L.last_error()
    for r in range(4):
        out.fill_(float("nan"))
        junk = torch.randn(1 << 20, device="cuda").sum()      # eager work between the replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref), (which, r)
        del junk

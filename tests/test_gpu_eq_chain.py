"""Dependent buffers: the DD-LMS equaliser continued from buffer to buffer.

ddlms_equalize_chain continues every instance from its own taps, so chained calls over
consecutive sample windows (overlapping by two samples) must give the decisions, outputs
and taps of one ddlms_equalize call over the whole window, bit for bit (the recursion is
the same sequence of IEEE double operations; ddlms_equalize itself is pinned bit for bit
against the FP64 oracle in test_gpu_ddlms).  The streaming receiver's equaliser stage
chains its buffers through events across its HIP streams; its outputs and per-bin
statistics must equal that single call followed by the demapper on the whole stream."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

IDENT_H = [1, 0, 0, 0]
ZERO = [0, 0, 0, 0]


def md():
    import paper_2104_06311_amd
    return paper_2104_06311_amd


@pytest.mark.parametrize("B,pieces,M,mu", [(300, [50, 50, 50, 50], 16, 0.01), (257, [1, 99, 0, 37, 63], 4, 0.05),
                                           (1, [7, 120], 16, 0.003)])
def test_chained_calls_equal_one_call(B, pieces, M, mu):
    N = sum(pieces)
    x, tx, C, labels = synth.equaliser_input(B, N, M=M, seed=700 + B)
    xd, Cd = torch.from_numpy(x).cuda(), torch.from_numpy(C).cuda()
    dec1, z1, h1, g1 = md().ddlms_equalize(xd, Cd, IDENT_H, ZERO, mu)
    h = torch.zeros((B, 4), dtype=torch.complex128, device="cuda")
    h[:, 0] = 1.0
    g = torch.zeros((B, 4), dtype=torch.complex128, device="cuda")
    decs, zs = [], []
    s = 0
    for n in pieces:
        d, z = md().ddlms_equalize_chain(xd[2 * s:2 * s + 2 * n + 2], Cd, h, g, mu)
        decs.append(d)
        zs.append(z)
        s += n
    dec2, z2 = torch.cat(decs), torch.cat(zs)
    assert torch.equal(dec1, dec2)
    assert np.array_equal(z1.cpu().numpy().view(np.uint32), z2.cpu().numpy().view(np.uint32))
    assert np.array_equal(h1.cpu().numpy().view(np.uint64), h.cpu().numpy().view(np.uint64))
    assert np.array_equal(g1.cpu().numpy().view(np.uint64), g.cpu().numpy().view(np.uint64))


def _receiver_case(mode, P=64, n=32, Nr=256, streams=3, mu=0.01):
    x, tx, C, labels = synth.equaliser_input(P, Nr, M=16, seed=811)
    X = np.stack([C.real, C.imag], axis=1).astype(np.float32)
    Xd, ld = torch.from_numpy(X).cuda(), torch.from_numpy(labels.astype(np.int32)).cuda()
    N = Nr * P
    y_h = torch.from_numpy(x.view(np.float32).reshape(2 * Nr + 2, 2 * P).copy()).pin_memory()
    tx_h = torch.from_numpy(tx[:Nr].reshape(-1).astype(np.int32)).pin_memory()
    m = 4
    out = (torch.empty(N, dtype=torch.int32) if mode == "hard" else torch.empty((N, m), dtype=torch.float32)).pin_memory()
    s2 = synth.sigma2_from_snr_db(X, 20.0)
    rx = md().RxStream(Xd, ld, s2, mode=mode, n_streams=streams, buf_symbols=n * P, bin_symbols=2 * n * P,
                       equaliser={"instances": P, "mu": mu, "h0": IDENT_H, "g0": ZERO})
    r = rx.run(y_h, tx_h, out=out)
    rx.close()
    # the reference: one equaliser call over the whole stream, then the demapper
    dec, z, _, _ = md().ddlms_equalize(torch.from_numpy(x).cuda(), torch.from_numpy(C).cuda(), IDENT_H, ZERO, mu)
    zf = torch.view_as_real(z).reshape(N, 2).contiguous()          # stream order (time-major)
    txd = torch.from_numpy(tx[:Nr].reshape(-1).astype(np.int32)).cuda()
    L = md().llr_maxlog(Xd, ld, zf, s2) if mode == "hard" else md().llr_exact(Xd, ld, zf, s2)
    return r, out, L, txd, ld, dec, labels, 2 * n * P


@pytest.mark.parametrize("mode", ["hard", "exact"])
def test_receiver_equaliser_stage_equals_one_call(mode):
    r, out, L, txd, ld, dec, labels, binsz = _receiver_case(mode)
    N = L.shape[0]
    if mode == "hard":
        # the label whose bit m-1-k is set where column k of the reference LLRs is negative
        Lh = L.cpu().numpy()
        want = np.zeros(N, dtype=np.int64)
        for k in range(Lh.shape[1]):
            want = (want << 1) | (Lh[:, k] < 0)
        assert np.array_equal(out.numpy().astype(np.int64), want)
        # which is the equaliser's own nearest-point decision, boundary ties aside
        agree = np.mean(want == labels.astype(np.int64)[dec.cpu().numpy().reshape(-1)])
        assert agree > 0.9999, agree
    else:
        assert np.array_equal(out.numpy().view(np.uint32), L.cpu().numpy().view(np.uint32))
    for b in range(N // binsz):
        sl = slice(b * binsz, (b + 1) * binsz)
        errs, _ = md().ber_count(L[sl].contiguous(), txd[sl].contiguous(), ld, per_bit=False)
        assert int(r["bin_errors"][b]) == int(errs.item())
        gb = md().gmi_reduce(L[sl].contiguous(), txd[sl].contiguous(), ld, per_bit=False, se=False)[0].item()
        assert abs(r["bin_gmi"][b] - gb) <= 1e-9 * max(1.0, abs(gb))
    # and the equaliser converged: few bit errors in the last bin at 25 dB
    assert int(r["bin_errors"][-1]) < 0.01 * binsz * 4, r["bin_errors"]


def test_receiver_equaliser_rejects_bad_rings():
    x, tx, C, labels = synth.equaliser_input(8, 16, M=16, seed=5)
    X = np.stack([C.real, C.imag], axis=1).astype(np.float32)
    rx = md().RxStream(torch.from_numpy(X).cuda(), torch.from_numpy(labels.astype(np.int32)).cuda(), 0.1,
                       n_streams=2, buf_symbols=32, equaliser={"instances": 8, "mu": 0.01, "h0": IDENT_H, "g0": ZERO})
    y = torch.from_numpy(x.view(np.float32).reshape(34, 16).copy()).pin_memory()
    with pytest.raises(md().MdemapError):
        rx.run(y, total=100)                     # not a multiple of the 8 channels
    with pytest.raises(ValueError):
        rx.run(torch.zeros((34, 12)).pin_memory())   # rows of 6, not 8, channels
    r = rx.run(y, stats=True)
    assert r["bin_errors"] is None and r["symbols_per_s"] > 0
    rx.close()

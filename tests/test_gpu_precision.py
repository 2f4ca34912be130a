"""Reduced-precision score variants of llr_exact (MD_PREC_FP16, MD_PREC_BF16_SCORES)
against the FP64 oracle.

Bound, derived from the arithmetic: the one-pass score of point j for symbol n is
sum_k u_jk w_nk + biases with u = a x, w = (2c/a) y (c = log2(e) / (2 sigma2)), each
operand rounded once to the format (unit roundoff e_f = 2^-11 for FP16, 2^-9 for BF16),
so the product carries a relative error of at most 2 e_f (1 + e_f) and the score an
error of at most 2 e_f (1 + e_f) * 2c sum_k |x_jk y_nk| base-2 units, plus the hi/lo
rounding of the two biases (at most 2 e_f^2 of |bias| + c ||y||^2 + c ||x||^2).  A log-sum-exp
moves by at most the largest change of its arguments, so each LLR (a difference of
two, in nats) moves by at most 2 ln 2 times the largest score error of the symbol, on
top of the FP32 path's own rounding (2e-3 + 2e-4 |L|).  GMI errors are reported, not
pinned (a loose band only guards against gross failure)."""
import math

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

UNIT = {"fp16": 2.0 ** -11, "bf16_scores": 2.0 ** -9}


def md():
    import paper_2104_06311_amd as m
    return m


def llr_bound(X, y, sigma2, prec, ref):
    e = UNIT[prec]
    c = math.log2(math.e) / (2.0 * sigma2)
    Xa = np.abs(X.astype(np.float64))
    ya = np.abs(y.astype(np.float64))
    cross = (ya @ Xa.T).max(axis=1)                              # max_j sum_k |x_jk y_nk|
    bias = 100.0 + c * np.sum(y.astype(np.float64) ** 2, axis=1) + c * np.max(np.sum(Xa ** 2, axis=1))
    dt = 2 * e * (1 + e) * 2 * c * cross + 2 * e * e * bias
    return 2e-3 + 2e-4 * np.abs(ref) + 2 * math.log(2.0) * 1.01 * dt[:, None]


@pytest.mark.parametrize("prec", ["fp16", "bf16_scores"])
@pytest.mark.parametrize("case", ["8d_m2048", "4d_m64", "2d_qam256", "12d_m512"])
def test_reduced_precision_scores_within_derived_bound(prec, case):
    if case == "8d_m2048":
        X, labels = synth.gaussian_constellation(2048, 8, synth.SEED_BASE + 1)
        snrs, N = (4.0, 9.0, 14.0), 6001
    elif case == "4d_m64":
        X, labels = synth.product_4d_8psk()
        snrs, N = (8.0,), 20003
    elif case == "2d_qam256":
        X, labels = synth.qam_gray(256)
        snrs, N = (10.0, 20.0), 9000
    else:
        X, labels = synth.gaussian_constellation(512, 12, 41)
        labels = synth.random_labels(512, 42)
        snrs, N = (6.0,), 3000
    Xd = torch.from_numpy(X).cuda()
    ld = torch.from_numpy(labels.astype(np.int32)).cuda()
    for snr in snrs:
        s2 = synth.sigma2_from_snr_db(X, snr)
        tx, y = md().awgn_sample(Xd, 7, 0, N, math.sqrt(s2))
        L = md().llr_exact(Xd, ld, y, s2, prec=prec).cpu().numpy()
        yh = y.cpu().numpy()
        ref = oracle.llr_exact(X, labels, yh, s2)
        assert np.all(np.isfinite(L))
        err = np.abs(L - ref)
        bound = llr_bound(X, yh, s2, prec, ref)
        bad = np.argwhere(err > bound)
        assert bad.size == 0, (case, snr, bad[:3], err[tuple(bad[0])], bound[tuple(bad[0])])
        g = md().gmi_reduce(md().llr_exact(Xd, ld, y, s2, prec=prec), tx, ld)[0].item()
        g_ref = oracle.gmi(ref, tx.cpu().numpy().astype(np.uint32), labels)[0]
        assert abs(g - g_ref) <= (3e-3 if prec == "fp16" else 3e-2), (case, snr, g, g_ref)


def test_reduced_precision_limits_and_noalloc():
    X, labels = synth.gaussian_constellation(256, 13, 3)
    Xd = torch.from_numpy(X).cuda()
    ld = torch.from_numpy(labels.astype(np.int32)).cuda()
    y = torch.zeros((10, 13), device="cuda")
    with pytest.raises(md().MdemapError) as e:
        md().llr_exact(Xd, ld, y, 0.1, prec="fp16")
    assert e.value.status == -8
    # the allocation-free entry point takes the same precision argument, same bits
    X, labels = synth.gaussian_constellation(1024, 8, 4)
    Xd = torch.from_numpy(X).cuda()
    ld = torch.from_numpy(labels.astype(np.int32)).cuda()
    s2 = synth.sigma2_from_snr_db(X, 12.0)
    _, y = md().awgn_sample(Xd, 9, 0, 4099, math.sqrt(s2))
    for prec in ("fp16", "bf16_scores"):
        a = md().llr_exact(Xd, ld, y, s2, prec=prec)
        b = md().llr_exact_noalloc(Xd, ld, y, s2, prec=prec)
        assert torch.equal(a, b)

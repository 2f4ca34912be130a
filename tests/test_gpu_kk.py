"""Kramers-Kronig front end (kk_frontend) against the FP64 oracle, over every output
sample, including the first and last half-blocks whose halo lies outside the stream.

Tolerance: the GPU works in FP32.  l = 0.5 ln x is exact to a few ulp; the 1024-point
FFT pair adds about log2(1024) eps ||l|| to the phase (below 1e-5 for |l| < 2); the field
exp(l) e^{i phi} then carries |E| (1e-5 + 1e-5).  So 1e-4 (1 + max |E|) bounds the error
with margin."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu


def md():
    import paper_2104_06311_amd
    return paper_2104_06311_amd


def check(x, A, nu):
    out = md().kk_frontend(torch.from_numpy(x).cuda(), A, nu).cpu().numpy()
    ref = oracle.kk_field(x, A, nu)
    tol = 1e-4 * (1.0 + np.max(np.abs(ref)) + A)      # |E| <= |s| + A
    err = np.max(np.abs(out - ref))
    assert err <= tol, (err, tol)
    return out, ref


@pytest.mark.parametrize("T,A,nu", [(8192, 1.5, 0.0), (512, 1.0, 0.129), (1536, 2.0, -0.0625),
                                    (65536, 1.5, 0.129)])
def test_parity_with_the_oracle(T, A, nu):
    x, s = synth.kk_input(T, A=A, seed=7 + T)
    check(x, A, nu)


def test_recovers_the_signal_at_full_size():
    """2^22 samples (one of the paper's ADC buffers): in the interior the front end
    returns the synthetic signal up to the intensity noise."""
    T, A = 1 << 22, 1.5
    x, s = synth.kk_input(T, A=A, snr_db=80.0)
    out = md().kk_frontend(torch.from_numpy(x).cuda(), A, 0.0).cpu().numpy()
    I = slice(512, T - 512)
    assert np.max(np.abs(out[I] - s[I])) < 5e-3
    # sampled blocks against the oracle (it runs over the whole stream)
    ref = oracle.kk_field(x, A, 0.0)
    rows = np.random.default_rng(3).choice(T, size=20000, replace=False)
    assert np.max(np.abs(out[rows] - ref[rows])) <= 1e-4 * (1.0 + 2.0 * A)


def test_empty_and_rejected():
    out = md().kk_frontend(torch.zeros(0, dtype=torch.float32, device="cuda"), 1.0, 0.0)
    assert out.shape == (0,)
    with pytest.raises(md().MdemapError):
        md().kk_frontend(torch.ones(1000, dtype=torch.float32, device="cuda"), 1.0, 0.0)


def test_non_positive_samples_stay_local():
    """A detected intensity of zero, a negative one (noise) and a NaN are floored at 2^-126
    on both sides: every output stays finite, and the result equals the oracle's within
    the FP32 bound scaled by the largest log-amplitude (|ln 2^-126| / 2 = 43.7), which the
    FFT pair now carries."""
    T, A = 8192, 1.5
    x, _ = synth.kk_input(T, A=A, seed=11)
    x[[700, 3001, 3002]] = [0.0, -0.25, np.nan]
    out = md().kk_frontend(torch.from_numpy(x).cuda(), A, 0.129).cpu().numpy()
    assert np.all(np.isfinite(out))
    ref = oracle.kk_field(x, A, 0.129)
    assert np.all(np.isfinite(ref))
    lmax = 0.5 * 126 * np.log(2.0)
    tol = 1e-4 * (1.0 + np.max(np.abs(ref)) + A) * lmax
    assert np.max(np.abs(out - ref)) <= tol
    # blocks whose windows do not reach the bad samples are unaffected: same bound as clean input
    far = np.r_[0:0, 1536:2048, 4608:T]
    assert np.max(np.abs(out[far] - ref[far])) <= 1e-4 * (1.0 + np.max(np.abs(ref)) + A)

"""GPU checks of the fast-kernel event timing (kernel_timing / kernel_timing_read): it
counts exactly the demapping calls made while it is on, on the stream it was switched on
for, and its milliseconds fit inside the call's own event-timed duration."""
import math

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def md():
    import paper_2104_06311_amd as m
    return m


def test_timing_counts_the_fast_kernels_and_fits_inside_the_call():
    X, labels = synth.gaussian_constellation(2048, 8, 7)
    Xd = torch.from_numpy(X).cuda()
    ld = torch.from_numpy(labels.astype(np.int32)).cuda()
    s2 = synth.sigma2_from_snr_db(X, 9.0)
    N = 200_000
    tx, y = md().awgn_sample(Xd, 3, 0, N, math.sqrt(s2))
    out = torch.empty((N, 11), device="cuda")
    md().llr_exact(Xd, ld, y, s2, out=out)            # untimed: timing is off
    md().kernel_timing(True)
    assert md().kernel_timing_read() == (0.0, 0)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(3):
        md().llr_exact(Xd, ld, y, s2, out=out)
    md().llr_maxlog(Xd, ld, y, s2, out=out)
    b.record()
    torch.cuda.synchronize()
    ms, n = md().kernel_timing_read()
    assert n == 4, n
    assert 0.0 < ms <= a.elapsed_time(b) * 1.02, (ms, a.elapsed_time(b))
    assert md().kernel_timing_read() == (0.0, 0)      # a read starts a new count
    # another stream is not timed
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        md().llr_exact(Xd, ld, y, s2, out=out)
        assert md().kernel_timing_read() == (0.0, 0)
    torch.cuda.synchronize()
    md().kernel_timing(False)
    md().llr_exact(Xd, ld, y, s2, out=out)
    assert md().kernel_timing_read() == (0.0, 0)

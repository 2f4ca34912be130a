"""GPU checks at the 16-dimensional size: Gaussian constellation M = 65536 (16 bits),
N = 1e6 seeded symbols at 10 and 16 dB.  The oracle evaluates a subset of the symbols
(the first rows of the same draw); the full draw is checked through properties that
hold at any size.  At 16 dB about 40 % of the symbols have a subset whose best point
lies beyond the first FP32 exponent window, so the wide-range pass carries a large
share of the work there.  Tolerances as in test_gpu_parity.
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
N_FULL = 1_000_000
N_ORACLE = 3000


def md():
    import paper_2104_06311_amd as m
    return m


def check_close(got, ref, what):
    err = np.abs(got.astype(np.float64) - ref)
    assert np.all(np.isfinite(got)), what
    bad = err > ATOL + RTOL * np.abs(ref)
    assert not bad.any(), f"{what}: {bad.sum()} entries out of tolerance, max |dL| {err.max():.3e}"


@pytest.fixture(scope="module")
def constellation():
    X, labels = synth.gaussian_constellation(65536, 16, synth.SEED_BASE + 4)
    return X, labels, torch.from_numpy(X).cuda(), torch.from_numpy(labels.astype(np.int32)).cuda()


@pytest.mark.parametrize("snr_db", [10.0, 16.0])
def test_16d_65536_exact_and_maxlog(constellation, snr_db):
    X, labels, Xd, ld = constellation
    s2 = synth.sigma2_from_snr_db(X, snr_db)
    seed = synth.SEED_BASE + 4
    offset = 0 if snr_db == 10.0 else N_FULL
    print(f"16D M=65536 snr={snr_db} N={N_FULL}", flush=True)
    tx, y = md().awgn_sample(Xd, seed, offset, N_FULL, math.sqrt(s2))
    L = md().llr_exact(Xd, ld, y, s2)
    n_wide, n_careful = md().llr_path_counts()
    Lm = md().llr_maxlog(Xd, ld, y, s2)
    g, gb, se = md().gmi_reduce(L, tx, ld)
    gm = md().gmi_reduce(Lm, tx, ld)[0].item()
    g, se = g.item(), se.item()
    print(f"  GMI exact {g:.5f} +- {se:.5f}, max-log {gm:.5f}; wide {n_wide}, careful {n_careful}", flush=True)
    assert 0.0 <= g <= 16.0 and gm <= g + 1e-3
    if snr_db == 16.0:
        assert n_wide > N_FULL // 10 and n_careful < N_FULL // 50
    # the oracle on the first rows of the same draw
    yh = y[:N_ORACLE].cpu().numpy()
    txh = tx[:N_ORACLE].cpu().numpy().astype(np.uint32)
    ref = oracle.llr_exact(X, labels, yh, s2)
    check_close(L[:N_ORACLE].cpu().numpy(), ref, f"exact {snr_db} dB")
    check_close(Lm[:N_ORACLE].cpu().numpy(), oracle.llr_maxlog(X, labels, yh, s2), f"max-log {snr_db} dB")
    g_sub = md().gmi_reduce(L[:N_ORACLE].contiguous(), tx[:N_ORACLE].contiguous(), ld)[0].item()
    assert abs(g_sub - oracle.gmi(ref, txh, labels)[0]) <= 1e-4
    # rows that blocks reach after their first symbol group (fragments streamed across
    # groups), and the ragged end of the draw
    for a in (500_000, N_FULL - 200):
        yh = y[a:a + 200].cpu().numpy()
        check_close(L[a:a + 200].cpu().numpy(), oracle.llr_exact(X, labels, yh, s2), f"exact {snr_db} dB rows {a}+")
        check_close(Lm[a:a + 200].cpu().numpy(), oracle.llr_maxlog(X, labels, yh, s2), f"max-log {snr_db} dB rows {a}+")


@pytest.mark.parametrize("maxlog", [False, True])
def test_streamed_fragments_against_oracle(maxlog):
    """M = 1024, D = 16: four K steps, 128 KiB of fragments, more than LDS holds next to the
    symbol staging: max-log streams them through two LDS buffers in four chunks, the exact
    path copies them chunk by chunk.  N = 110,000 symbols: every block also takes a later
    symbol group (for max-log its first chunk is loaded during the previous group's last
    one).  Every row against the oracle."""
    X, labels = synth.gaussian_constellation(1024, 16, 77)
    labels = synth.random_labels(1024, 16)
    Xd, ld = torch.from_numpy(X).cuda(), torch.from_numpy(labels.astype(np.int32)).cuda()
    s2 = synth.sigma2_from_snr_db(X, 11.0)
    N = 110_000
    print(f"M=1024 D=16 N={N} maxlog={maxlog}", flush=True)
    tx, y = md().awgn_sample(Xd, 91, 0, N, math.sqrt(s2))
    L = (md().llr_maxlog if maxlog else md().llr_exact)(Xd, ld, y, s2).cpu().numpy()
    yh = y.cpu().numpy()
    ref = (oracle.llr_maxlog if maxlog else oracle.llr_exact)(X, labels, yh, s2)
    check_close(L, ref, f"M=1024 D=16 {'max-log' if maxlog else 'exact'}")

"""Pins of the oracle's Kramers-Kronig front end (section "Experimental setup"), fixed by
the mathematics rather than by the oracle's own formula:
  * the blockwise Hilbert transform of a cosine on an FFT bin is the sine;
  * the Kramers-Kronig theorem: for a carrier A plus a signal with positive frequencies
    only and |s| < A, the phase of A + s is the Hilbert transform of ln|A + s|, so the
    front end returns s exactly (to rounding) when s is periodic in the block and its
    harmonics stay far below half the FFT length;
  * the downshift by nu moves a tone at frequency nu to DC.
The first and last half-blocks see the zeros outside the stream, so the checks cover the
interior samples [512, T - 512).
"""
import numpy as np

import oracle


def kk_signal(T, A, K, seed, f_shift=0.0):
    rng = np.random.default_rng(seed)
    c = (rng.standard_normal(K) + 1j * rng.standard_normal(K))
    c *= 0.3 * A / np.sum(np.abs(c))          # |s| <= 0.3 A
    t = np.arange(T)
    s = np.zeros(T, dtype=np.complex128)
    for k in range(1, K + 1):
        s += c[k - 1] * np.exp(2j * np.pi * k * t / 1024)
    return s


def test_hilbert_of_a_bin_centred_cosine_is_the_sine():
    T = 4096
    t = np.arange(T)
    l = 0.2 * np.cos(2 * np.pi * 37 * t / 1024)
    x = np.exp(2 * l)                              # so that 0.5 ln x = l
    s = oracle.kk_field(x, 0.0, 0.0)               # A = 0, no shift: s = exp(l + i H(l))
    phi = np.angle(s)
    I = slice(512, T - 512)
    assert np.max(np.abs(phi[I] - 0.2 * np.sin(2 * np.pi * 37 * t[I] / 1024))) < 1e-12


def test_kramers_kronig_recovers_the_signal():
    T, A = 8192, 1.5
    s = kk_signal(T, A, 12, seed=4)
    x = np.abs(A + s) ** 2
    out = oracle.kk_field(x, A, 0.0)
    I = slice(512, T - 512)
    assert np.max(np.abs(out[I] - s[I])) < 1e-10
    assert np.max(np.abs(out[:256] - s[:256])) > 1e-3     # the zero halo does show at the edge


def test_downshift_moves_a_tone_to_dc():
    T, A = 4096, 2.0
    t = np.arange(T)
    k = 5
    s = 0.4 * np.exp(2j * np.pi * k * t / 1024)
    x = np.abs(A + s) ** 2
    out = oracle.kk_field(x, A, k / 1024)
    assert np.max(np.abs(out[512:T - 512] - 0.4)) < 1e-10

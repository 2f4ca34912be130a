"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module only builds inputs: labelled constellations, noise variances for a
given SNR, and the workload descriptions.  It holds none of the demapping
arithmetic (no distances, LLRs, GMI or noise draws of the channel itself -- the
channel's random numbers are drawn by ``awgn_sample`` on the GPU and by its CPU
twin in the oracle).  Both the oracle and the GPU library receive exactly the
arrays produced here.

Constellations
  * 8-PSK with binary-reflected Gray labels (BRGC, named in the paper's acronym
    glossary): x_i = (cos 2 pi i/8, sin 2 pi i/8), label i ^ (i >> 1).
  * 4D 8-PSK x 8-PSK (64 points, 6 bits): point j = 8a + b is
    (x_a, x_b), label (l_a << 3) | l_b.
  * Gaussian: M points i.i.d. N(0, I_D) from numpy's PCG64 with the given seed,
    scaled in float64 so that the average energy per two real dimensions is 1,
    then rounded once to float32; label = point index.
  * BPSK and Gray QPSK (closed-form test cases).
  * 4D product of two square QAMs (M = 4096 for 64-QAM x 64-QAM), labels concatenated
    like the 8-PSK product: a structured large constellation whose LLRs a small
    network can represent (each bit depends on one real coordinate).
  * Square M-QAM (M = 4, 16, 64, 256) with a BRGC label per axis: point (i, q) sits at
    (2i - L + 1, 2q - L + 1) / sqrt(E) with L = sqrt(M) and E = 2 (L^2 - 1) / 3 (unit
    energy per 2D), label (g(i) << log2 L) | g(q), g(x) = x ^ (x >> 1); the paper's
    test signals are QAM formats.

SNR convention: sigma^2 = E_s / (D * SNR_lin), E_s = mean ||x||^2 (so SNR is the
energy per real dimension over the noise variance per real dimension; for
unit energy per 2D this is sigma^2 = 1 / (2 SNR_lin)).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


# --------------------------------------------------------------------------- constellations
def bpsk():
    X = np.array([[1.0], [-1.0]], dtype=np.float32)
    labels = np.array([0, 1], dtype=np.uint32)
    return X, labels


def gray_qpsk():
    a = 1.0 / math.sqrt(2.0)
    X = np.array([[a, a], [-a, a], [-a, -a], [a, -a]], dtype=np.float32)
    labels = np.array([0b00, 0b01, 0b11, 0b10], dtype=np.uint32)
    return X, labels


def psk8_brgc(phase: float = 0.0):
    i = np.arange(8)
    th = 2.0 * np.pi * i / 8.0 + phase
    X = np.stack([np.cos(th), np.sin(th)], axis=1).astype(np.float32)
    labels = (i ^ (i >> 1)).astype(np.uint32)
    return X, labels


def qam_gray(M: int):
    L = int(round(math.sqrt(M)))
    if L * L != M or L < 2 or (L & (L - 1)):
        raise ValueError("square QAM needs M = 4^k")
    b = L.bit_length() - 1
    E = 2.0 * (L * L - 1) / 3.0
    X = np.zeros((M, 2), dtype=np.float64)
    labels = np.zeros(M, dtype=np.uint32)
    for i in range(L):
        for q in range(L):
            j = i * L + q
            X[j] = [(2 * i - L + 1) / math.sqrt(E), (2 * q - L + 1) / math.sqrt(E)]
            labels[j] = ((i ^ (i >> 1)) << b) | (q ^ (q >> 1))
    return X.astype(np.float32), labels


def product_4d_8psk():
    X2, l2 = psk8_brgc()
    X = np.zeros((64, 4), dtype=np.float32)
    labels = np.zeros(64, dtype=np.uint32)
    for a in range(8):
        for b in range(8):
            j = 8 * a + b
            X[j, 0:2] = X2[a]
            X[j, 2:4] = X2[b]
            labels[j] = (int(l2[a]) << 3) | int(l2[b])
    return X, labels


def qam_product_4d(M2: int = 64):
    """4D product of two square M2-QAM (BRGC per axis, unit energy per 2D): point
    j = M2 a + b is (x_a, x_b), label (l_a << log2 M2) | l_b; M = M2^2 points."""
    X2, l2 = qam_gray(M2)
    b2 = M2.bit_length() - 1
    M = M2 * M2
    X = np.zeros((M, 4), dtype=np.float32)
    labels = np.zeros(M, dtype=np.uint32)
    for a in range(M2):
        for b in range(M2):
            j = M2 * a + b
            X[j, 0:2] = X2[a]
            X[j, 2:4] = X2[b]
            labels[j] = (int(l2[a]) << b2) | int(l2[b])
    return X, labels


def gaussian_constellation(M: int, D: int, seed: int):
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((M, D))
    es = np.mean(np.sum(g * g, axis=1))
    X = (g * math.sqrt((D / 2.0) / es)).astype(np.float32)
    labels = np.arange(M, dtype=np.uint32)
    return X, labels


def random_labels(M: int, seed: int):
    return np.random.default_rng(seed).permutation(M).astype(np.uint32)


# --------------------------------------------------------------------------- noise level
def symbol_energy(X) -> float:
    X = np.asarray(X, dtype=np.float64)
    return float(np.mean(np.sum(X * X, axis=1)))


def sigma2_from_snr_db(X, snr_db: float) -> float:
    D = np.asarray(X).shape[1]
    return symbol_energy(X) / (D * 10.0 ** (snr_db / 10.0))


# --------------------------------------------------------------------------- workloads
SEED_BASE = 2104


@dataclass
class Workload:
    name: str
    X: np.ndarray
    labels: np.ndarray
    snr_db: list
    N: int
    seed: int
    extra: dict = field(default_factory=dict)

    @property
    def M(self):
        return self.X.shape[0]

    @property
    def D(self):
        return self.X.shape[1]

    @property
    def m(self):
        return int(self.M).bit_length() - 1

    def sigma2(self, snr_db):
        return sigma2_from_snr_db(self.X, snr_db)


def workload_4d64(N: int = 100_000):
    """4D M=64: product of two unit-energy 8-PSK (BRGC, 6 bits), 8 dB, N=1e5."""
    X, labels = product_4d_8psk()
    return Workload("4d_m64_8psk2_8dB", X, labels, [8.0], N, SEED_BASE + 0)


def workload_8d2048(N: int = 10_000_000, snrs=None):
    """8D M=2048 (11 bits): Gaussian points, unit energy per 2D, binary-index labels;
    N symbols per SNR, 4..14 dB in 1 dB steps."""
    X, labels = gaussian_constellation(2048, 8, SEED_BASE + 1)
    if snrs is None:
        snrs = [float(s) for s in range(4, 15)]
    return Workload("8d_m2048_gauss", X, labels, snrs, N, SEED_BASE + 1)


def workload_16d65536(N: int = 1_000_000, snrs=(10.0, 16.0)):
    """16D M=65536 (16 bits): Gaussian points, unit energy per 2D, binary-index labels."""
    X, labels = gaussian_constellation(65536, 16, SEED_BASE + 4)
    return Workload("16d_m65536_gauss", X, labels, list(snrs), N, SEED_BASE + 4)


def batched_instances(n_inst: int = 64, seed: int = SEED_BASE + 2, n_min: int = 100_000,
                      n_max: int = 4_000_000):
    """Mixed batch: M from {16,64,256,1024,4096} with weights (.30,.25,.20,.15,.10), D from
    {2,4,8} with weights (.5,.3,.2), N uniform in [n_min, n_max]; Gaussian points with
    per-instance seeds; 11 SNR points 2..12 dB."""
    rng = np.random.default_rng(seed)
    Ms = rng.choice([16, 64, 256, 1024, 4096], size=n_inst, p=[0.30, 0.25, 0.20, 0.15, 0.10])
    Ds = rng.choice([2, 4, 8], size=n_inst, p=[0.5, 0.3, 0.2])
    Ns = rng.integers(n_min, n_max + 1, size=n_inst)
    out = []
    for i in range(n_inst):
        X, labels = gaussian_constellation(int(Ms[i]), int(Ds[i]), seed * 1000 + i)
        out.append(Workload(f"inst{i}", X, labels, [float(s) for s in range(2, 13)], int(Ns[i]),
                            seed * 1000 + i))
    return out


def equaliser_input(B: int, N: int, M: int = 16, a: complex = 0.95 + 0.1j, b: complex = 0.08 - 0.04j,
                    isi: complex = 0.25 + 0.05j, snr_db: float = 25.0, seed: int = SEED_BASE + 5):
    """Seeded input of the widely-linear equaliser, time-major: B independent instances of
    N + 1 square M-QAM symbols (Gray labels) at 2 samples per symbol through an IQ
    imbalance (a s + b conj(s)), a half-symbol sample that mixes neighbours
    (isi s_n + conj(isi) s_{n+1}) and complex AWGN.  Returns x ((2N + 2, B) complex64),
    sent indices ((N + 1, B) uint32), reference points C ((M,) complex64) and labels."""
    X, labels = qam_gray(M)
    C = (X[:, 0].astype(np.float64) + 1j * X[:, 1].astype(np.float64))
    rng = np.random.default_rng(seed)
    tx = rng.integers(0, M, size=(N + 2, B), dtype=np.int64)
    s = C[tx]
    sig = 10.0 ** (-snr_db / 20.0) / math.sqrt(2.0)
    x = np.zeros((2 * N + 2, B), dtype=np.complex128)
    x[0::2] = a * s[:N + 1] + b * np.conj(s[:N + 1])
    x[1::2] = isi * s[:N + 1] + np.conj(isi) * s[1:N + 2]
    x += sig * (rng.standard_normal(x.shape) + 1j * rng.standard_normal(x.shape))
    return x.astype(np.complex64), tx[:N + 1].astype(np.uint32), C.astype(np.complex64), labels


def kk_input(T: int, A: float = 1.5, K: int = 24, snr_db: float = 30.0, seed: int = SEED_BASE + 6):
    """Seeded detected intensity of a Kramers-Kronig receiver: a carrier A plus a signal of
    K random tones on the positive FFT bins 1..K of a 1024-point block (|s| <= 0.3 A, so
    the field is minimum phase) with a little real noise on the intensity.  Returns
    (x (T,) float32 intensities, s (T,) complex128 the signal)."""
    rng = np.random.default_rng(seed)
    c = rng.standard_normal(K) + 1j * rng.standard_normal(K)
    c *= 0.3 * A / np.sum(np.abs(c))
    t = np.arange(T)
    s = np.zeros(T, dtype=np.complex128)
    for k in range(1, K + 1):
        s += c[k - 1] * np.exp(2j * np.pi * k * t / 1024)
    x = np.abs(A + s) ** 2
    x = x * (1.0 + 10.0 ** (-snr_db / 20.0) * rng.standard_normal(T))
    return x.astype(np.float32), s

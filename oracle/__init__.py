"""FP64 CPU oracle for bit-wise demapping over AWGN -- TEST INFRASTRUCTURE.

Only the test suite, the package smoke check and the benchmark's CPU-baseline leg
may import this module.  The product library (``paper_2104_06311_amd``) never
imports it and shares no code with it; both receive the same inputs from the
seeded generators in ``synth``.

The arithmetic lives in ``oracle.c`` (plain C, double precision, built with gcc
by ``oracle/build_oracle.py``); this file only marshals numpy arrays.  What each
function computes, and the passage of the paper it follows, is documented at the
top of ``oracle.c``.

Parity-pinning status of each function (what fixes it independently of itself
is in ``tests/test_oracle_pins.py``):
  llr_exact, llr_maxlog, gmi   pinned (closed forms, quadrature, brute force,
                               invariants)
  awgn / philox                pinned (published Philox known-answer vectors,
                               distribution tests, transform identities)
  mlp_forward / mlp_loss_grad  pinned (finite differences, closed-form layers)
  adam_step                    pinned (closed-form first step)
  hard_decision                pinned (brute force on tiny inputs)
  bit_errors, q_factor_db      pinned (BPSK/QPSK closed-form error rates, the
                               Gaussian tail identity)
  ddlms                        pinned (frozen identity taps reduce it to the sampled
                               input and a nearest-point search; the closed-form
                               inverse of a widely-linear distortion is a fixed point;
                               convergence to that inverse from identity taps)
  kk_field                     pinned (Hilbert of a bin-centred cosine is the sine; the
                               Kramers-Kronig theorem recovers a minimum-phase signal;
                               the downshift moves a tone to DC)
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from .build_oracle import build
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    I = ctypes.c_int
    I64 = ctypes.c_int64
    U64 = ctypes.c_uint64
    Dbl = ctypes.c_double
    lib.orc_philox4x32_10.argtypes = [P, P, P]
    lib.orc_gen_box_muller.argtypes = [P, P]
    lib.orc_awgn.argtypes = [P, I, I, U64, U64, I64, Dbl, P, P]
    lib.orc_llr_exact.argtypes = [P, P, I, I, P, I64, Dbl, P]
    lib.orc_llr_maxlog.argtypes = [P, P, I, I, P, I64, Dbl, P]
    lib.orc_hard_decision.argtypes = [P, I, I, P, I64, P]
    lib.orc_gmi_terms.argtypes = [P, I64, I, P, P, P, P]
    lib.orc_gmi.argtypes = [P, I64, I, P, P, P, P, P]
    lib.orc_mlp_forward.argtypes = [I, I, I, I, P, P, P, P, P, P, Dbl, Dbl, P, I64, P]
    lib.orc_mlp_loss_grad.argtypes = [I, I, I, I, P, P, P, P, P, P, Dbl, Dbl, P, P, I64, P, P, P, P, P, P]
    lib.orc_mlp_loss_grad.restype = Dbl
    lib.orc_gelu_eval.argtypes = [P, I64, P, P]
    lib.orc_adam_step.argtypes = [P, P, P, P, I64, I, Dbl, Dbl, Dbl, Dbl]
    lib.orc_ddlms.argtypes = [P, I64, I64, P, I, P, P, Dbl, P, P, P, P]
    lib.orc_num_threads.restype = I
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _u32(a):
    return np.ascontiguousarray(a, dtype=np.uint32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _log2_exact(M: int) -> int:
    m = int(M).bit_length() - 1
    if M < 2 or (1 << m) != M:
        raise ValueError(f"M={M} is not a power of two >= 2")
    return m


def philox4x32_10(ctr, key) -> np.ndarray:
    """Philox4x32-10 block (Salmon et al., SC'11) of counter ctr[4] under key key[2]."""
    lib = _load()
    c = _u32(ctr)
    k = _u32(key)
    out = np.zeros(4, dtype=np.uint32)
    lib.orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def box_muller(words) -> np.ndarray:
    """The generator's normal pair (z0, z1) for a radius word and an angle word."""
    lib = _load()
    w = _u32(words)
    z = np.zeros(2, dtype=np.float64)
    lib.orc_gen_box_muller(_ptr(w), _ptr(z))
    return z


def awgn(X, seed: int, offset: int, N: int, sigma: float):
    """CPU twin of the counter-based AWGN channel: returns (tx indices uint32[N], y float32[N, D])."""
    lib = _load()
    X = _f32(X)
    M, D = X.shape
    _log2_exact(M)
    tx = np.zeros(N, dtype=np.uint32)
    y = np.zeros((N, D), dtype=np.float32)
    lib.orc_awgn(_ptr(X), M, D, ctypes.c_uint64(seed), ctypes.c_uint64(offset), N, float(sigma),
                 _ptr(tx), _ptr(y))
    return tx, y


def llr_exact(X, labels, y, sigma2: float) -> np.ndarray:
    """Exact bit-wise LLRs, float64[N, m]; column k is label bit m-1-k; sign ln P(0)/P(1)."""
    lib = _load()
    X = _f32(X)
    labels = _u32(labels)
    y = _f32(y)
    M, D = X.shape
    m = _log2_exact(M)
    N = y.shape[0]
    out = np.zeros((N, m), dtype=np.float64)
    lib.orc_llr_exact(_ptr(X), _ptr(labels), M, D, _ptr(y), N, float(sigma2), _ptr(out))
    return out


def llr_maxlog(X, labels, y, sigma2: float) -> np.ndarray:
    """Max-log bit-wise LLRs, float64[N, m]."""
    lib = _load()
    X = _f32(X)
    labels = _u32(labels)
    y = _f32(y)
    M, D = X.shape
    m = _log2_exact(M)
    N = y.shape[0]
    out = np.zeros((N, m), dtype=np.float64)
    lib.orc_llr_maxlog(_ptr(X), _ptr(labels), M, D, _ptr(y), N, float(sigma2), _ptr(out))
    return out


def hard_decision(X, y) -> np.ndarray:
    """Index of the nearest constellation point for every received symbol."""
    lib = _load()
    X = _f32(X)
    y = _f32(y)
    M, D = X.shape
    N = y.shape[0]
    out = np.zeros(N, dtype=np.uint32)
    lib.orc_hard_decision(_ptr(X), M, D, _ptr(y), N, _ptr(out))
    return out


def bit_errors(decided_labels, tx, labels, m: int) -> np.ndarray:
    """Bit errors per label bit column (column k = bit m-1-k) of decided labels against
    the labels of the transmitted points: the hard-decision receiver of the paper's
    Results section, which reports the Q-factor of the bit-error rate."""
    sent = np.asarray(labels, dtype=np.int64)[np.asarray(tx, dtype=np.int64)]
    diff = sent ^ np.asarray(decided_labels, dtype=np.int64)
    return np.array([int(((diff >> (m - 1 - k)) & 1).sum()) for k in range(m)], dtype=np.int64)


def llr_decisions(llr) -> np.ndarray:
    """Decided labels from LLR signs: bit m-1-k is 1 where column k is negative."""
    L = np.asarray(llr)
    m = L.shape[1]
    out = np.zeros(L.shape[0], dtype=np.int64)
    for k in range(m):
        out |= (L[:, k] < 0).astype(np.int64) << (m - 1 - k)
    return out


def q_factor_db(ber: float) -> float:
    """Q-factor of a bit-error rate, 20 log10(sqrt(2) erfc^-1(2 BER)): the Gaussian tail
    relation BER = erfc(Q / sqrt 2) / 2 (the paper quotes Q from measured BER without
    printing the relation; this is the standard one)."""
    from scipy.special import erfcinv
    return float(20.0 * np.log10(np.sqrt(2.0) * erfcinv(2.0 * ber)))


def gmi_terms(llr, tx, labels):
    """Per-symbol bits lost T_n and per-(symbol, bit) terms."""
    lib = _load()
    llr = _f64(llr)
    tx = _u32(tx)
    labels = _u32(labels)
    N, m = llr.shape
    T = np.zeros(N, dtype=np.float64)
    Tb = np.zeros((N, m), dtype=np.float64)
    lib.orc_gmi_terms(_ptr(llr), N, m, _ptr(tx), _ptr(labels), _ptr(T), _ptr(Tb))
    return T, Tb


def gmi(llr, tx, labels):
    """(GMI in bits per symbol, per-bit GMI float64[m], standard error)."""
    lib = _load()
    llr = _f64(llr)
    tx = _u32(tx)
    labels = _u32(labels)
    N, m = llr.shape
    if N == 0:
        raise ValueError("GMI of an empty sample is undefined")
    g = np.zeros(1, dtype=np.float64)
    gb = np.zeros(m, dtype=np.float64)
    se = np.zeros(1, dtype=np.float64)
    lib.orc_gmi(_ptr(llr), N, m, _ptr(tx), _ptr(labels), _ptr(g), _ptr(gb), _ptr(se))
    return float(g[0]), gb, float(se[0])


class MLPParams:
    """FP64 parameters of the D -> H1 -> H2 -> m GELU network (row-major [out][in]) and its
    fixed input / output scales: f(y) = out_scale * net(in_scale * y)."""

    def __init__(self, W1, b1, W2, b2, W3, b3, in_scale=1.0, out_scale=1.0):
        self.in_scale = float(in_scale)
        self.out_scale = float(out_scale)
        self.W1 = _f64(W1)
        self.b1 = _f64(b1)
        self.W2 = _f64(W2)
        self.b2 = _f64(b2)
        self.W3 = _f64(W3)
        self.b3 = _f64(b3)

    @property
    def dims(self):
        H1, D = self.W1.shape
        H2 = self.W2.shape[0]
        m = self.W3.shape[0]
        return D, H1, H2, m

    def flat(self):
        return [self.W1, self.b1, self.W2, self.b2, self.W3, self.b3]


def gelu(a):
    """(g(a), g'(a)) of the network's activation, GELU g(a) = a Phi(a), at the points a."""
    a = _f64(np.atleast_1d(a))
    g = np.empty_like(a)
    dg = np.empty_like(a)
    _load().orc_gelu_eval(_ptr(a), a.size, _ptr(g), _ptr(dg))
    return g, dg


def mlp_forward(p: MLPParams, y) -> np.ndarray:
    lib = _load()
    y = _f32(y)
    D, H1, H2, m = p.dims
    N = y.shape[0]
    out = np.zeros((N, m), dtype=np.float64)
    lib.orc_mlp_forward(D, H1, H2, m, *[_ptr(a) for a in p.flat()], p.in_scale, p.out_scale, _ptr(y), N, _ptr(out))
    return out


def mlp_loss_grad(p: MLPParams, y, target):
    """(mean distillation loss, [gW1, gb1, gW2, gb2, gW3, gb3])."""
    lib = _load()
    y = _f32(y)
    target = _f32(target)
    D, H1, H2, m = p.dims
    B = y.shape[0]
    grads = [np.zeros_like(a) for a in p.flat()]
    loss = lib.orc_mlp_loss_grad(D, H1, H2, m, *[_ptr(a) for a in p.flat()], p.in_scale, p.out_scale, _ptr(y),
                                 _ptr(target), B,
                                 *[_ptr(g) for g in grads])
    return float(loss), grads


def adam_step(w, g, m1, m2, t: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """In-place Adam update of float64 arrays w, m1, m2 with gradient g."""
    lib = _load()
    for a in (w, g, m1, m2):
        assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    lib.orc_adam_step(_ptr(w), _ptr(g), _ptr(m1), _ptr(m2), w.size, t, lr, beta1, beta2, eps)


def num_threads() -> int:
    """OpenMP threads used by the parallel oracle loops."""
    return int(_load().orc_num_threads())


def ddlms(x, C, h0, g0, mu: float):
    """Four-tap widely-linear DD-LMS equaliser over B independent instances (see orc_ddlms
    in oracle.c).  x: (2N + 2, B) complex64 samples, time-major; C: (M,) complex reference
    points; h0, g0: 4 complex starting taps.  Returns (dec (N, B) uint32, z (N, B)
    complex64, h (B, 4) complex128, g (B, 4) complex128)."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.complex64)
    T, B = x.shape
    N = (T - 2) // 2
    if T != 2 * N + 2 or N < 0:
        raise ValueError("x must hold 2 N + 2 samples per instance")
    C = np.ascontiguousarray(C, dtype=np.complex64)
    h0 = np.ascontiguousarray(h0, dtype=np.complex128)
    g0 = np.ascontiguousarray(g0, dtype=np.complex128)
    dec = np.zeros((N, B), dtype=np.uint32)
    z = np.zeros((N, B), dtype=np.complex64)
    h = np.zeros((B, 4), dtype=np.complex128)
    g = np.zeros((B, 4), dtype=np.complex128)
    lib.orc_ddlms(_ptr(x), B, N, _ptr(C), C.shape[0], _ptr(h0), _ptr(g0), float(mu), _ptr(dec), _ptr(z), _ptr(h),
                  _ptr(g))
    return dec, z, h, g


def kk_field(x, A: float, nu: float, nfft: int = 1024):
    """Kramers-Kronig front end of the paper's receiver (section "Experimental setup", the
    DSP-chain paragraph: square root and logarithm of the detected samples, a Hilbert
    transform by 1024-point overlap-save FFTs, the field rebuilt from amplitude and phase
    and downshifted to DC).  FP64, written from the definition:
      l_t   = ln sqrt(x_t) = 0.5 ln x_t                      (x: real intensity samples)
      phi   = Hilbert(l), block k of the stream: the FFT of the nfft samples starting at
              k nfft/2 - nfft/4 (zero outside the stream) is multiplied by the analytic
              mask (1, 2 .. 2, 1, 0 .. 0), transformed back, and the imaginary parts of
              its middle nfft/2 samples are phi for t in [k nfft/2, (k+1) nfft/2)
      E_t   = exp(l_t) (cos phi_t + i sin phi_t)
      s_t   = (E_t - A) exp(-i 2 pi frac(nu t))             (carrier removed, downshifted)
    x holds T samples, T a multiple of nfft/2.  Returns s as complex128."""
    x = np.asarray(x, dtype=np.float64)
    T = x.shape[0]
    hop, pad = nfft // 2, nfft // 4
    if T % hop:
        raise ValueError("T must be a multiple of nfft / 2")
    l = 0.5 * np.log(np.fmax(x, 2.0 ** -126))   # samples below the smallest normal float are floored
    U = np.zeros(nfft)
    U[0] = 1.0
    U[1:nfft // 2] = 2.0
    U[nfft // 2] = 1.0
    phi = np.zeros(T)
    for k in range(T // hop):
        idx = np.arange(k * hop - pad, k * hop - pad + nfft)
        inside = (idx >= 0) & (idx < T)
        seg = np.zeros(nfft)
        seg[inside] = l[idx[inside]]
        za = np.fft.ifft(np.fft.fft(seg) * U)
        phi[k * hop:(k + 1) * hop] = za.imag[pad:pad + hop]
    E = np.exp(l) * (np.cos(phi) + 1j * np.sin(phi))
    t = np.arange(T, dtype=np.float64)
    frac = nu * t - np.floor(nu * t)
    return (E - A) * np.exp(-2j * np.pi * frac)

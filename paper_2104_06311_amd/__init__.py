"""MI355X-native bit-wise soft demapping of labelled multidimensional constellations
over AWGN: counter-based AWGN channel, exact and max-log LLRs, Monte-Carlo GMI.

Thin Python layer over the C ABI of ``libmdemap.so`` (see ``include/mdemap.h``):
the functions below have the names of the C entry points and only marshal
arguments.  Inputs are CUDA/HIP torch tensors; outputs are allocated with torch on
the same device and every call is enqueued on torch's current stream.
"""
from __future__ import annotations

import torch

from ._lib import MdemapError, PREC, check, lib

__all__ = ["awgn_sample", "llr_exact", "llr_exact_noalloc", "llr_exact_gmi", "gmi_status", "alloc_fault_inject", "alloc_stats",
           "llr_maxlog", "llr_path_counts", "gmi_reduce", "ber_count", "q_factor_db", "llr_learned", "MLP", "SweepPlan", "RxStream", "release_cache",
           "ddlms_equalize", "ddlms_equalize_chain", "kk_frontend", "ubench", "UBENCH_KINDS", "kernel_timing", "kernel_timing_read", "MdemapError",
           "log2_exact"]


def _stream():
    return ctypes_void(torch.cuda.current_stream().cuda_stream)


def ctypes_void(v):
    import ctypes
    return ctypes.c_void_p(v)


def _ptr(t):
    return None if t is None else t.data_ptr()


def _dev(t: torch.Tensor, name: str, dtype: torch.dtype, ndim: int):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must live on the GPU")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if t.dim() != ndim:
        raise ValueError(f"{name} must have {ndim} dimensions")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _out(out, shape, dtype: torch.dtype, device):
    """A caller-given output tensor must be a contiguous device tensor of the right shape."""
    if out is None:
        return torch.empty(shape, dtype=dtype, device=device)
    _dev(out, "out", dtype, len(shape))
    if tuple(out.shape) != tuple(shape) or out.device != device:
        raise ValueError(f"out must be {list(shape)} on {device}")
    return out


def log2_exact(M: int) -> int:
    m = int(M).bit_length() - 1
    if M < 2 or (1 << m) != M:
        raise ValueError(f"M={M} is not a power of two >= 2")
    return m


def awgn_sample(X: torch.Tensor, seed: int, offset: int, N: int, sigma: float, tx=None, y=None):
    """(tx uint32[N] as int32 storage, y float32[N, D]) for the channel defined in mdemap.h."""
    _dev(X, "X", torch.float32, 2)
    M, D = X.shape
    if N < 0:
        raise ValueError("N must be >= 0")
    if tx is None:
        tx = torch.empty(N, dtype=torch.int32, device=X.device)
    else:
        _dev(tx, "tx", torch.int32, 1)
        if tx.shape[0] != N or tx.device != X.device:
            raise ValueError("tx must hold N entries on X's device")
    if y is None:
        y = torch.empty((N, D), dtype=torch.float32, device=X.device)
    else:
        _dev(y, "y", torch.float32, 2)
        if tuple(y.shape) != (N, D) or y.device != X.device:
            raise ValueError("y must be [N, D] on X's device")
    st = lib().awgn_sample(_ptr(X), M, D, seed & (2 ** 64 - 1), offset & (2 ** 64 - 1), N, float(sigma),
                           _ptr(tx), _ptr(y), _stream())
    check("awgn_sample", st)
    return tx, y


def _demap_args(X, labels, y):
    _dev(X, "X", torch.float32, 2)
    _dev(labels, "labels", torch.int32, 1)
    _dev(y, "y", torch.float32, 2)
    M, D = X.shape
    if labels.shape[0] != M:
        raise ValueError("labels must have M entries")
    if y.shape[1] != D:
        raise ValueError("y must have D columns")
    if labels.device != X.device or y.device != X.device:
        raise ValueError("X, labels and y must be on one device")
    return M, D, y.shape[0]


def llr_exact(X, labels, y, sigma2: float, prec: str = "fp32", out=None):
    """Exact bit-wise LLRs float32[N, m] (column k = label bit m-1-k, sign ln P0/P1)."""
    M, D, N = _demap_args(X, labels, y)
    m = log2_exact(M)
    out = _out(out, (N, m), torch.float32, X.device)
    st = lib().llr_exact(_ptr(X), _ptr(labels), M, D, _ptr(y), N, float(sigma2), PREC[prec], _ptr(out), _stream())
    check("llr_exact", st)
    return out


def llr_exact_noalloc(X, labels, y, sigma2: float, prec: str = "fp32", out=None):
    """llr_exact through the allocation-free entry point (N <= 2^20; calls overlapping on
    one device race, see mdemap.h).  Pass `out` to keep the call free of allocations."""
    M, D, N = _demap_args(X, labels, y)
    m = log2_exact(M)
    out = _out(out, (N, m), torch.float32, X.device)
    st = lib().llr_exact_noalloc(_ptr(X), _ptr(labels), M, D, _ptr(y), N, float(sigma2), PREC[prec], _ptr(out),
                                 _stream())
    check("llr_exact_noalloc", st)
    return out


def llr_maxlog(X, labels, y, sigma2: float, out=None):
    """Max-log bit-wise LLRs float32[N, m]."""
    M, D, N = _demap_args(X, labels, y)
    m = log2_exact(M)
    out = _out(out, (N, m), torch.float32, X.device)
    st = lib().llr_maxlog(_ptr(X), _ptr(labels), M, D, _ptr(y), N, float(sigma2), _ptr(out), _stream())
    check("llr_maxlog", st)
    return out


def ber_count(llr, tx, labels, per_bit: bool = True):
    """(bit errors int64[1], per-column bit errors int64[m] or None), device tensors; the
    hard decision of column k is 1 where the LLR is negative."""
    _dev(llr, "llr", torch.float32, 2)
    _dev(tx, "tx", torch.int32, 1)
    _dev(labels, "labels", torch.int32, 1)
    N, m = llr.shape
    if tx.shape[0] != N:
        raise ValueError("tx must have N entries")
    if labels.shape[0] != (1 << m):
        raise ValueError("labels must have 2^m entries")
    if tx.device != llr.device or labels.device != llr.device:
        raise ValueError("llr, tx and labels must be on one device")
    errors = torch.zeros(1, dtype=torch.int64, device=llr.device)
    bit_errors = torch.zeros(m, dtype=torch.int64, device=llr.device) if per_bit else None
    check("ber_count", lib().ber_count(_ptr(llr), N, m, _ptr(tx), _ptr(labels), _ptr(bit_errors), _ptr(errors),
                                        _stream()))
    return errors, bit_errors


def q_factor_db(errors, n_bits: int):
    """Q-factor in dB of a bit-error count (device int64[1] tensor, e.g. ber_count's first
    output) over n_bits bits: a device float64[1] tensor, NaN where BER is 0 or >= 1/2."""
    _dev(errors, "errors", torch.int64, 1)
    if errors.shape[0] != 1:
        raise ValueError("errors must hold one count")
    q = torch.empty(1, dtype=torch.float64, device=errors.device)
    check("q_factor_db", lib().q_factor_db(_ptr(errors), int(n_bits), _ptr(q), _stream()))
    return q


def llr_path_counts():
    """(symbols of the wide-range pass, symbols of the FP64 careful kernel) of the last
    llr_exact / llr_maxlog call on torch's current stream; waits for that stream."""
    import ctypes
    a, b = ctypes.c_int64(0), ctypes.c_int64(0)
    check("llr_path_counts", lib().llr_path_counts(_stream(), ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def gmi_reduce(llr, tx, labels, per_bit: bool = True, se: bool = True):
    """(gmi float64[1], gmi_per_bit float64[m] or None, se float64[1] or None), device tensors."""
    _dev(llr, "llr", torch.float32, 2)
    _dev(tx, "tx", torch.int32, 1)
    _dev(labels, "labels", torch.int32, 1)
    N, m = llr.shape
    if tx.shape[0] != N:
        raise ValueError("tx must have N entries")
    if labels.shape[0] != (1 << m):
        raise ValueError("labels must have 2^m entries")
    if tx.device != llr.device or labels.device != llr.device:
        raise ValueError("llr, tx and labels must be on one device")
    g = torch.empty(1, dtype=torch.float64, device=llr.device)
    gb = torch.empty(m, dtype=torch.float64, device=llr.device) if per_bit else None
    s = torch.empty(1, dtype=torch.float64, device=llr.device) if se else None
    st = lib().gmi_reduce(_ptr(llr), N, m, _ptr(tx), _ptr(labels), _ptr(g), _ptr(gb), _ptr(s), _stream())
    check("gmi_reduce", st)
    return g, gb, s


def gmi_status():
    """Number of symbols with a non-finite loss term in the last GMI on the current stream
    (waits for the stream).  Returns the count; 0 means the GMI is a finite average."""
    import ctypes
    n = ctypes.c_int64()
    st = lib().gmi_status(_stream(), ctypes.byref(n))
    if st not in (0, -9):
        check("gmi_status", st)
    return n.value


def llr_exact_gmi(X, labels, y, tx, sigma2: float, prec: str = "fp32", out=None, se: bool = True):
    """Exact LLRs float32[N, m] and their GMI (float64[1], SE float64[1] or None) from one
    fused pass (llr_exact_gmi in mdemap.h)."""
    M, D, N = _demap_args(X, labels, y)
    _dev(tx, "tx", torch.int32, 1)
    if tx.shape[0] != N or tx.device != X.device:
        raise ValueError("tx must hold N indices on the constellation's device")
    m = log2_exact(M)
    out = _out(out, (N, m), torch.float32, X.device)
    g = torch.empty(1, dtype=torch.float64, device=X.device)
    sv = torch.empty(1, dtype=torch.float64, device=X.device) if se else None
    check("llr_exact_gmi", lib().llr_exact_gmi(_ptr(X), _ptr(labels), M, D, _ptr(y), N, float(sigma2), PREC[prec],
                                               _ptr(tx), _ptr(out), _ptr(g), _ptr(sv), _stream()))
    return out, g, sv


def alloc_fault_inject(k: int):
    """Test hook: the k-th next device allocation of the library fails (k < 0: off)."""
    check("alloc_fault_inject", lib().alloc_fault_inject(int(k)))


def alloc_stats():
    """(bytes, allocations) of device memory the library holds right now."""
    import ctypes
    nb, na = ctypes.c_int64(), ctypes.c_int64()
    check("alloc_stats", lib().alloc_stats(ctypes.byref(nb), ctypes.byref(na)))
    return nb.value, na.value


def release_cache():
    check("release_cache", lib().release_cache())


def ddlms_equalize(x, C, h0, g0, mu: float, want_z: bool = True, want_taps: bool = True):
    """Four-tap widely-linear DD-LMS equaliser over B independent instances (see
    ddlms_equalize in mdemap.h).  x: (2N + 2, B) complex64 device tensor, time-major;
    C: (M,) complex64 device tensor of reference points; h0, g0: 4 complex starting taps.
    Returns (dec (N, B) int32, z (N, B) complex64 or None, h (B, 4) complex128 or None,
    g (B, 4) complex128 or None)."""
    import ctypes
    import numpy as np
    if not isinstance(x, torch.Tensor) or x.dtype != torch.complex64 or x.dim() != 2 or not x.is_cuda:
        raise ValueError("x must be a 2-D complex64 device tensor")
    if not isinstance(C, torch.Tensor) or C.dtype != torch.complex64 or C.dim() != 1 or not C.is_cuda:
        raise ValueError("C must be a 1-D complex64 device tensor")
    x = x.contiguous()
    C = C.contiguous()
    T, B = x.shape
    if T < 2 or T % 2:
        raise ValueError("x must hold 2 N + 2 samples per instance")
    N = (T - 2) // 2
    t0 = np.ascontiguousarray(np.asarray(h0, dtype=np.complex128).reshape(4)).view(np.float64)
    t1 = np.ascontiguousarray(np.asarray(g0, dtype=np.complex128).reshape(4)).view(np.float64)
    dec = torch.empty((N, B), dtype=torch.int32, device=x.device)
    z = torch.empty((N, B), dtype=torch.complex64, device=x.device) if want_z else None
    h = torch.empty((B, 4), dtype=torch.complex128, device=x.device) if want_taps else None
    g = torch.empty((B, 4), dtype=torch.complex128, device=x.device) if want_taps else None
    st = lib().ddlms_equalize(_ptr(x), B, N, _ptr(C), C.shape[0], t0.ctypes.data_as(ctypes.c_void_p),
                              t1.ctypes.data_as(ctypes.c_void_p), float(mu), _ptr(dec), _ptr(z), _ptr(h), _ptr(g),
                              _stream())
    check("ddlms_equalize", st)
    return dec, z, h, g


def ddlms_equalize_chain(x, C, h, g, mu: float, want_z: bool = True):
    """ddlms_equalize continued from each instance's own taps (ddlms_equalize_chain in
    mdemap.h): h, g (B, 4) complex128 device tensors, updated in place to the final taps.
    x (2N + 2, B) complex64 time-major, C (M,) complex64.  Returns (dec (N, B) int32, z (N, B)
    complex64 or None)."""
    if not isinstance(x, torch.Tensor) or x.dtype != torch.complex64 or x.dim() != 2 or not x.is_cuda:
        raise ValueError("x must be a 2-D complex64 device tensor")
    if not isinstance(C, torch.Tensor) or C.dtype != torch.complex64 or C.dim() != 1 or not C.is_cuda:
        raise ValueError("C must be a 1-D complex64 device tensor")
    T, B = x.shape
    for name, t in (("h", h), ("g", g)):
        if (not isinstance(t, torch.Tensor) or t.dtype != torch.complex128 or tuple(t.shape) != (B, 4)
                or not t.is_cuda or not t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous (B, 4) complex128 device tensor")
    if T < 2 or T % 2:
        raise ValueError("x must hold 2 N + 2 samples per instance")
    x = x.contiguous()
    C = C.contiguous()
    N = (T - 2) // 2
    dec = torch.empty((N, B), dtype=torch.int32, device=x.device)
    z = torch.empty((N, B), dtype=torch.complex64, device=x.device) if want_z else None
    check("ddlms_equalize_chain", lib().ddlms_equalize_chain(_ptr(x), B, N, _ptr(C), C.shape[0], float(mu), _ptr(dec),
                                                             _ptr(z), _ptr(h), _ptr(g), _stream()))
    return dec, z


def kk_frontend(x, A: float, nu: float, out=None):
    """Kramers-Kronig front end (see kk_frontend in mdemap.h): x is a 1-D float32 device
    tensor of T intensity samples (T a multiple of 512); returns T complex64 samples."""
    if not isinstance(x, torch.Tensor) or x.dtype != torch.float32 or x.dim() != 1 or not x.is_cuda:
        raise ValueError("x must be a 1-D float32 device tensor")
    x = x.contiguous()
    T = x.shape[0]
    if out is None:
        out = torch.empty(T, dtype=torch.complex64, device=x.device)
    elif out.dtype != torch.complex64 or out.shape != (T,) or not out.is_contiguous():
        raise ValueError("out must be a contiguous complex64 tensor of T samples")
    check("kk_frontend", lib().kk_frontend(_ptr(x), T, float(A), float(nu), _ptr(out), _stream()))
    return out


def kernel_timing(enable: bool):
    """Switch event timing of the demappers' fast kernel on or off on the current stream
    (kernel_timing in mdemap.h)."""
    check("kernel_timing", lib().kernel_timing(1 if enable else 0, _stream()))


def kernel_timing_read():
    """(summed milliseconds, launches) of the fast kernels timed on the current stream
    since the last read (kernel_timing_read in mdemap.h)."""
    import ctypes
    ms, n = ctypes.c_double(), ctypes.c_int64()
    check("kernel_timing_read", lib().kernel_timing_read(ctypes.byref(ms), ctypes.byref(n), _stream()))
    return ms.value, n.value


UBENCH_KINDS = {"exp": 0, "add_f32": 1, "mfma_f16": 2, "mfma_bf16": 3, "mfma_f32": 4, "copy": 5, "exp_add2": 6, "tile_mix": 7, "tile_mix4": 8, "tile_mix1": 9}


def ubench(kind: str, work: int = 0, src=None, dst=None):
    """Measured peak rate of one instruction kind on the current device (see ubench in
    mdemap.h): returns (rate, ms).  kind "copy" needs device tensors src and dst of at
    least `work` bytes."""
    import ctypes
    if kind == "copy":
        for name, t in (("src", src), ("dst", dst)):
            if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous():
                raise ValueError(f"ubench copy: {name} must be a contiguous device tensor")
            if t.numel() * t.element_size() < work:
                raise ValueError(f"ubench copy: {name} holds fewer than {work} bytes")
    rate, ms = ctypes.c_double(), ctypes.c_double()
    st = lib().ubench(UBENCH_KINDS[kind], int(work), _ptr(src) if src is not None else None,
                      _ptr(dst) if dst is not None else None, ctypes.byref(rate), ctypes.byref(ms), _stream())
    check("ubench", st)
    return rate.value, ms.value


# ----------------------------------------------------------------------------- learned demapper
class MLP:
    """Handle of a learned demapper D -> hidden -> hidden -> m (see mlp_* in mdemap.h)."""

    def __init__(self, D: int = 0, hidden: int = 0, m: int = 0, seed: int = 0, _handle=None):
        import ctypes
        if _handle is None:
            h = ctypes.c_void_p()
            check("mlp_create", lib().mlp_create(D, hidden, m, seed & (2 ** 64 - 1), ctypes.byref(h)))
            _handle = h
        self._h = _handle
        d, hh, mm, st = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int64()
        check("mlp_info", lib().mlp_info(self._h, ctypes.byref(d), ctypes.byref(hh), ctypes.byref(mm),
                                         ctypes.byref(st)))
        self.D, self.hidden, self.m = d.value, hh.value, mm.value

    @property
    def handle(self):
        return self._h

    @property
    def num_params(self) -> int:
        return int(lib().mlp_num_params(self._h))

    @property
    def step(self) -> int:
        import ctypes
        st = ctypes.c_int64()
        check("mlp_info", lib().mlp_info(self._h, None, None, None, ctypes.byref(st)))
        return st.value

    def set_scales(self, in_scale: float, out_scale: float):
        """Fixed input / output scales: f(y) = out_scale * net(in_scale * y)."""
        check("mlp_set_scales", lib().mlp_set_scales(self._h, float(in_scale), float(out_scale)))

    @property
    def scales(self):
        import ctypes
        a, b = ctypes.c_float(), ctypes.c_float()
        check("mlp_get_scales", lib().mlp_get_scales(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def close(self):
        if self._h is not None:
            check("mlp_destroy", lib().mlp_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            if self._h is not None:
                lib().mlp_destroy(self._h)
        except Exception:
            pass

    def get(self, which: int = 0):
        import numpy as np
        out = np.zeros(self.num_params, dtype=np.float32)
        check("mlp_get", lib().mlp_get(self._h, which, out.ctypes.data))
        return out

    def set(self, values, which: int = 0):
        import numpy as np
        v = np.ascontiguousarray(values, dtype=np.float32)
        if v.size != self.num_params:
            raise ValueError("wrong number of parameters")
        check("mlp_set", lib().mlp_set(self._h, which, v.ctypes.data))

    def grad(self, y, target):
        _dev(y, "y", torch.float32, 2)
        _dev(target, "target", torch.float32, 2)
        loss = torch.empty(1, dtype=torch.float64, device=y.device)
        check("mlp_grad", lib().mlp_grad(self._h, _ptr(y), _ptr(target), y.shape[0], _ptr(loss), _stream()))
        return loss

    def adam_step(self, lr: float):
        check("mlp_adam_step", lib().mlp_adam_step(self._h, float(lr), _stream()))

    def train_step(self, y, target, lr: float):
        _dev(y, "y", torch.float32, 2)
        _dev(target, "target", torch.float32, 2)
        loss = torch.empty(1, dtype=torch.float64, device=y.device)
        check("mlp_train_step", lib().mlp_train_step(self._h, _ptr(y), _ptr(target), y.shape[0], float(lr),
                                                     _ptr(loss), _stream()))
        return loss

    def fit(self, y, target, steps: int, batch: int = 4096, lr_max: float = 1e-3, lr_min: float = 1e-5,
            seed: int = 0, trace: bool = True):
        _dev(y, "y", torch.float32, 2)
        _dev(target, "target", torch.float32, 2)
        tr = torch.empty(max(steps, 1), dtype=torch.float64, device=y.device) if trace else None
        check("mlp_fit", lib().mlp_fit(self._h, _ptr(y), _ptr(target), y.shape[0], steps, batch, float(lr_max),
                                       float(lr_min), seed & (2 ** 64 - 1), _ptr(tr), _stream()))
        return tr

    def save(self, path: str):
        check("mlp_save", lib().mlp_save(self._h, path.encode()))

    @classmethod
    def load(cls, path: str) -> "MLP":
        import ctypes
        h = ctypes.c_void_p()
        check("mlp_load", lib().mlp_load(path.encode(), ctypes.byref(h)))
        return cls(_handle=h)


def llr_learned(mlp: MLP, y, out=None):
    """Network LLRs float32[N, m] for received symbols y float32[N, D]."""
    _dev(y, "y", torch.float32, 2)
    if y.shape[1] != mlp.D:
        raise ValueError("y must have D columns")
    N = y.shape[0]
    out = _out(out, (N, mlp.m), torch.float32, y.device)
    check("llr_learned", lib().llr_learned(mlp.handle, _ptr(y), N, _ptr(out), _stream()))
    return out


# ----------------------------------------------------------------------------- batched sweep
class RxStream:
    """Streaming receiver (rx_* in mdemap.h): buffers of a host-resident symbol stream
    demapped on several HIP streams with overlapping copies and kernels.  X float32 [M, D]
    and labels int32 [M] on the GPU (copied at creation); mode "hard" (max-log LLRs, nearest-
    point decisions) or "exact" (exact LLRs)."""

    def __init__(self, X, labels, sigma2: float, mode: str = "hard", n_streams: int = 4,
                 buf_symbols: int = 1 << 20, bin_symbols: int | None = None, equaliser: dict | None = None):
        """equaliser: None, or {"instances": P, "mu": step, "h0": 4 complex, "g0": 4 complex}:
        the ring then holds complex samples (see run) that pass the DD-LMS equaliser, taps
        carried from buffer to buffer, before demapping."""
        import ctypes
        import numpy as np
        from ._lib import RX_MODE, RxConfig
        _dev(X, "X", torch.float32, 2)
        _dev(labels, "labels", torch.int32, 1)
        if mode not in RX_MODE:
            raise ValueError("mode must be 'hard' or 'exact'")
        self.M, self.D = X.shape
        self.m = self.M.bit_length() - 1
        self.mode = mode
        self.buf_symbols = int(buf_symbols)
        self.bin_symbols = int(bin_symbols if bin_symbols is not None else buf_symbols)
        self.P = 0
        cfg = RxConfig(RX_MODE[mode], int(n_streams), self.buf_symbols, self.bin_symbols)
        if equaliser is not None:
            self.P = int(equaliser["instances"])
            cfg.eq_instances = self.P
            cfg.eq_mu = float(equaliser["mu"])
            h0 = np.ascontiguousarray(np.asarray(equaliser["h0"], dtype=np.complex128).reshape(4)).view(np.float64)
            g0 = np.ascontiguousarray(np.asarray(equaliser["g0"], dtype=np.complex128).reshape(4)).view(np.float64)
            for i in range(8):
                cfg.eq_h0[i] = float(h0[i])
                cfg.eq_g0[i] = float(g0[i])
        h = ctypes.c_void_p()
        check("rx_create", lib().rx_create(_ptr(X), _ptr(labels), self.M, self.D, float(sigma2), ctypes.byref(cfg),
                                           ctypes.byref(h)))
        self._h = h

    def run(self, y, tx=None, total: int | None = None, out=None, stats: bool = True):
        """Runs `total` stream symbols (default: the ring once) from the pinned host ring y
        float32 [N, D] (with the equaliser: complex samples float32 [2 N/P + 2, 2 P], stream
        symbol i being symbol i // P of channel i % P) and tx int32 [N] (stream order);
        decisions (hard, int32 [N]) or LLRs (exact, float32 [N, m]) go to the pinned host ring
        `out` if given.  Returns a dict with the per-bin bit errors and GMI (when tx is given)
        and the run's timing."""
        import numpy as np
        for name, t in (("y", y), ("tx", tx), ("out", out)):
            if t is not None and (t.is_cuda or not t.is_pinned() or not t.is_contiguous()):
                raise ValueError(f"{name} must be a contiguous pinned host tensor")
        if self.P:
            # complex samples, time-major: (2 N/P + 2) rows of P (re, im) pairs
            if (y.dtype != torch.float32 or y.dim() != 2 or y.shape[1] != 2 * self.P or y.shape[0] < 4
                    or y.shape[0] % 2):
                raise ValueError("with the equaliser y must be float32 [2 N/P + 2, 2 P]")
            N = (y.shape[0] - 2) // 2 * self.P
        else:
            if y.dtype != torch.float32 or y.dim() != 2 or y.shape[1] != self.D:
                raise ValueError("y must be float32 [N, D]")
            N = y.shape[0]
        if tx is not None and (tx.dtype != torch.int32 or tx.shape != (N,)):
            raise ValueError("tx must be int32 [N]")
        if out is not None:
            want = (torch.int32, (N,)) if self.mode == "hard" else (torch.float32, (N, self.m))
            if out.dtype != want[0] or tuple(out.shape) != want[1]:
                raise ValueError(f"out must be {want[0]} {list(want[1])}")
        total = N if total is None else int(total)
        nb = (total + self.bin_symbols - 1) // self.bin_symbols
        err = np.zeros(nb, dtype=np.uint64) if tx is not None else None
        gmi = np.zeros(nb, dtype=np.float64) if tx is not None else None
        st = np.zeros(4, dtype=np.float64)
        check("rx_run", lib().rx_run(self._h, y.data_ptr(), tx.data_ptr() if tx is not None else None, N, total,
                                     out.data_ptr() if out is not None else None,
                                     err.ctypes.data if err is not None else None,
                                     gmi.ctypes.data if gmi is not None else None, st.ctypes.data if stats else None))
        return {"bin_errors": err, "bin_gmi": gmi, "seconds": float(st[0]), "symbols_per_s": float(st[1]),
                "latency_ms_mean": float(st[2]), "latency_ms_max": float(st[3])}

    def close(self):
        if self._h is not None:
            check("rx_destroy", lib().rx_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            if getattr(self, "_h", None) is not None:
                lib().rx_destroy(self._h)
        except Exception:
            pass


class SweepPlan:
    """Batched channel + exact-LLR + GMI sweep over many constellations and noise levels
    (sweep_* in mdemap.h).  instances: list of (X, labels, N, seed) with X float32 [M, D]
    and labels int32 [M] on the GPU (kept alive by the plan); sigma2: [n_inst, n_snr]."""

    def __init__(self, instances, sigma2, variant: int = -1):
        import ctypes
        import numpy as np
        from ._lib import SweepInstance
        self._keep = []
        arr = (SweepInstance * len(instances))()
        for i, (X, labels, N, seed) in enumerate(instances):
            _dev(X, "X", torch.float32, 2)
            _dev(labels, "labels", torch.int32, 1)
            self._keep += [X, labels]
            arr[i] = SweepInstance(X.data_ptr(), labels.data_ptr(), X.shape[0], X.shape[1], int(N),
                                   int(seed) & (2 ** 64 - 1))
        s2 = np.ascontiguousarray(sigma2, dtype=np.float64)
        if s2.shape[0] != len(instances):
            raise ValueError("sigma2 must have one row per instance")
        self.n_inst, self.n_snr = s2.shape
        h = ctypes.c_void_p()
        check("sweep_plan_create", lib().sweep_plan_create(ctypes.cast(arr, ctypes.c_void_p), len(instances),
                                                           s2.ctypes.data, self.n_snr, variant, ctypes.byref(h)))
        self._h = h
        w, sb, gpi, ni = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        check("sweep_plan_info", lib().sweep_plan_info(self._h, ctypes.byref(w), ctypes.byref(sb), ctypes.byref(gpi),
                                                       ctypes.byref(ni)))
        self.shape = (w.value, sb.value, gpi.value)
        self.n_items = ni.value

    def run(self, out=None, use_graph: bool = True):
        """GMI float64 [n_inst, n_snr] (device tensor)."""
        if out is None:
            out = torch.empty((self.n_inst, self.n_snr), dtype=torch.float64, device="cuda")
        check("sweep_run", lib().sweep_run(self._h, _ptr(out), 1 if use_graph else 0, _stream()))
        return out

    def classes(self, with_times: bool = False):
        """[(K steps, label bits, launch shape 0..4, work items)] of the plan's classes, plus
        the autotuner's measured class time in ms (-1 if none) when with_times."""
        import ctypes
        out = []
        while True:
            v = [ctypes.c_int() for _ in range(4)]
            t = ctypes.c_float()
            if lib().sweep_plan_class(self._h, len(out), *[ctypes.byref(x) for x in v], ctypes.byref(t)) != 0:
                return out
            out.append(tuple(x.value for x in v) + ((t.value,) if with_times else ()))

    @staticmethod
    def tuning_clear():
        """Forget the autotuner's cached launch shapes."""
        check("sweep_tuning_clear", lib().sweep_tuning_clear())

    def stats(self):
        """(symbols re-evaluated by the FP64 fallback in the last run, queue overflowed)."""
        import ctypes
        n, ov = ctypes.c_int64(), ctypes.c_int()
        check("sweep_run_stats", lib().sweep_run_stats(self._h, ctypes.byref(n), ctypes.byref(ov), _stream()))
        return n.value, bool(ov.value)

    def close(self):
        if self._h is not None:
            check("sweep_plan_destroy", lib().sweep_plan_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            if getattr(self, "_h", None) is not None:
                lib().sweep_plan_destroy(self._h)
        except Exception:
            pass

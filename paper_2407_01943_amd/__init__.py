"""Python binding of libm2n.so, the MI355X M2NuFFT library (C-ABI in
include/m2n.h).  Argument marshalling only: torch provides device memory and
the current stream, every computation runs in the library's HIP kernels.

The functions keep the C-ABI names:

    gpss_tapers(ctx, t, fmax, fw, K, fc0=0.0)            -> (w [K, N], lam [K])
    m2nufft_eigcoeffs(ctx, t, x, w, f_lo, df, I, prec)   -> J [K, I] complex
    m2nufft_psd(ctx, t, x, w, lam, fmax, fw, f_lo, df, I, prec, ...) -> dict
    m2n_batch_psd(ctx, series, prec, ...)                -> list of dicts

If libm2n.so is missing or cannot be loaded the import fails: there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libm2n.so")

M2N_OK = 0
M2N_ERR_ARG = -1
M2N_ERR_T_ORDER = -2
M2N_ERR_NOT_PD = -3
M2N_ERR_NO_CONVERGE = -4
M2N_ERR_OOM = -5
M2N_ERR_HIP = -6
M2N_ERR_NOT_READY = -7
M2N_ERR_UNSUPPORTED = -8
M2N_ERR_CANCELLED = -9
M2N_FP32 = 1
M2N_FP64 = 2

EXPORTED = ["m2n_create", "m2n_destroy", "m2n_last_error", "m2n_workspace_bytes",
            "gpss_tapers", "m2nufft_eigcoeffs", "m2nufft_psd", "m2n_check", "m2n_stream_status",
            "m2n_profile_enable", "m2n_profile_reset", "m2n_profile_read",
            "m2n_batch_psd", "m2n_queue_create", "m2n_submit", "m2n_poll", "m2n_wait",
            "m2n_queue_destroy", "gpss_tapers_subband", "m2nufft_psd_subband",
            "idpss_tapers", "gpss_tapers_multiband", "m2nufft_psd_at",
            "m2nufft_psd_at_noalloc", "m2n_batch_create", "m2n_batch_launch",
            "m2n_batch_get_info", "m2n_batch_destroy", "m2nufft_psd_freqs", "gpss_tapers_rr"]
M2N_BATCH_GRAPH = 1
M2N_BATCH_TUNE = 2


class M2NSubBand(ctypes.Structure):
    """m2n_subband of include/m2n.h (host array, device output pointers)."""
    _fields_ = [("fmin", ctypes.c_double), ("fmax", ctypes.c_double), ("fc0", ctypes.c_double),
                ("w", ctypes.c_void_p), ("lam", ctypes.c_void_p)]


class M2NSeries(ctypes.Structure):
    """m2n_series of include/m2n.h (device pointers, host array)."""
    _fields_ = [("t", ctypes.c_void_p), ("x", ctypes.c_void_p), ("N", ctypes.c_int64),
                ("K", ctypes.c_int), ("fmax", ctypes.c_double), ("fw", ctypes.c_double),
                ("f_lo", ctypes.c_double), ("df", ctypes.c_double), ("I", ctypes.c_int64),
                ("weights", ctypes.c_void_p), ("w", ctypes.c_void_p),
                ("lam", ctypes.c_void_p), ("P", ctypes.c_void_p), ("E", ctypes.c_void_p),
                ("J", ctypes.c_void_p), ("F", ctypes.c_void_p)]


class M2NBatchInfo(ctypes.Structure):
    """m2n_batch_info of include/m2n.h."""
    _fields_ = [("graph", ctypes.c_int), ("graph_nodes", ctypes.c_int), ("tuned", ctypes.c_int),
                ("from_cache", ctypes.c_int), ("candidates", ctypes.c_int), ("l1", ctypes.c_int),
                ("B", ctypes.c_int), ("M", ctypes.c_int), ("nufft_ms_default", ctypes.c_double),
                ("nufft_ms_tuned", ctypes.c_double), ("series", ctypes.c_int),
                ("band_counts", ctypes.c_int)]


class M2NQueueCfg(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("max_batch", ctypes.c_int),
                ("slots", ctypes.c_int), ("prec", ctypes.c_int), ("nufft_tol", ctypes.c_double),
                ("outputs_pinned", ctypes.c_int), ("inputs_borrowed", ctypes.c_int)]


class M2NRequest(ctypes.Structure):
    _fields_ = [("t", ctypes.c_void_p), ("x", ctypes.c_void_p), ("N", ctypes.c_int64),
                ("K", ctypes.c_int), ("fmax", ctypes.c_double), ("fw", ctypes.c_double),
                ("f_lo", ctypes.c_double), ("df", ctypes.c_double), ("I", ctypes.c_int64),
                ("w", ctypes.c_void_p), ("lam", ctypes.c_void_p), ("P", ctypes.c_void_p),
                ("E", ctypes.c_void_p)]


class M2NResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("batch_size", ctypes.c_int),
                ("latency_us", ctypes.c_double), ("service_us", ctypes.c_double)]


class M2NError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where}: status {code}: {msg}")
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, d, i = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int
    L.m2n_create.argtypes = [i, ctypes.c_size_t, ctypes.POINTER(vp)]
    L.m2n_create.restype = i
    L.m2n_destroy.argtypes = [vp]
    L.m2n_destroy.restype = None
    L.m2n_last_error.argtypes = [vp]
    L.m2n_last_error.restype = ctypes.c_char_p
    L.m2n_workspace_bytes.argtypes = [vp]
    L.m2n_workspace_bytes.restype = ctypes.c_size_t
    L.m2n_profile_enable.argtypes = [vp, i]
    L.m2n_profile_enable.restype = i
    L.m2n_profile_reset.argtypes = [vp]
    L.m2n_profile_reset.restype = i
    L.m2n_profile_read.argtypes = [vp, ctypes.c_char_p, ctypes.c_size_t,
                                   ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_int64), i]
    L.m2n_profile_read.restype = i
    L.m2n_check.argtypes = [vp, vp]
    L.m2n_check.restype = i
    L.m2n_stream_status.argtypes = [vp, vp]
    L.m2n_stream_status.restype = i
    L.gpss_tapers.argtypes = [vp, vp, vp, i64, d, d, d, i, vp, vp]
    L.gpss_tapers.restype = i
    L.m2nufft_eigcoeffs.argtypes = [vp, vp, vp, vp, i64, vp, i, d, d, i64, i, d, vp]
    L.m2nufft_psd_at.restype = i
    L.m2nufft_psd_at.argtypes = [vp, vp, vp, vp, i64, vp, i, vp, i64, vp, vp, vp]
    L.gpss_tapers_rr.restype = i
    L.gpss_tapers_rr.argtypes = [vp, vp, vp, i64, d, d, i, d, vp, vp, ctypes.POINTER(ctypes.c_int64)]
    L.m2nufft_psd_freqs.restype = i
    L.m2nufft_psd_freqs.argtypes = [vp, vp, vp, vp, i64, vp, i, vp, i64, i, d, vp, vp, vp]
    L.m2nufft_psd_at_noalloc.restype = i
    L.m2nufft_psd_at_noalloc.argtypes = [vp, vp, vp, vp, i64, vp, i, vp, i64, vp, vp, vp]
    L.gpss_tapers_multiband.restype = i
    L.gpss_tapers_multiband.argtypes = [vp, vp, vp, i64, d, i, ctypes.POINTER(M2NSubBand), i]
    L.idpss_tapers.restype = i
    L.idpss_tapers.argtypes = [vp, vp, vp, i64, d, d, i, vp, vp]
    L.gpss_tapers_subband.restype = i
    L.gpss_tapers_subband.argtypes = [vp, vp, vp, i64, d, d, d, d, i, vp, vp]
    L.m2nufft_psd_subband.restype = i
    L.m2nufft_psd_subband.argtypes = [vp, vp, vp, vp, i64, vp, i, d, d, i64, i, d, vp, vp, vp]
    L.m2nufft_eigcoeffs.restype = i
    L.m2nufft_psd.argtypes = [vp, vp, vp, vp, i64, vp, vp, i, d, d, d, d, i64, i, d,
                              vp, vp, vp, vp, vp]
    L.m2nufft_psd.restype = i
    L.m2n_batch_psd.argtypes = [vp, vp, ctypes.POINTER(M2NSeries), i, i, d]
    L.m2n_batch_psd.restype = i
    L.m2n_batch_create.argtypes = [vp, vp, ctypes.POINTER(M2NSeries), i, i, d, i, ctypes.POINTER(vp)]
    L.m2n_batch_create.restype = i
    L.m2n_batch_launch.argtypes = [vp, vp]
    L.m2n_batch_launch.restype = i
    L.m2n_batch_get_info.argtypes = [vp, ctypes.POINTER(M2NBatchInfo)]
    L.m2n_batch_get_info.restype = i
    L.m2n_batch_destroy.argtypes = [vp]
    L.m2n_batch_destroy.restype = i
    L.m2n_queue_create.argtypes = [vp, ctypes.POINTER(M2NQueueCfg), ctypes.POINTER(vp)]
    L.m2n_queue_create.restype = i
    L.m2n_submit.argtypes = [vp, ctypes.POINTER(M2NRequest), ctypes.POINTER(ctypes.c_uint64)]
    L.m2n_submit.restype = i
    L.m2n_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(M2NResult)]
    L.m2n_poll.restype = i
    L.m2n_wait.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(M2NResult), i64]
    L.m2n_wait.restype = i
    L.m2n_queue_destroy.argtypes = [vp]
    L.m2n_queue_destroy.restype = i
    return L


lib = _load()


def _err(code, where):
    if code != M2N_OK:
        raise M2NError(code, where, lib.m2n_last_error(None).decode(errors="replace"))


def _ptr(x):
    return None if x is None else ctypes.c_void_p(x.data_ptr())


def _stream(stream):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dev(x, dtype=torch.float64):
    assert x.is_cuda and x.dtype == dtype and x.is_contiguous(), (x.device, x.dtype)
    return x


class Context:
    """Owns one m2n_ctx (plans, caches, workspace) on a HIP device."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        self.device = device
        h = ctypes.c_void_p()
        _err(lib.m2n_create(device, hbm_budget_bytes, ctypes.byref(h)), "m2n_create")
        self.handle = h

    def close(self):
        if self.handle:
            lib.m2n_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_bytes(self) -> int:
        return lib.m2n_workspace_bytes(self.handle)

    def profile(self, on: bool):
        """Bracket every library kernel launch with HIP events (on the launch stream)."""
        _err(lib.m2n_profile_enable(self.handle, 1 if on else 0), "m2n_profile_enable")

    def profile_reset(self):
        _err(lib.m2n_profile_reset(self.handle), "m2n_profile_reset")

    def profile_read(self):
        """{kernel name: (total ms, launches)} since the last reset."""
        cap = 128
        buf = ctypes.create_string_buffer(16384)
        ms = (ctypes.c_double * cap)()
        cnt = (ctypes.c_int64 * cap)()
        n = lib.m2n_profile_read(self.handle, buf, len(buf), ms, cnt, cap)
        if n < 0:
            _err(n, "m2n_profile_read")
        names = buf.value.decode().split("\n")[:n]
        return {nm: (ms[i], int(cnt[i])) for i, nm in enumerate(names)}

    def check(self, stream=None):
        _err(lib.m2n_stream_status(self.handle, _stream(stream)), "m2n_stream_status")


def gpss_tapers(ctx: Context, t, fmax, fw, K, fc0=0.0, stream=None, out=None):
    """Table 3 step 3 (GEP branch): the K largest GPSS tapers at A0."""
    t = _dev(t)
    N = t.shape[0]
    if out is None:
        w = torch.empty((K, N), dtype=torch.float64, device=t.device)
        lam = torch.empty((K,), dtype=torch.float64, device=t.device)
    else:
        w, lam = out
    _err(lib.gpss_tapers(ctx.handle, _stream(stream), _ptr(t), N, float(fmax), float(fw),
                         float(fc0), int(K), _ptr(w), _ptr(lam)), "gpss_tapers")
    return w, lam


def m2nufft_psd_at(ctx: Context, t, x, w, freqs, weights=None, want_J=False, stream=None, check=True):
    """P (and J) at an arbitrary list of band centres, by direct FP64
    summation.  Returns {"P": [I], "J": [K, I] or None}."""
    t, x, w, freqs = _dev(t), _dev(x), _dev(w), _dev(freqs)
    K, N = w.shape
    I = freqs.shape[0]
    P = torch.empty((I,), dtype=torch.float64, device=t.device)
    J = torch.empty((K, I), dtype=torch.complex128, device=t.device) if want_J else None
    if weights is not None:
        weights = _dev(weights)
    _err(lib.m2nufft_psd_at(ctx.handle, _stream(stream), _ptr(t), _ptr(x), N, _ptr(w), K, _ptr(freqs), I,
                            _ptr(weights), _ptr(P), _ptr(J)), "m2nufft_psd_at")
    if check:
        ctx.check(stream)
    return {"P": P, "J": J}


def gpss_tapers_rr(ctx: Context, t, fmax, fw, K, rank_tol=0.0, stream=None):
    """Tapers after the rank-revealing reduction of R(B): (w [K, N], lam [K],
    number of samples kept)."""
    t = _dev(t)
    N = t.shape[0]
    w = torch.empty((K, N), dtype=torch.float64, device=t.device)
    lam = torch.empty((K,), dtype=torch.float64, device=t.device)
    r = ctypes.c_int64(0)
    _err(lib.gpss_tapers_rr(ctx.handle, _stream(stream), _ptr(t), N, float(fmax), float(fw), int(K),
                            float(rank_tol), _ptr(w), _ptr(lam), ctypes.byref(r)), "gpss_tapers_rr")
    return w, lam, int(r.value)


def m2nufft_psd_freqs(ctx: Context, t, x, w, freqs, prec=M2N_FP64, nufft_tol=0.0, weights=None, want_J=False,
                      stream=None, check=True):
    """P (and J) at an arbitrary list of band centres by the type-3 NuFFT.
    Returns {"P": [I], "J": [K, I] or None}."""
    t, x, w, freqs = _dev(t), _dev(x), _dev(w), _dev(freqs)
    K, N = w.shape
    I = freqs.shape[0]
    rdt = torch.float32 if prec == M2N_FP32 else torch.float64
    cdt = torch.complex64 if prec == M2N_FP32 else torch.complex128
    P = torch.empty((I,), dtype=rdt, device=t.device)
    J = torch.empty((K, I), dtype=cdt, device=t.device) if want_J else None
    if weights is not None:
        weights = _dev(weights)
    _err(lib.m2nufft_psd_freqs(ctx.handle, _stream(stream), _ptr(t), _ptr(x), N, _ptr(w), K, _ptr(freqs), I,
                               int(prec), float(nufft_tol), _ptr(weights), _ptr(P), _ptr(J)),
         "m2nufft_psd_freqs")
    if check:
        ctx.check(stream)
    return {"P": P, "J": J}


def m2nufft_psd_at_noalloc(ctx: Context, t, x, w, freqs, P, J=None, weights=None, stream=None):
    """m2nufft_psd_at into caller-allocated outputs P [I] (float64) and J
    [K, I] (complex128 or None); the library allocates nothing (its partial
    sums use a fixed per-device scratch array)."""
    K, N = w.shape
    I = freqs.shape[0]
    _err(lib.m2nufft_psd_at_noalloc(ctx.handle, _stream(stream), _ptr(t), _ptr(x), N, _ptr(w), K,
                                    _ptr(freqs), I, _ptr(weights), _ptr(P), _ptr(J)),
         "m2nufft_psd_at_noalloc")


def idpss_tapers(ctx: Context, t, fmax, fw, K, stream=None, out=None):
    """Interpolated-DPSS tapers (Table 3 step 3 for fc0 = 0): w [K, N] and the
    uniform-grid DPSS concentrations [K]."""
    t = _dev(t)
    N = t.shape[0]
    if out is None:
        w = torch.empty((K, N), dtype=torch.float64, device=t.device)
        lam = torch.empty((K,), dtype=torch.float64, device=t.device)
    else:
        w, lam = out
    _err(lib.idpss_tapers(ctx.handle, _stream(stream), _ptr(t), N, float(fmax), float(fw), int(K),
                          _ptr(w), _ptr(lam)), "idpss_tapers")
    return w, lam


def gpss_tapers_subband(ctx: Context, t, fmin, fmax, fw, fc0, K, stream=None, out=None):
    """One sub-band f_min <= |f| <= f_max, nominal band |f - fc0| <= f_w
    (Sec. 2.4, Sec. 3.2): planar complex tapers [2K, N] (real parts, then
    imaginary parts) and lambda [K].  ``as_complex`` turns w into [K, N]."""
    t = _dev(t)
    N = t.shape[0]
    if out is None:
        w = torch.empty((2 * K, N), dtype=torch.float64, device=t.device)
        lam = torch.empty((K,), dtype=torch.float64, device=t.device)
    else:
        w, lam = out
    _err(lib.gpss_tapers_subband(ctx.handle, _stream(stream), _ptr(t), N, float(fmin), float(fmax),
                                 float(fw), float(fc0), int(K), _ptr(w), _ptr(lam)),
         "gpss_tapers_subband")
    return w, lam


def gpss_tapers_multiband(ctx: Context, t, subbands, fw, K, stream=None):
    """Several sub-bands at once; `subbands` is a list of (fmin, fmax, fc0).
    Returns a list of (planar w [2K, N], lambda [K]), one per sub-band."""
    t = _dev(t)
    N = t.shape[0]
    outs = [(torch.empty((2 * K, N), dtype=torch.float64, device=t.device),
             torch.empty((K,), dtype=torch.float64, device=t.device)) for _ in subbands]
    arr = (M2NSubBand * len(subbands))()
    for a, (fmin, fmax, fc0), (w, lam) in zip(arr, subbands, outs):
        a.fmin, a.fmax, a.fc0 = float(fmin), float(fmax), float(fc0)
        a.w, a.lam = w.data_ptr(), lam.data_ptr()
    _err(lib.gpss_tapers_multiband(ctx.handle, _stream(stream), _ptr(t), N, float(fw), int(K), arr,
                                   len(subbands)), "gpss_tapers_multiband")
    return outs


def as_complex(w):
    """[2K, N] planar tapers -> complex128 [K, N] (a copy)."""
    K = w.shape[0] // 2
    return torch.complex(w[:K], w[K:])


def m2nufft_psd_subband(ctx: Context, t, x, w, f_lo, df, I, prec=M2N_FP64, nufft_tol=0.0,
                        weights=None, want_J=False, stream=None, out=None, check=True):
    """Eigencoefficients and PSD of one sub-band on frequencies f_lo + i df
    relative to its nominal centre.  w is planar [2K, N].  `out` is (P, J).
    Returns {"P": [I], "J": [K, I] or None}."""
    t, x, w = _dev(t), _dev(x), _dev(w)
    K2, N = w.shape
    K = K2 // 2
    rdt = torch.float32 if prec == M2N_FP32 else torch.float64
    cdt = torch.complex64 if prec == M2N_FP32 else torch.complex128
    if out is None:
        P = torch.empty((I,), dtype=rdt, device=t.device)
        J = torch.empty((K, I), dtype=cdt, device=t.device) if want_J else None
    else:
        P, J = out
    if weights is not None:
        weights = _dev(weights)
    _err(lib.m2nufft_psd_subband(ctx.handle, _stream(stream), _ptr(t), _ptr(x), N, _ptr(w), K,
                                 float(f_lo), float(df), int(I), int(prec), float(nufft_tol),
                                 _ptr(weights), _ptr(P), _ptr(J)), "m2nufft_psd_subband")
    if check:
        ctx.check(stream)
    return {"P": P, "J": J}


def m2nufft_eigcoeffs(ctx: Context, t, x, w, f_lo, df, I, prec=M2N_FP64, nufft_tol=0.0,
                      stream=None, out=None, check=True):
    """Table 3 step 4: J_k(A_i) for all bands (complex [K, I])."""
    t, x, w = _dev(t), _dev(x), _dev(w)
    K, N = w.shape
    cdt = torch.complex64 if prec == M2N_FP32 else torch.complex128
    J = torch.empty((K, I), dtype=cdt, device=t.device) if out is None else out
    _err(lib.m2nufft_eigcoeffs(ctx.handle, _stream(stream), _ptr(t), _ptr(x), N, _ptr(w),
                               K, float(f_lo), float(df), int(I), int(prec), float(nufft_tol),
                               _ptr(J)), "m2nufft_eigcoeffs")
    if check:
        ctx.check(stream)
    return J


def m2nufft_psd(ctx: Context, t, x, w, lam, fmax, fw, f_lo, df, I, prec=M2N_FP64,
                nufft_tol=0.0, weights=None, want_E=True, want_J=False, stream=None,
                out=None, check=True, want_F=False):
    """Table 3 steps 4-5 fused, plus the Appendix B suboptimality estimate and,
    with want_F, the Thomson F-statistic (Sec. 3.6).  `out` is (P, E, J) or
    (P, E, J, F).  Returns {"P": [I], "E": [I] or None, "J": [K, I] or None,
    "F": [I] or None}."""
    t, x, w = _dev(t), _dev(x), _dev(w)
    K, N = w.shape
    rdt = torch.float32 if prec == M2N_FP32 else torch.float64
    cdt = torch.complex64 if prec == M2N_FP32 else torch.complex128
    if out is None:
        P = torch.empty((I,), dtype=rdt, device=t.device)
        E = torch.empty((I,), dtype=rdt, device=t.device) if want_E else None
        J = torch.empty((K, I), dtype=cdt, device=t.device) if want_J else None
        F = torch.empty((I,), dtype=rdt, device=t.device) if want_F else None
    else:
        P, E, J = out[:3]
        F = out[3] if len(out) > 3 else None
    if lam is not None:
        lam = _dev(lam)
    if weights is not None:
        weights = _dev(weights)
    _err(lib.m2nufft_psd(ctx.handle, _stream(stream), _ptr(t), _ptr(x), N, _ptr(w),
                         _ptr(lam), K, float(fmax), float(fw), float(f_lo), float(df), int(I),
                         int(prec), float(nufft_tol), _ptr(weights), _ptr(P), _ptr(E), _ptr(J),
                         _ptr(F)),
         "m2nufft_psd")
    if check:
        ctx.check(stream)
    return {"P": P, "E": E, "J": J, "F": F}


def batch_descriptors(series, prec=M2N_FP32, want_E=True, want_J=False, want_F=False):
    """The m2n_series array of a batch and its output tensors, built once so
    that repeated m2n_batch_psd calls on the same tensors skip the per-series
    Python work.  `series` is as for m2n_batch_psd.  Returns (array, outputs)."""
    rdt = torch.float32 if prec == M2N_FP32 else torch.float64
    cdt = torch.complex64 if prec == M2N_FP32 else torch.complex128
    arr = (M2NSeries * len(series))()
    outs = []
    for j, s in enumerate(series):
        t, x = _dev(s["t"]), _dev(s["x"])
        N, K, I = t.shape[0], int(s["K"]), int(s["I"])
        dev = t.device
        w = s.get("w") if s.get("w") is not None else torch.empty((K, N), dtype=torch.float64, device=dev)
        lam = s.get("lam") if s.get("lam") is not None else torch.empty((K,), dtype=torch.float64, device=dev)
        P = s.get("P") if s.get("P") is not None else torch.empty((I,), dtype=rdt, device=dev)
        wE = s.get("want_E", want_E)
        E = s.get("E") if s.get("E") is not None else (torch.empty((I,), dtype=rdt, device=dev) if wE else None)
        J = s.get("J") if s.get("J") is not None else (torch.empty((K, I), dtype=cdt, device=dev) if want_J else None)
        wF = s.get("want_F", want_F)
        F = s.get("F") if s.get("F") is not None else (torch.empty((I,), dtype=rdt, device=dev) if wF else None)
        wt = s.get("weights")
        arr[j] = M2NSeries(t.data_ptr(), x.data_ptr(), N, K, float(s["fmax"]), float(s["fw"]),
                           float(s["f_lo"]), float(s["df"]), I,
                           None if wt is None else _dev(wt).data_ptr(), w.data_ptr(),
                           lam.data_ptr(), P.data_ptr(), None if E is None else E.data_ptr(),
                           None if J is None else J.data_ptr(), None if F is None else F.data_ptr())
        outs.append({"w": w, "lam": lam, "P": P, "E": E, "J": J, "F": F})
    return arr, outs


def m2n_batch_psd(ctx: Context, series, prec=M2N_FP32, nufft_tol=0.0, want_E=True,
                  want_J=False, stream=None, check=True, prepared=None, want_F=False):
    """Tapers and PSD of many series in batched launches.  `series` is a list of
    dicts with device tensors t, x and the numbers fmax, fw, K, f_lo, df, I
    (optional "weights", "want_E", "want_F", and "w", "lam", "P", "E", "J", "F" output
    tensors); `prepared` is the result of batch_descriptors for the same list.
    Returns a list of {"w", "lam", "P", "E", "J"}."""
    arr, outs = prepared if prepared is not None else batch_descriptors(series, prec, want_E, want_J,
                                                                        want_F)
    _err(lib.m2n_batch_psd(ctx.handle, _stream(stream), arr, len(outs), int(prec),
                           float(nufft_tol)), "m2n_batch_psd")
    if check:
        ctx.check(stream)
    return outs


class Batch:
    """m2n_batch: the batched form prepared once (t checked, workspaces sized,
    optionally the NuFFT schedule tuned and the launches captured into a HIP
    graph) and launched many times.  `series` is as for m2n_batch_psd; the
    tensors must outlive the batch.  `outputs` lists the output tensors."""

    def __init__(self, ctx: Context, series, prec=M2N_FP32, nufft_tol=0.0, graph=True, tune=False,
                 want_E=True, want_J=False, want_F=False, stream=None):
        self.ctx = ctx
        self._series = series
        self._arr, self.outputs = batch_descriptors(series, prec, want_E, want_J, want_F)
        flags = (M2N_BATCH_GRAPH if graph else 0) | (M2N_BATCH_TUNE if tune else 0)
        h = ctypes.c_void_p()
        _err(lib.m2n_batch_create(ctx.handle, _stream(stream), self._arr, len(self.outputs), int(prec),
                                  float(nufft_tol), flags, ctypes.byref(h)), "m2n_batch_create")
        self.handle = h

    def launch(self, stream=None):
        _err(lib.m2n_batch_launch(self.handle, _stream(stream)), "m2n_batch_launch")
        return self.outputs

    def info(self):
        inf = M2NBatchInfo()
        _err(lib.m2n_batch_get_info(self.handle, ctypes.byref(inf)), "m2n_batch_get_info")
        return {f[0]: getattr(inf, f[0]) for f in M2NBatchInfo._fields_}

    def close(self):
        if self.handle:
            lib.m2n_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Queue:
    """The served form: m2n_queue with continuous batching.  Inputs are host
    numpy arrays (copied at submit); outputs are host numpy arrays owned by
    this object until the request is collected."""

    def __init__(self, ctx: Context, hbm_budget_bytes=0, max_batch=0, slots=0,
                 prec=M2N_FP32, nufft_tol=0.0, pinned_outputs=False, borrow_inputs=False):
        """borrow_inputs: t and x are not copied at submit; this object keeps
        the arrays it was given alive until the result is collected, and the
        caller must not change them meanwhile."""
        import numpy as np
        self._np = np
        self.ctx = ctx
        self.prec = prec
        self.pinned = bool(pinned_outputs)
        self.borrow = bool(borrow_inputs)
        cfg = M2NQueueCfg(hbm_budget_bytes, max_batch, slots, prec, nufft_tol, 1 if self.pinned else 0,
                          1 if self.borrow else 0)
        h = ctypes.c_void_p()
        _err(lib.m2n_queue_create(ctx.handle, ctypes.byref(cfg), ctypes.byref(h)),
             "m2n_queue_create")
        self.handle = h
        self._out = {}

    def submit(self, t, x, fmax, fw, K, f_lo, df, I, want_E=True, want_w=True, out=None):
        """`out` (optional): the caller's output arrays {"P", "E", "lam", "w"}
        (pinned memory when the queue was made with pinned_outputs), e.g. views
        of a pool the caller reuses; "E" and "w" may be None."""
        np = self._np
        t = np.ascontiguousarray(t, dtype=np.float64)
        x = np.ascontiguousarray(x, dtype=np.float64)
        N = t.shape[0]
        if out is not None:
            out = dict(out)
        elif self.pinned:
            # pinned host tensors (torch's pinned allocator), handed out as numpy views
            rdt = torch.float32 if self.prec == M2N_FP32 else torch.float64

            def buf(shape, dt):
                return torch.empty(shape, dtype=dt, pin_memory=True).numpy()
            out = {"w": buf((K, N), torch.float64) if want_w else None, "lam": buf((K,), torch.float64),
                   "P": buf((I,), rdt), "E": buf((I,), rdt) if want_E else None}
        else:
            rdt = np.float32 if self.prec == M2N_FP32 else np.float64
            out = {"w": np.empty((K, N)) if want_w else None, "lam": np.empty(K),
                   "P": np.empty(I, dtype=rdt), "E": np.empty(I, dtype=rdt) if want_E else None}
        req = M2NRequest(t.ctypes.data, x.ctypes.data, N, int(K), float(fmax), float(fw),
                         float(f_lo), float(df), int(I),
                         None if out["w"] is None else out["w"].ctypes.data,
                         out["lam"].ctypes.data, out["P"].ctypes.data,
                         None if out["E"] is None else out["E"].ctypes.data)
        tk = ctypes.c_uint64()
        _err(lib.m2n_submit(self.handle, ctypes.byref(req), ctypes.byref(tk)), "m2n_submit")
        if self.borrow:
            out["_inputs"] = (t, x)     # alive until the result is collected
        self._out[tk.value] = out
        return tk.value

    def _finish(self, ticket, code, res):
        out = self._out.pop(ticket, None)
        if out is not None:
            out.pop("_inputs", None)
        _err(code, "m2n_wait")
        out.update(status=res.status, batch_size=res.batch_size, latency_us=res.latency_us,
                   service_us=res.service_us)
        return out

    def poll(self, ticket):
        res = M2NResult()
        code = lib.m2n_poll(self.handle, ticket, ctypes.byref(res))
        if code == M2N_ERR_NOT_READY:
            return None
        return self._finish(ticket, code, res)

    def wait(self, ticket, timeout_us=-1):
        res = M2NResult()
        code = lib.m2n_wait(self.handle, ticket, ctypes.byref(res), int(timeout_us))
        if code == M2N_ERR_NOT_READY:
            return None
        return self._finish(ticket, code, res)

    def close(self):
        if self.handle:
            lib.m2n_queue_destroy(self.handle)
            self.handle = None
            self._out.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

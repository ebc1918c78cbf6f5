"""Python binding of libfurax (include/furax.h): argument marshalling only.

Every operation runs in the HIP library; this module converts torch tensors
(device memory) and the current HIP stream into the C structs of the ABI and
turns non-OK statuses into FuraxError.  There is no fallback: if the library
is missing, importing the binding raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libfurax.so")

F32, F64 = 0, 1
OK, EINVAL, ENOMEM, EHIP, EBREAKDOWN, ENOTCONV, EUNSUPPORTED = range(7)
STATUS_NAMES = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EHIP", 4: "EBREAKDOWN", 5: "ENOTCONV",
                6: "EUNSUPPORTED"}
STOP_MAXITER, STOP_RTOL, STOP_BREAKDOWN = 0, 1, 2


class FuraxError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"furax {STATUS_NAMES.get(status, status)}: {message}")
        self.status = status
        self.message = message


class _Pointing(C.Structure):
    _fields_ = [("nside", C.c_int64), ("n_det", C.c_int64), ("n_samp", C.c_int64),
                ("dtype", C.c_int32), ("theta", C.c_void_p), ("phi", C.c_void_p),
                ("psi", C.c_void_p), ("gain", C.c_void_p), ("dpsi", C.c_void_p),
                ("hwp", C.c_int32), ("hwp_num", C.c_int64), ("hwp_den", C.c_int64),
                ("hwp_phase0", C.c_double), ("bore_quat", C.c_void_p), ("det_quat", C.c_void_p)]


class _Noise(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_det", C.c_int64), ("n_samp", C.c_int64),
                ("inv_var", C.c_void_p), ("bandwidth", C.c_int64), ("toeplitz", C.c_void_p),
                ("toeplitz_stride", C.c_int64), ("tmpl_seg_len", C.c_int64),
                ("tmpl_order", C.c_int32)]


class _PcgOpts(C.Structure):
    _fields_ = [("max_iter", C.c_int32), ("rtol", C.c_double), ("precision", C.c_int32),
                ("rcond_min", C.c_double), ("min_hits", C.c_int32), ("valid_in", C.c_void_p),
                ("no_early_exit", C.c_int32)]


class _GapOpts(C.Structure):
    _fields_ = [("max_iter", C.c_int32), ("rtol", C.c_double)]


class _GapInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("rel_resid", C.c_double)]


class _PcgTiming(C.Structure):
    _fields_ = [("iters", C.c_int32), ("ms_apply", C.c_double), ("ms_noise", C.c_double),
                ("ms_transpose", C.c_double), ("ms_update", C.c_double)]


class _PcgInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("stop_reason", C.c_int32), ("rel_resid", C.c_double),
                ("resid_history", C.POINTER(C.c_double)), ("n_valid", C.c_int64)]


def _load() -> C.CDLL:
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"libfurax.so not built at {_LIB_PATH}; run "
                          "`python -m paper_2603_19600_amd.build`")
    lib = C.CDLL(_LIB_PATH)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    P, N = C.POINTER(_Pointing), C.POINTER(_Noise)
    sigs = {
        "furax_ang2pix": [i64, i32, vp, vp, i64, vp, vp],
        "furax_pointing_apply": [P, i32, vp, i32, vp, vp],
        "furax_pointing_transpose": [P, i32, vp, vp, i32, vp],
        "furax_noise_apply": [N, i32, vp, vp, vp],
        "furax_template_fit": [N, i32, vp, vp, vp],
        "furax_gap_fill": [N, i32, vp, vp, vp, vp, C.POINTER(_GapOpts), C.POINTER(_GapInfo), vp],
        "furax_bj_build": [P, N, vp, vp, vp],
        "furax_bj_invert": [i64, vp, vp, dbl, i32, vp, vp, vp, vp],
        "furax_normal_workspace_bytes": [P, N, i32],
        "furax_normal_apply": [P, N, i32, vp, vp, vp, vp, vp],
        "furax_pcg_mapmake": [P, N, i32, vp, vp, vp, C.POINTER(_PcgOpts), C.POINTER(_PcgInfo), vp],
        "furax_pcg_create": [P, N, i32, vp, C.POINTER(_PcgOpts), vp, C.POINTER(vp)],
        "furax_pcg_iterate": [vp, i32],
        "furax_pcg_finish": [vp, vp, vp, C.POINTER(_PcgInfo)],
        "furax_pcg_destroy": [vp],
        "furax_pcg_set_timing": [vp, i32],
        "furax_pcg_read_timing": [vp, C.POINTER(_PcgTiming)],
        "furax_chi2": [P, N, i32, vp, vp, vp, vp, vp],
        "furax_pointing_vjp": [P, i32, vp, vp, vp, vp, vp, vp],
        "furax_chi2_grad": [P, N, i32, vp, vp, vp, vp, vp, vp, vp],
        "furax_chi2_grad_noalloc": [P, N, i32, vp, vp, vp, vp, vp, vp, vp],
        "furax_stream_copy": [vp, vp, i64, i32, vp],
        "furax_last_error": [],
        "furax_release_caches": [],
        "furax_version": [],
    }
    for name, args in sigs.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = i32
    lib.furax_last_error.restype = C.c_char_p
    lib.furax_release_caches.restype = None
    lib.furax_normal_workspace_bytes.restype = i64
    return lib


_lib = _load()

# Every symbol the header declares (checked by the CPU test suite).
EXPORTS = ("furax_ang2pix", "furax_pointing_apply", "furax_pointing_transpose",
           "furax_noise_apply", "furax_template_fit", "furax_gap_fill", "furax_bj_build",
           "furax_bj_invert",
           "furax_normal_workspace_bytes", "furax_normal_apply", "furax_pcg_mapmake",
           "furax_pcg_create", "furax_pcg_iterate", "furax_pcg_finish", "furax_pcg_destroy",
           "furax_pcg_set_timing", "furax_pcg_read_timing",
           "furax_chi2", "furax_pointing_vjp", "furax_chi2_grad", "furax_chi2_grad_noalloc",
           "furax_stream_copy",
           "furax_last_error", "furax_release_caches", "furax_version")


def library() -> C.CDLL:
    return _lib


def _check(status: int):
    if status != OK:
        raise FuraxError(status, _lib.furax_last_error().decode())


def _stream(device=None) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _dt(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.float64:
        return F64
    raise TypeError(f"unsupported dtype {t.dtype}")


def _dt_of(dtype: torch.dtype) -> int:
    if dtype == torch.float32:
        return F32
    if dtype == torch.float64:
        return F64
    raise TypeError(f"unsupported dtype {dtype}")


def _dev(t: torch.Tensor, name: str, dtype=None, shape=None) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


@dataclass
class Pointing:
    """Device pointing of n_det detectors x n_samp samples (see furax_pointing)."""
    nside: int
    theta: torch.Tensor
    phi: torch.Tensor
    psi: torch.Tensor
    gain: Optional[torch.Tensor] = None      # [n_det] float64
    dpsi: Optional[torch.Tensor] = None      # [n_det] float64
    hwp: Optional[tuple] = None              # (hwp_num, hwp_den, phase0)

    def __post_init__(self):
        _dev(self.theta, "theta")
        dt = self.theta.dtype
        _dev(self.phi, "phi", dt, self.theta.shape)
        _dev(self.psi, "psi", dt, self.theta.shape)
        if self.theta.dim() != 2:
            raise ValueError("pointing planes must be [n_det, n_samp]")
        if self.gain is not None:
            _dev(self.gain, "gain", torch.float64, (self.n_det,))
        if self.dpsi is not None:
            _dev(self.dpsi, "dpsi", torch.float64, (self.n_det,))

    @property
    def n_det(self) -> int:
        return self.theta.shape[0]

    @property
    def n_samp(self) -> int:
        return self.theta.shape[1]

    @property
    def npix(self) -> int:
        return 12 * self.nside * self.nside

    @property
    def dtype(self) -> torch.dtype:
        return self.theta.dtype

    @property
    def device(self):
        return self.theta.device

    def c(self) -> _Pointing:
        h = self.hwp
        return _Pointing(self.nside, self.n_det, self.n_samp, _dt(self.theta), _ptr(self.theta),
                         _ptr(self.phi), _ptr(self.psi), _ptr(self.gain), _ptr(self.dpsi),
                         1 if h else 0, int(h[0]) if h else 0, int(h[1]) if h else 1,
                         float(h[2]) if h else 0.0, None, None)

    def with_(self, **kw) -> "Pointing":
        d = dict(nside=self.nside, theta=self.theta, phi=self.phi, psi=self.psi, gain=self.gain,
                 dpsi=self.dpsi, hwp=self.hwp)
        d.update(kw)
        return Pointing(**d)


@dataclass
class QuatPointing:
    """Boresight-quaternion pointing (see furax_pointing): the boresight attitude
    bore_quat [n_samp, 4] and the detector attitudes det_quat [n_det, 4], both
    float64 (w, x, y, z); `dtype` is the TOD / arithmetic precision."""
    nside: int
    bore_quat: torch.Tensor
    det_quat: torch.Tensor
    dtype: torch.dtype = torch.float64
    gain: Optional[torch.Tensor] = None      # [n_det] float64
    dpsi: Optional[torch.Tensor] = None      # [n_det] float64
    hwp: Optional[tuple] = None              # (hwp_num, hwp_den, phase0)

    def __post_init__(self):
        _dev(self.bore_quat, "bore_quat", torch.float64)
        _dev(self.det_quat, "det_quat", torch.float64)
        if self.bore_quat.dim() != 2 or self.bore_quat.shape[1] != 4:
            raise ValueError("bore_quat must be [n_samp, 4]")
        if self.det_quat.dim() != 2 or self.det_quat.shape[1] != 4:
            raise ValueError("det_quat must be [n_det, 4]")
        if self.dtype not in (torch.float32, torch.float64):
            raise ValueError("dtype must be float32 or float64")
        if self.gain is not None:
            _dev(self.gain, "gain", torch.float64, (self.n_det,))
        if self.dpsi is not None:
            _dev(self.dpsi, "dpsi", torch.float64, (self.n_det,))

    @property
    def n_det(self) -> int:
        return self.det_quat.shape[0]

    @property
    def n_samp(self) -> int:
        return self.bore_quat.shape[0]

    @property
    def npix(self) -> int:
        return 12 * self.nside * self.nside

    @property
    def device(self):
        return self.bore_quat.device

    def c(self) -> _Pointing:
        h = self.hwp
        dt = _dt_of(self.dtype)
        return _Pointing(self.nside, self.n_det, self.n_samp, dt, None, None, None,
                         _ptr(self.gain), _ptr(self.dpsi), 1 if h else 0, int(h[0]) if h else 0,
                         int(h[1]) if h else 1, float(h[2]) if h else 0.0,
                         _ptr(self.bore_quat), _ptr(self.det_quat))

    def with_(self, **kw) -> "QuatPointing":
        d = dict(nside=self.nside, bore_quat=self.bore_quat, det_quat=self.det_quat,
                 dtype=self.dtype, gain=self.gain, dpsi=self.dpsi, hwp=self.hwp)
        d.update(kw)
        return QuatPointing(**d)


@dataclass
class Noise:
    """The estimator's weight (see furax_noise): kind "diag" with inv_var [n_det];
    "band" with lags [b] or [n_det, b]; "deproj" (template deprojection F_T of
    Eq. (3)) with inv_var [n_det], seg_len and order of the Legendre baselines."""
    kind: str
    n_det: int
    n_samp: int
    inv_var: Optional[torch.Tensor] = None
    lags: Optional[torch.Tensor] = None
    seg_len: int = 0
    order: int = 0

    def c(self) -> _Noise:
        if self.kind == "diag":
            _dev(self.inv_var, "inv_var", torch.float64, (self.n_det,))
            return _Noise(0, self.n_det, self.n_samp, _ptr(self.inv_var), 0, None, 0, 0, 0)
        if self.kind == "band":
            _dev(self.lags, "lags", torch.float64)
            b = self.lags.shape[-1]
            stride = 0 if self.lags.dim() == 1 else b
            if self.lags.dim() == 2 and self.lags.shape[0] != self.n_det:
                raise ValueError("per-detector lags must be [n_det, b]")
            return _Noise(1, self.n_det, self.n_samp, None, b, _ptr(self.lags), stride, 0, 0)
        if self.kind == "deproj":
            _dev(self.inv_var, "inv_var", torch.float64, (self.n_det,))
            return _Noise(2, self.n_det, self.n_samp, _ptr(self.inv_var), 0, None, 0,
                          int(self.seg_len), int(self.order))
        raise ValueError(f"unknown noise kind {self.kind!r}")


def ang2pix(nside: int, theta: torch.Tensor, phi: torch.Tensor) -> torch.Tensor:
    _dev(theta, "theta")
    _dev(phi, "phi", theta.dtype, theta.shape)
    out = torch.empty(theta.shape, dtype=torch.int64, device=theta.device)
    _check(_lib.furax_ang2pix(nside, _dt(theta), _ptr(theta), _ptr(phi), theta.numel(),
                              _ptr(out), _stream(theta.device)))
    return out


def pointing_apply(P: Pointing, m: torch.Tensor, out: Optional[torch.Tensor] = None):
    _dev(m, "map", shape=(3, P.npix))
    if out is None:
        out = torch.empty(P.n_det, P.n_samp, dtype=P.dtype, device=P.device)
    _dev(out, "tod", P.dtype, (P.n_det, P.n_samp))
    c = P.c()
    _check(_lib.furax_pointing_apply(C.byref(c), _dt(m), _ptr(m), _dt(out), _ptr(out),
                                     _stream(P.device)))
    return out


def pointing_transpose(P: Pointing, tod: torch.Tensor, out: Optional[torch.Tensor] = None,
                       accumulate: bool = False):
    _dev(tod, "tod", P.dtype, (P.n_det, P.n_samp))
    if out is None:
        out = torch.empty(3, P.npix, dtype=torch.float64, device=P.device)
        accumulate = False
    _dev(out, "map", torch.float64, (3, P.npix))
    c = P.c()
    _check(_lib.furax_pointing_transpose(C.byref(c), _dt(tod), _ptr(tod), _ptr(out),
                                         1 if accumulate else 0, _stream(P.device)))
    return out


def noise_apply(N: Noise, tod: torch.Tensor, out: Optional[torch.Tensor] = None):
    _dev(tod, "tod", shape=(N.n_det, N.n_samp))
    if out is None:
        out = torch.empty_like(tod)
    _dev(out, "out", tod.dtype, tod.shape)
    c = N.c()
    _check(_lib.furax_noise_apply(C.byref(c), _dt(tod), _ptr(tod), _ptr(out),
                                  _stream(tod.device)))
    return out


def template_fit(N: Noise, tod: torch.Tensor) -> torch.Tensor:
    """Template amplitudes (T^T W T)^-1 T^T W y of a "deproj" noise model's
    baselines: [n_det, n_seg, order + 1] float64."""
    _dev(tod, "tod", None, (N.n_det, N.n_samp))
    nseg = max(1, N.n_samp // N.seg_len) if N.seg_len > 0 else 1
    amp = torch.empty(N.n_det, nseg, N.order + 1, dtype=torch.float64, device=tod.device)
    c = N.c()
    _check(_lib.furax_template_fit(C.byref(c), _dt(tod), _ptr(tod), _ptr(amp),
                                   _stream(tod.device)))
    return amp


def gap_fill(cov: Noise, gaps: torch.Tensor, tod: torch.Tensor, noise_real: torch.Tensor,
             max_iter: int = 200, rtol: float = 1e-10, out: Optional[torch.Tensor] = None,
             raise_on: Sequence[int] = (EINVAL, ENOMEM, EHIP, EUNSUPPORTED)):
    """Constrained Gaussian realisation of the missing samples (see furax_gap_fill):
    cov describes the noise covariance ("band": autocorrelation lags).  Returns
    (out, iters, rel_resid, status)."""
    _dev(tod, "tod", None, (cov.n_det, cov.n_samp))
    _dev(noise_real, "noise_real", tod.dtype, tod.shape)
    _dev(gaps, "gaps", torch.uint8, tod.shape)
    if out is None:
        out = torch.empty_like(tod)
    _dev(out, "out", tod.dtype, tod.shape)
    c = cov.c()
    opt = _GapOpts(int(max_iter), float(rtol))
    info = _GapInfo(0, 0.0)
    st = _lib.furax_gap_fill(C.byref(c), _dt(tod), _ptr(gaps), _ptr(tod), _ptr(noise_real),
                             _ptr(out), C.byref(opt), C.byref(info), _stream(tod.device))
    if st in raise_on:
        _check(st)
    return out, info.iters, info.rel_resid, st


def bj_build(P: Pointing, N: Noise):
    M6 = torch.empty(6, P.npix, dtype=torch.float64, device=P.device)
    hits = torch.empty(P.npix, dtype=torch.int32, device=P.device)
    cp, cn = P.c(), N.c()
    _check(_lib.furax_bj_build(C.byref(cp), C.byref(cn), _ptr(M6), _ptr(hits),
                               _stream(P.device)))
    return M6, hits


def bj_invert(M6: torch.Tensor, hits: torch.Tensor, rcond_min: float = 1e-3, min_hits: int = 3):
    npix = M6.shape[1]
    _dev(M6, "M6", torch.float64, (6, npix))
    _dev(hits, "hits", torch.int32, (npix,))
    Minv = torch.empty_like(M6)
    valid = torch.empty(npix, dtype=torch.uint8, device=M6.device)
    rcond = torch.empty(npix, dtype=torch.float64, device=M6.device)
    _check(_lib.furax_bj_invert(npix, _ptr(M6), _ptr(hits), rcond_min, min_hits, _ptr(Minv),
                                _ptr(valid), _ptr(rcond), _stream(M6.device)))
    return Minv, valid, rcond


def normal_workspace_bytes(P: Pointing, N: Noise) -> int:
    cp, cn = P.c(), N.c()
    n = _lib.furax_normal_workspace_bytes(C.byref(cp), C.byref(cn), _dt_of(P.dtype))
    if n < 0:
        raise FuraxError(EINVAL, _lib.furax_last_error().decode())
    return n


def normal_apply(P: Pointing, N: Noise, p: torch.Tensor, valid: Optional[torch.Tensor] = None,
                 out: Optional[torch.Tensor] = None, work: Optional[torch.Tensor] = None):
    """q = P^T N^-1 P p in the pointing's precision (FP64 accumulation of q)."""
    _dev(p, "p", torch.float64, (3, P.npix))
    if valid is not None:
        _dev(valid, "valid", torch.uint8, (P.npix,))
    if out is None:
        out = torch.empty_like(p)
    _dev(out, "q", torch.float64, (3, P.npix))
    if work is not None:
        _dev(work, "work", torch.uint8)
        if work.numel() < normal_workspace_bytes(P, N):
            raise ValueError("workspace too small")
    cp, cn = P.c(), N.c()
    _check(_lib.furax_normal_apply(C.byref(cp), C.byref(cn), _dt_of(P.dtype), _ptr(p), _ptr(out),
                                   _ptr(valid), _ptr(work), _stream(P.device)))
    return out


@dataclass
class PcgInfo:
    iters: int
    stop_reason: int
    rel_resid: float
    resid_history: list
    n_valid: int


def _opts(P, max_iter, rtol, rcond_min, min_hits, valid_in, no_early_exit):
    if valid_in is not None:
        _dev(valid_in, "valid_in", torch.uint8, (P.npix,))
    return _PcgOpts(int(max_iter), float(rtol), _dt_of(P.dtype), float(rcond_min), int(min_hits),
                    _ptr(valid_in), 1 if no_early_exit else 0)


def pcg_mapmake(P: Pointing, N: Noise, tod: torch.Tensor, max_iter: int = 50, rtol: float = 0.0,
                rcond_min: float = 1e-3, min_hits: int = 3,
                valid_in: Optional[torch.Tensor] = None, no_early_exit: bool = False,
                raise_on: Sequence[int] = (EINVAL, ENOMEM, EHIP, EUNSUPPORTED)):
    """Block-Jacobi PCG solve of (P^T N^-1 P) m = P^T N^-1 d.

    Returns (map [3, npix] float64, valid [npix] uint8, PcgInfo, status).
    """
    _dev(tod, "tod", P.dtype, (P.n_det, P.n_samp))
    out = torch.empty(3, P.npix, dtype=torch.float64, device=P.device)
    valid = torch.empty(P.npix, dtype=torch.uint8, device=P.device)
    hist = (C.c_double * (max_iter + 1))()
    info = _PcgInfo(0, 0, 0.0, C.cast(hist, C.POINTER(C.c_double)), 0)
    opt = _opts(P, max_iter, rtol, rcond_min, min_hits, valid_in, no_early_exit)
    cp, cn = P.c(), N.c()
    st = _lib.furax_pcg_mapmake(C.byref(cp), C.byref(cn), _dt(tod), _ptr(tod), _ptr(out),
                                _ptr(valid), C.byref(opt), C.byref(info), _stream(P.device))
    if st in raise_on:
        _check(st)
    pinfo = PcgInfo(info.iters, info.stop_reason, info.rel_resid,
                    [hist[i] for i in range(info.iters + 1)], info.n_valid)
    return out, valid, pinfo, st


class PCGSession:
    """Resumable PCG solve (furax_pcg_create / _iterate / _finish / _destroy)."""

    def __init__(self, P: Pointing, N: Noise, tod: torch.Tensor, max_iter: int = 50,
                 rtol: float = 0.0, rcond_min: float = 1e-3, min_hits: int = 3,
                 valid_in: Optional[torch.Tensor] = None, no_early_exit: bool = True):
        _dev(tod, "tod", P.dtype, (P.n_det, P.n_samp))
        self._keep = (P, N, tod, valid_in)       # the C side keeps raw pointers
        self._cp, self._cn = P.c(), N.c()
        self._opt = _opts(P, max_iter, rtol, rcond_min, min_hits, valid_in, no_early_exit)
        self.max_iter = max_iter
        self.P = P
        self._h = C.c_void_p()
        _check(_lib.furax_pcg_create(C.byref(self._cp), C.byref(self._cn), _dt(tod), _ptr(tod),
                                     C.byref(self._opt), _stream(P.device), C.byref(self._h)))

    def iterate(self, n: int):
        _check(_lib.furax_pcg_iterate(self._h, int(n)))

    def set_timing(self, enable: bool = True):
        """Record HIP events between the phases of every following iteration."""
        _check(_lib.furax_pcg_set_timing(self._h, 1 if enable else 0))

    def read_timing(self) -> dict:
        """Device ms of each phase summed over the iterations timed since the last read."""
        t = _PcgTiming()
        _check(_lib.furax_pcg_read_timing(self._h, C.byref(t)))
        return {"iters": t.iters, "apply": t.ms_apply, "noise": t.ms_noise,
                "transpose": t.ms_transpose, "update": t.ms_update}

    def finish(self, raise_on: Sequence[int] = (EINVAL, ENOMEM, EHIP, EUNSUPPORTED)):
        out = torch.empty(3, self.P.npix, dtype=torch.float64, device=self.P.device)
        valid = torch.empty(self.P.npix, dtype=torch.uint8, device=self.P.device)
        hist = (C.c_double * (self.max_iter + 1))()
        info = _PcgInfo(0, 0, 0.0, C.cast(hist, C.POINTER(C.c_double)), 0)
        st = _lib.furax_pcg_finish(self._h, _ptr(out), _ptr(valid), C.byref(info))
        if st in raise_on:
            _check(st)
        return out, valid, PcgInfo(info.iters, info.stop_reason, info.rel_resid,
                                   [hist[i] for i in range(info.iters + 1)], info.n_valid), st

    def close(self):
        if self._h:
            _check(_lib.furax_pcg_destroy(self._h))
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def chi2(P: Pointing, N: Noise, m: torch.Tensor, tod: torch.Tensor, want_resid: bool = False):
    """(chi2 as a 0-d float64 device tensor, u = N^-1 (d - P m) or None)."""
    _dev(m, "map", shape=(3, P.npix))
    _dev(tod, "tod", P.dtype, (P.n_det, P.n_samp))
    out = torch.empty((), dtype=torch.float64, device=P.device)
    u = torch.empty_like(tod) if want_resid else None
    cp, cn = P.c(), N.c()
    _check(_lib.furax_chi2(C.byref(cp), C.byref(cn), _dt(m), _ptr(m), _ptr(tod), _ptr(out),
                           _ptr(u), _stream(P.device)))
    return out, u


def pointing_vjp(P: Pointing, m: Optional[torch.Tensor], cot: torch.Tensor,
                 grad_map: Optional[torch.Tensor] = None, want_map: bool = True,
                 want_gain: bool = True, want_dpsi: bool = True):
    """Transpose of the Jacobian of s = P(m; g, dpsi) applied to a TOD cotangent.

    Returns (grad_map [3, npix] or None, grad_gain [n_det] or None, grad_dpsi [n_det] or None).
    """
    _dev(cot, "cotangent", P.dtype, (P.n_det, P.n_samp))
    if m is not None:
        _dev(m, "map", shape=(3, P.npix))
    if want_map and grad_map is None:
        grad_map = torch.zeros(3, P.npix, dtype=torch.float64, device=P.device)
    gg = torch.empty(P.n_det, dtype=torch.float64, device=P.device) if want_gain else None
    gd = torch.empty(P.n_det, dtype=torch.float64, device=P.device) if want_dpsi else None
    map_dt = _dt(m) if m is not None else F64
    cp = P.c()
    _check(_lib.furax_pointing_vjp(C.byref(cp), map_dt, _ptr(m), _ptr(cot),
                                   _ptr(grad_map) if want_map else None, _ptr(gg), _ptr(gd),
                                   _stream(P.device)))
    return (grad_map if want_map else None), gg, gd


def chi2_grad(P: Pointing, N: Noise, m: torch.Tensor, tod: torch.Tensor, want_map: bool = True,
              want_gain: bool = True, want_dpsi: bool = True, want_chi2: bool = False):
    """Gradient of chi2 = r^T N^-1 r, r = d - P m, by furax_chi2_grad (one pass).

    Returns (grad_map [3, npix] or None, grad_gain [n_det] or None,
    grad_dpsi [n_det] or None, chi2 as a 0-d float64 tensor or None).
    """
    _dev(m, "map", shape=(3, P.npix))
    _dev(tod, "tod", P.dtype, (P.n_det, P.n_samp))
    gm = torch.zeros(3, P.npix, dtype=torch.float64, device=P.device) if want_map else None
    gg = torch.empty(P.n_det, dtype=torch.float64, device=P.device) if want_gain else None
    gd = torch.empty(P.n_det, dtype=torch.float64, device=P.device) if want_dpsi else None
    c2 = torch.empty((), dtype=torch.float64, device=P.device) if want_chi2 else None
    cp, cn = P.c(), N.c()
    _check(_lib.furax_chi2_grad(C.byref(cp), C.byref(cn), _dt(m), _ptr(m), _ptr(tod), _ptr(c2),
                                _ptr(gm), _ptr(gg), _ptr(gd), _stream(P.device)))
    return gm, gg, gd, c2


class Chi2Fn(torch.autograd.Function):
    """chi2(m, g, dpsi) = r^T N^-1 r,  r = d - P(psi + dpsi; g) m  (diagonal N).

    Forward runs furax_chi2 and saves only (m, g, dpsi).  Backward runs
    furax_chi2_grad, which recomputes the pointing and the weighted residual
    u = N^-1 r on the device and applies the hand-written adjoint:
        d chi2 / d m     = -2 P^T u,
        d chi2 / d g_k   = -2 sum_i u[k,i] (P_1 m)[k,i],
        d chi2 / d dpsi_k = -2 sum_i u[k,i] g_k (-2 Q sin 2psi_eff + 2 U cos 2psi_eff);
    the binding only scales them by the incoming gradient.
    Use through chi2_loss(); P's own gain/dpsi are replaced by the arguments.
    """

    @staticmethod
    def forward(ctx, m, gain, dpsi, P, N, d):
        Pg = P.with_(gain=gain.detach().contiguous(), dpsi=dpsi.detach().contiguous())
        val, _ = chi2(Pg, N, m.detach().contiguous(), d)
        ctx.save_for_backward(m, gain, dpsi)
        ctx.P, ctx.N, ctx.d = P, N, d
        return val

    @staticmethod
    def backward(ctx, gout):
        m, gain, dpsi = ctx.saved_tensors
        P = ctx.P.with_(gain=gain.detach().contiguous(), dpsi=dpsi.detach().contiguous())
        m = m.detach().contiguous()
        gm, gg, gd, _ = chi2_grad(P, ctx.N, m, ctx.d, want_map=ctx.needs_input_grad[0],
                                  want_gain=ctx.needs_input_grad[1],
                                  want_dpsi=ctx.needs_input_grad[2])   # pointing recomputed
        return (None if gm is None else (gout * gm).to(m.dtype),
                None if gg is None else gout * gg,
                None if gd is None else gout * gd, None, None, None)


def chi2_loss(P: Pointing, N: Noise, d: torch.Tensor, m: torch.Tensor, gain: torch.Tensor,
              dpsi: torch.Tensor) -> torch.Tensor:
    """Differentiable chi-square of the data d for the map m, detector gains and
    polarisation-angle offsets (0-d float64 device tensor)."""
    if N.kind != "diag":
        raise ValueError("chi2_loss supports diagonal noise")
    return Chi2Fn.apply(m, gain, dpsi, P, N, d)


def stream_copy(src: torch.Tensor, dst: torch.Tensor, nontemporal: bool = False):
    """dst[:] = src[:] by the library's device copy (a measurement utility)."""
    _dev(src, "src")
    _dev(dst, "dst")
    nb = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nb or not src.is_contiguous() or not dst.is_contiguous():
        raise ValueError("stream_copy needs two contiguous buffers of the same size")
    _check(_lib.furax_stream_copy(_ptr(src), _ptr(dst), nb, 1 if nontemporal else 0,
                                  _stream(src.device)))


def release_caches():
    _lib.furax_release_caches()


def version() -> int:
    return _lib.furax_version()

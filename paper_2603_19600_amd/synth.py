"""Seeded synthetic inputs for the map-making hot path.

This module produces INPUTS only: scan pointing (theta, phi, psi), detector
focal-plane offsets, random IQU sky maps, white or 1/f noise streams and the
band-Toeplitz inverse-noise coefficients.  It contains none of the method's
arithmetic (no pixelisation, no pointing matrix, no noise weighting, no
solver), so both the HIP path and the FP64 CPU oracle can consume what it
makes without sharing any of the computation being checked.

The paper names no dataset or benchmark suite; these generators stand in for
the unstated CMB time-ordered-data workloads of its statement of need
(section "Statement of Need": experiments producing massive TOD streams).

Random numbers come from one counter-based generator (the SplitMix64 output
function of Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014) keyed by (config seed, stream, sub-stream) and
indexed by a sample counter.  It is written with 64-bit integer tensor ops,
so it gives the same bits on the CPU and on a GPU, and detector k's data does
not depend on how many detectors are generated: a detector subset is an exact
prefix of the full set.

Scan law: a spin axis precessing around a fixed anti-sun axis (opening 45 deg,
period 90 min) and a boresight spinning around the spin axis (opening 50 deg,
period 1 min), sampled at 50 Hz, with detectors offset from the boresight by
up to +-1 deg in two orthogonal directions.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import Optional

import numpy as np
import torch

_M64 = (1 << 64) - 1
_GOLDEN = 0x9E3779B97F4A7C15
_MIX1 = 0xBF58476D1CE4E5B9
_MIX2 = 0x94D049BB133111EB


def _s64(x: int) -> int:
    """Reinterpret an unsigned 64-bit Python int as a signed int64."""
    x &= _M64
    return x - (1 << 64) if x >= (1 << 63) else x


def _mix64_int(z: int) -> int:
    z &= _M64
    z = ((z ^ (z >> 30)) * _MIX1) & _M64
    z = ((z ^ (z >> 27)) * _MIX2) & _M64
    return z ^ (z >> 31)


def _srl(z: torch.Tensor, s: int) -> torch.Tensor:
    """Logical right shift of an int64 tensor (torch's >> is arithmetic)."""
    return (z >> s) & ((1 << (64 - s)) - 1)


def _mix64(z: torch.Tensor) -> torch.Tensor:
    z = (z ^ _srl(z, 30)) * _s64(_MIX1)
    z = (z ^ _srl(z, 27)) * _s64(_MIX2)
    return z ^ _srl(z, 31)


STREAM_SCAN = 0
STREAM_MAP = 1
SUB_PSI = 0
SUB_OFFSET = 1
SUB_NOISE = 2
SUB_GAIN = 3
SUB_GAPS = 4


def stream_key(seed: int, stream: int, sub: int = 0) -> int:
    """64-bit key of one random stream (unsigned, as a Python int)."""
    k = _mix64_int(seed * _GOLDEN + 0x632BE59BD9B4E019)
    k = _mix64_int(k ^ ((stream + 1) * 0xD1B54A32D192ED03))
    return _mix64_int(k ^ ((sub + 1) * 0x8CB92BA72F3D8DD7))


def uniform(key, counter: torch.Tensor) -> torch.Tensor:
    """U[0,1) doubles: output `counter` of the SplitMix64 sequence started at `key`.

    key is one stream key (a Python int) or an int64 tensor of signed keys that
    broadcasts against counter (several streams at once)."""
    k = key if isinstance(key, torch.Tensor) else _s64(key)
    z = (counter.to(torch.int64) + 1) * _s64(_GOLDEN) + k
    z = _mix64(z)
    return _srl(z, 11).to(torch.float64) * (2.0 ** -53)


def normal(key, counter: torch.Tensor) -> torch.Tensor:
    """N(0,1) doubles by Box-Muller from the uniform pair (2c, 2c+1)."""
    c = counter.to(torch.int64)
    u1 = uniform(key, 2 * c)
    u2 = uniform(key, 2 * c + 1)
    return torch.sqrt(-2.0 * torch.log1p(-u1)) * torch.cos(2.0 * math.pi * u2)


@dataclass(frozen=True)
class Workload:
    """One synthetic map-making workload."""
    name: str
    seed: int
    nside: int
    n_det: int
    n_samp: int
    noise: str                    # "diag" (white), "band" (1/f, band-Toeplitz inverse) or
                                  # "deproj" (white weights with template deprojection)
    bandwidth: int = 1            # number of Toeplitz lags t[0..b-1]
    hwp: bool = False
    dtype: str = "f64"            # canonical pointing / TOD dtype: "f64" or "f32"
    pointing: str = "angles"      # "angles": theta/phi/psi planes; "quat": boresight quaternions
    tmpl_seg_len: int = 4096      # noise "deproj": baseline segments of ~82 s at 50 Hz
    tmpl_order: int = 3           # noise "deproj": Legendre degrees 0..3 per segment
    iters: int = 20
    offsets_deg: float = 1.0      # detector offsets uniform in +-offsets_deg (0: boresight)
    fs: float = 50.0              # sampling rate [Hz]
    spin_period: float = 60.0     # [s]
    prec_period: float = 5400.0   # [s]
    spin_angle_deg: float = 50.0
    prec_angle_deg: float = 45.0
    f_hwp: float = 2.0            # [Hz]
    f_knee: float = 0.1
    alpha: float = -1.0
    sigma: float = 1.0
    psd_len: int = 1 << 20        # frequency grid length used to build the Toeplitz lags

    @property
    def npix(self) -> int:
        return 12 * self.nside * self.nside

    @property
    def n_samples(self) -> int:
        return self.n_det * self.n_samp

    @property
    def hwp_num(self) -> int:
        return int(round(self.f_hwp)) if self.hwp else 0

    @property
    def hwp_den(self) -> int:
        return int(round(self.fs)) if self.hwp else 1

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


# The five workloads the method is exercised on (1: CPU-size FP64; 2: FP64 at
# scale with 1/f noise and a HWP; 3: FP32 variant of 2; 4: differentiation;
# 5: the large single-GPU run).
WORKLOADS = {
    1: Workload("nside64_4x65536_diag_f64", 1001, 64, 4, 65536, "diag", 1, False, "f64",
                iters=20, offsets_deg=0.0),
    2: Workload("nside512_256x2^20_band4096_hwp_f64", 1002, 512, 256, 1 << 20, "band", 4096,
                True, "f64", iters=50),
    3: Workload("nside512_256x2^20_band4096_hwp_f32", 1003, 512, 256, 1 << 20, "band", 4096,
                True, "f32", iters=50),
    4: Workload("nside256_64x2^20_diag_f32_grad", 1004, 256, 64, 1 << 20, "diag", 1, False,
                "f32", iters=0),
    5: Workload("nside1024_1024x2^20_band8192_hwp_f32", 1005, 1024, 1024, 1 << 20, "band", 8192,
                True, "f32", iters=100),
}


def _rot(axis: str, a: torch.Tensor) -> torch.Tensor:
    """Right-handed rotation matrices about a coordinate axis, shape a.shape + (3, 3)."""
    c, s = torch.cos(a), torch.sin(a)
    o, z = torch.ones_like(a), torch.zeros_like(a)
    if axis == "x":
        rows = [[o, z, z], [z, c, -s], [z, s, c]]
    elif axis == "y":
        rows = [[c, z, s], [z, o, z], [-s, z, c]]
    else:
        rows = [[c, -s, z], [s, c, z], [z, z, o]]
    return torch.stack([torch.stack(r, -1) for r in rows], -2)


def detector_offsets(w: Workload, det: torch.Tensor) -> torch.Tensor:
    """Focal-plane offsets (dx_k, dy_k) in radians, shape [len(det), 2]."""
    out = torch.empty(len(det), 2, dtype=torch.float64)
    lim = math.radians(w.offsets_deg)
    for j, k in enumerate(det.tolist()):
        key = stream_key(w.seed, 2 + k, SUB_OFFSET)
        u = uniform(key, torch.arange(2))
        out[j] = (2.0 * u - 1.0) * lim
    return out


def boresight_rotations(w: Workload, i0: int, n: int, device) -> torch.Tensor:
    """Scan rotation R(t_i) for samples i0..i0+n-1, shape [n, 3, 3], float64."""
    key = stream_key(w.seed, STREAM_SCAN, 0)
    ph = uniform(key, torch.arange(2)) * (2.0 * math.pi)
    t = torch.arange(i0, i0 + n, dtype=torch.float64, device=device) / w.fs
    wp = 2.0 * math.pi / w.prec_period
    ws = 2.0 * math.pi / w.spin_period
    r_a = _rot("y", torch.tensor(math.pi / 2, dtype=torch.float64, device=device))
    r_p = _rot("z", wp * t + float(ph[0]))
    r_45 = _rot("y", torch.tensor(math.radians(w.prec_angle_deg), dtype=torch.float64,
                                  device=device))
    r_s = _rot("z", ws * t + float(ph[1]))
    r_50 = _rot("y", torch.tensor(math.radians(w.spin_angle_deg), dtype=torch.float64,
                                  device=device))
    out = _mat3(_mat3(_mat3(_mat3(r_a, r_p), r_45), r_s), r_50)
    return out


def _mat3(a: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    """Batched 3x3 product written out element by element (no BLAS call)."""
    a, b = torch.broadcast_tensors(a, b) if a.dim() == b.dim() else (a, b)
    rows = []
    for i in range(3):
        rows.append(torch.stack([a[..., i, 0] * b[..., 0, j] + a[..., i, 1] * b[..., 1, j]
                                 + a[..., i, 2] * b[..., 2, j] for j in range(3)], -1))
    return torch.stack(rows, -2)


@dataclass
class Pointing:
    """Detector pointing: theta, phi, psi planes [n_det][n_samp] (radians)."""
    theta: torch.Tensor
    phi: torch.Tensor
    psi: torch.Tensor


def pointing(w: Workload, det0: int = 0, n_det: Optional[int] = None, i0: int = 0,
             n_samp: Optional[int] = None, device="cpu", dtype: Optional[str] = None,
             det_chunk: int = 16) -> Pointing:
    """Generate detector pointing for detectors [det0, det0+n_det) and samples [i0, i0+n_samp).

    Directions are computed in float64 and rounded once to the requested dtype
    (the workload's canonical dtype by default).
    """
    n_det = w.n_det - det0 if n_det is None else n_det
    n_samp = w.n_samp - i0 if n_samp is None else n_samp
    dt = {"f64": torch.float64, "f32": torch.float32}[dtype or w.dtype]
    theta = torch.empty(n_det, n_samp, dtype=dt, device=device)
    phi = torch.empty_like(theta)
    psi = torch.empty_like(theta)
    rot = boresight_rotations(w, i0, n_samp, device)
    dets = torch.arange(det0, det0 + n_det)
    offs = detector_offsets(w, dets)
    zhat = torch.tensor([0.0, 0.0, 1.0], dtype=torch.float64)
    counters = torch.arange(i0, i0 + n_samp, dtype=torch.int64, device=device)
    two_pi = 2.0 * math.pi
    for c0 in range(0, n_det, det_chunk):
        c1 = min(n_det, c0 + det_chunk)
        u = torch.stack([_rot("x", offs[j, 1]) @ _rot("y", offs[j, 0]) @ zhat
                         for j in range(c0, c1)]).to(device)            # [d, 3]
        v = torch.stack([rot[None, :, i, 0] * u[:, None, 0] + rot[None, :, i, 1] * u[:, None, 1]
                         + rot[None, :, i, 2] * u[:, None, 2] for i in range(3)], -1)  # [d, t, 3]
        vz = v[..., 2].clamp(-1.0, 1.0)
        theta[c0:c1] = torch.arccos(vz).to(dt)
        ph = torch.atan2(v[..., 1], v[..., 0])
        ph = torch.where(ph < 0, ph + two_pi, ph)
        phi[c0:c1] = ph.to(dt)
        for j in range(c0, c1):
            key = stream_key(w.seed, 2 + det0 + j, SUB_PSI)
            psi[j] = (uniform(key, counters) * two_pi).to(dt)
        del v
    return Pointing(theta, phi, psi)


# ---------------------------------------------------------------------------
# Boresight-quaternion form of the same scan: one attitude per sample for the
# telescope and one fixed attitude per detector.  Quaternions are (w, x, y, z),
# scalar first; the scan's own rotations are composed here only to MAKE the
# boresight attitudes (input generation).
# ---------------------------------------------------------------------------
def _axis_quat(axis: str, a: torch.Tensor) -> torch.Tensor:
    """Unit quaternion of a right-handed rotation by angle a about a coordinate axis."""
    h = 0.5 * a
    q = torch.zeros(a.shape + (4,), dtype=torch.float64, device=a.device)
    q[..., 0] = torch.cos(h)
    q[..., "xyz".index(axis) + 1] = torch.sin(h)
    return q


def _compose(a: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    """Attitude a followed by b in the body frame (quaternion product a b)."""
    aw, ax, ay, az = a.unbind(-1)
    bw, bx, by, bz = b.unbind(-1)
    return torch.stack([aw * bw - ax * bx - ay * by - az * bz,
                        aw * bx + ax * bw + ay * bz - az * by,
                        aw * by - ax * bz + ay * bw + az * bx,
                        aw * bz + ax * by - ay * bx + az * bw], -1)


def boresight_quaternions(w: Workload, i0: int = 0, n: Optional[int] = None,
                          device="cpu") -> torch.Tensor:
    """Boresight attitude of samples i0..i0+n-1, [n, 4] float64: the scan of
    boresight_rotations (R(q) equals that rotation matrix)."""
    n = w.n_samp - i0 if n is None else n
    key = stream_key(w.seed, STREAM_SCAN, 0)
    ph = uniform(key, torch.arange(2)) * (2.0 * math.pi)
    t = torch.arange(i0, i0 + n, dtype=torch.float64, device=device) / w.fs
    wp = 2.0 * math.pi / w.prec_period
    ws = 2.0 * math.pi / w.spin_period
    one = torch.ones((), dtype=torch.float64, device=device)
    q = _axis_quat("y", one * (math.pi / 2))
    q = _compose(q, _axis_quat("z", wp * t + float(ph[0])))
    q = _compose(q, _axis_quat("y", one * math.radians(w.prec_angle_deg)))
    q = _compose(q, _axis_quat("z", ws * t + float(ph[1])))
    q = _compose(q, _axis_quat("y", one * math.radians(w.spin_angle_deg)))
    return q / torch.linalg.vector_norm(q, dim=-1, keepdim=True)


def detector_quaternions(w: Workload, det0: int = 0, n_det: Optional[int] = None,
                         device="cpu") -> torch.Tensor:
    """Detector attitudes relative to the boresight, [n_det, 4] float64: the
    focal-plane offset of detector_offsets (R_x(dy) R_y(dx)) followed by a turn
    of the polarisation direction about the line of sight by (k mod 4) pi/4
    (the usual four orientations of a focal plane)."""
    n_det = w.n_det - det0 if n_det is None else n_det
    dets = torch.arange(det0, det0 + n_det)
    offs = detector_offsets(w, dets)
    chi = (dets % 4).to(torch.float64) * (math.pi / 4)
    q = _compose(_compose(_axis_quat("x", offs[:, 1]), _axis_quat("y", offs[:, 0])),
                 _axis_quat("z", chi))
    q = q / torch.linalg.vector_norm(q, dim=-1, keepdim=True)
    return q.to(device)


def sky_map(w: Workload, device="cpu") -> torch.Tensor:
    """Random IQU map, i.i.d. N(0,1) per pixel and Stokes, shape [3, npix], float64."""
    key = stream_key(w.seed, STREAM_MAP, 0)
    return normal(key, torch.arange(3 * w.npix, device=device)).reshape(3, w.npix)


def psd(w: Workload, f: np.ndarray) -> np.ndarray:
    """Noise power spectrum sigma^2 (1 + (f/f_knee)^alpha)."""
    with np.errstate(divide="ignore"):
        return w.sigma ** 2 * (1.0 + (f / w.f_knee) ** w.alpha)


def toeplitz_lags(w: Workload, b: Optional[int] = None) -> np.ndarray:
    """Inverse-noise autocorrelation lags t[0..b-1] (float64) from the PSD.

    The inverse PSD is sampled on the frequency grid j*fs/L (L = psd_len), its
    zero-frequency value replaced by the first non-zero bin, and transformed
    back to lags with an inverse real FFT; the first b lags are kept.
    """
    b = w.bandwidth if b is None else b
    L = w.psd_len
    f = np.arange(L // 2 + 1) * (w.fs / L)
    p = psd(w, f)
    p[0] = p[1]
    t = np.fft.irfft(1.0 / p, n=L)
    return np.ascontiguousarray(t[:b])


def covariance_lags(w: Workload, b: Optional[int] = None) -> np.ndarray:
    """Noise autocorrelation lags c[0..b-1] (float64) of the PSD, for gap filling.

    The PSD sampled on the frequency grid j*fs/L (L = psd_len, zero frequency
    set to the first non-zero bin) is transformed to lags with an inverse real
    FFT and the first b kept with a triangular taper (1 - tau/b): the taper
    makes the band's symbol the PSD smoothed by a non-negative (Fejer) kernel,
    so the band-Toeplitz covariance stays positive definite."""
    b = w.bandwidth if b is None else b
    L = w.psd_len
    f = np.arange(L // 2 + 1) * (w.fs / L)
    p = psd(w, f)
    p[0] = p[1]
    c = np.fft.irfft(p, n=L)[:b]
    return np.ascontiguousarray(c * (1.0 - np.arange(b) / b))


def gap_mask(w: Workload, det0: int = 0, n_det: Optional[int] = None, frac: float = 0.01,
             mean_len: int = 200) -> np.ndarray:
    """Missing-sample mask [n_det, n_samp] (bool): gaps of random length (1 to
    2 mean_len - 1 samples) at random positions, covering about `frac` of each
    detector's stream, seeded per detector."""
    n_det = w.n_det - det0 if n_det is None else n_det
    out = np.zeros((n_det, w.n_samp), dtype=bool)
    n_gaps = max(1, int(round(frac * w.n_samp / mean_len)))
    for j in range(n_det):
        key = stream_key(w.seed, 2 + det0 + j, SUB_GAPS)
        u = uniform(key, torch.arange(2 * n_gaps)).numpy()
        starts = (u[:n_gaps] * w.n_samp).astype(np.int64)
        lens = 1 + (u[n_gaps:] * (2 * mean_len - 1)).astype(np.int64)
        for s0, ln in zip(starts, lens):
            out[j, s0:s0 + ln] = True
    return out


def white_lags(w: Workload) -> np.ndarray:
    return np.array([1.0 / w.sigma ** 2])


def noise(w: Workload, det0: int = 0, n_det: Optional[int] = None, i0: int = 0,
          n_samp: Optional[int] = None, device="cpu", shape_1f: bool = True) -> torch.Tensor:
    """Noise streams [n_det][n_samp] float64: white sigma, or 1/f shaped in Fourier space.

    shape_1f=False returns the white streams even for a 1/f workload (the
    operators' cost does not depend on the data values)."""
    n_det = w.n_det - det0 if n_det is None else n_det
    n_samp = w.n_samp - i0 if n_samp is None else n_samp
    out = torch.empty(n_det, n_samp, dtype=torch.float64, device=device)
    cnt = torch.arange(i0, i0 + n_samp, dtype=torch.int64, device=device)
    shape = None
    if w.noise == "band" and shape_1f:
        f = np.arange(n_samp // 2 + 1) * (w.fs / n_samp)
        p = psd(w, f)
        p[0] = p[1] if n_samp > 2 else p[0]
        shape = torch.from_numpy(np.sqrt(p) / w.sigma).to(device)
    chunk = 32                                  # detectors drawn per batch of kernels
    for j0 in range(0, n_det, chunk):
        j1 = min(n_det, j0 + chunk)
        keys = torch.tensor([_s64(stream_key(w.seed, 2 + det0 + j, SUB_NOISE))
                             for j in range(j0, j1)], dtype=torch.int64, device=device)
        x = normal(keys[:, None], cnt[None, :]) * w.sigma
        if shape is not None:
            x = torch.fft.irfft(torch.fft.rfft(x, dim=-1) * shape, n=n_samp, dim=-1)
        out[j0:j1] = x
    return out


def gains(w: Workload, det0: int = 0, n_det: Optional[int] = None, scale: float = 0.01):
    """Per-detector gains 1 + scale * N(0,1), float64 [n_det]."""
    n_det = w.n_det - det0 if n_det is None else n_det
    out = torch.empty(n_det, dtype=torch.float64)
    for j in range(n_det):
        key = stream_key(w.seed, 2 + det0 + j, SUB_GAIN)
        out[j] = 1.0 + scale * normal(key, torch.arange(1))[0]
    return out


def angle_offsets(w: Workload, det0: int = 0, n_det: Optional[int] = None,
                  sigma_deg: float = 0.5):
    """Per-detector polarisation-angle offsets N(0, sigma_deg^2) in radians, float64 [n_det]."""
    n_det = w.n_det - det0 if n_det is None else n_det
    out = torch.empty(n_det, dtype=torch.float64)
    for j in range(n_det):
        key = stream_key(w.seed, 2 + det0 + j, SUB_GAIN)
        out[j] = math.radians(sigma_deg) * normal(key, torch.arange(1, 2))[0]
    return out


def uniform_sphere(seed: int, n: int, device="cpu"):
    """n points uniform on the sphere: (theta, phi) float64."""
    key = stream_key(seed, 7, 0)
    c = torch.arange(n, device=device)
    z = 1.0 - 2.0 * uniform(key, 2 * c)
    ph = 2.0 * math.pi * uniform(key, 2 * c + 1)
    return torch.arccos(z.clamp(-1, 1)), ph

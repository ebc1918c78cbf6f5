"""Inverse-noise weighting N^-1, FP64, NumPy (oracle; test infrastructure only).

What is computed (paper, section "Software Design", Table 2 and the
paragraph after it):
  * white noise: HomothetyOperator / DiagonalOperator, N_k^-1 = w_k I;
  * correlated (1/f) noise: SymmetricBandToeplitzOperator, block-diagonal
    over detectors (BlockDiagonalOperator), which the paper applies by
    direct convolution, FFT or overlap-save.

Reading of the open points: a band of b lags t[0..b-1] (half band b-1), and
TRUNCATED linear convolution per detector, i.e. samples outside [0, n_samp)
are zero:
    z[i] = sum_{|tau| <= b-1, 0 <= i+tau < n} t[|tau|] y[i+tau].

Three independent evaluations are given: the direct sum over lags, the dense
Toeplitz matrix (scipy.linalg.toeplitz) and linear convolution by a single
zero-padded real FFT.  The oracle's default is the direct sum for small n and
the FFT for large n; the GPU uses blocked overlap-save, a different algorithm.

Pins: the three evaluations agree; symmetry and positive-definiteness;
b = 1 reduces to the diagonal case; the white-noise limit.
"""
from __future__ import annotations

import numpy as np


def diag_apply(tod, inv_var) -> np.ndarray:
    tod = np.asarray(tod, dtype=np.float64)
    return np.asarray(inv_var, dtype=np.float64)[:, None] * tod


def toeplitz_direct_row(y, t) -> np.ndarray:
    """Direct sum over lags for one detector's stream."""
    y = np.asarray(y, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    n = y.shape[0]
    b = t.shape[0]
    z = t[0] * y
    for tau in range(1, min(b, n)):
        z[:n - tau] += t[tau] * y[tau:]      # partner at i + tau
        z[tau:] += t[tau] * y[:n - tau]      # partner at i - tau
    return z


def toeplitz_dense(n: int, t) -> np.ndarray:
    """Dense symmetric band-Toeplitz matrix n x n from lags t."""
    import scipy.linalg
    col = np.zeros(n)
    b = min(len(t), n)
    col[:b] = t[:b]
    return scipy.linalg.toeplitz(col)


def toeplitz_fft_row(y, t) -> np.ndarray:
    """Linear convolution with the symmetric kernel by one zero-padded real FFT."""
    y = np.asarray(y, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    n = y.shape[0]
    b = t.shape[0]
    kern = np.concatenate([t[::-1], t[1:]])          # taps for tau = -(b-1) .. b-1
    L = 1
    while L < n + 2 * b:
        L *= 2
    full = np.fft.irfft(np.fft.rfft(y, L) * np.fft.rfft(kern, L), L)
    return full[b - 1:b - 1 + n]


def band_apply(tod, t, method: str = "auto") -> np.ndarray:
    """Apply the per-detector band-Toeplitz N^-1 to tod [n_det, n_samp].

    t is [b] (one kernel for all detectors) or [n_det, b].
    """
    tod = np.asarray(tod, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    out = np.empty_like(tod)
    for k in range(tod.shape[0]):
        tk = t if t.ndim == 1 else t[k]
        m = method
        if m == "auto":
            m = "direct" if tod.shape[1] * len(tk) <= 1 << 24 else "fft"
        out[k] = toeplitz_direct_row(tod[k], tk) if m == "direct" else toeplitz_fft_row(tod[k], tk)
    return out


def noise_apply(kind: str, tod, inv_var=None, t=None, method: str = "auto",
                tmpl=None) -> np.ndarray:
    """The weight of the estimator: N^-1 ("diag", "band") or, with templates,
    F_T of Eq. (3) with W = diag(inv_var) ("deproj", tmpl = (seg_len, order))."""
    if kind == "diag":
        return diag_apply(tod, inv_var)
    if kind == "band":
        return band_apply(tod, t, method)
    if kind == "deproj":
        from .templates import deproject_apply
        return deproject_apply(tod, inv_var, tmpl[0], tmpl[1])
    raise ValueError(kind)


def diag_of_inverse(kind: str, n_det: int, inv_var=None, t=None) -> np.ndarray:
    """Per-detector diagonal of the weight without templates (w_k, or t_k[0]
    for the band case); the block-Jacobi preconditioner uses it."""
    if kind in ("diag", "deproj"):
        return np.asarray(inv_var, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    return np.full(n_det, t[0]) if t.ndim == 1 else t[:, 0].copy()


def symbol_min(t, grid: int = 1 << 22) -> float:
    """Minimum over frequency of the kernel's symbol t0 + 2 sum t_tau cos(w tau)."""
    t = np.asarray(t, dtype=np.float64)
    c = np.zeros(grid)
    b = len(t)
    c[:b] = t
    c[grid - b + 1:] = t[1:][::-1]
    return float(np.fft.rfft(c).real.min())

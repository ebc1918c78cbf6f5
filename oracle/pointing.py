"""Pointing operator P and its transpose, FP64, NumPy (oracle; test infrastructure only).

What is computed (paper, section "Software Design"):
  * PointingOperator (Table 3) projects the sky onto time-ordered data and
    rotates it into the instrument frame; IndexOperator (Table 2) is the
    gather of sky pixels into TOD.
  * The acquisition chain of the code listing in that section,
    detector_response @ ... @ hwp @ rotation @ pointing, reduces for one sky
    component and an ideal band to gain * polariser * HWP * rotation * pointing.
  * "Algebraic reductions": consecutive QU rotations add their angles, and an
    ideal HWP obeys R(theta) o HWP = HWP o R(-theta).  Together they collapse
    the chain into ONE effective angle per sample,
        psi_eff[k,i] = psi[k,i] + dpsi[k] + 2 * alpha[i],
    where alpha[i] is the HWP angle.  The ideal linear polariser then reads
        d[k,i] = g[k] * (I[p] + Q[p] cos(2 psi_eff) + U[p] sin(2 psi_eff)),
    with p = ang2pix(theta[k,i], phi[k,i]).

Readings of points the paper leaves open:
  * row (1, cos 2psi_eff, sin 2psi_eff) with no 1/2 polariser factor;
  * the HWP angle is alpha_i = 2 pi ((hwp_num * i) mod hwp_den) / hwp_den
    + phase0, formed from integers so that it stays exact for long scans;
  * a sample whose pixel is -1 (invalid pointing or a flagged sample) reads
    0 in P and contributes nothing to P^T.

Pins: dense brute-force matrix at tiny nside, the adjoint identity
<P m, d> = <m, P^T d>, constant-I map -> constant TOD (bitwise), hits summing
to the unflagged sample count, psi = 0 and psi = pi/4 special cases, the
Mueller-matrix HWP chain, a hand-worked golden example.
"""
from __future__ import annotations

import math

import numpy as np

from .healpix import ang2pix_ring


def hwp_angle(n_samp: int, hwp_num: int, hwp_den: int, phase0: float = 0.0) -> np.ndarray:
    """HWP angle alpha_i for samples i = 0..n_samp-1 (radians, float64)."""
    i = np.arange(n_samp, dtype=np.int64)
    frac = np.mod(hwp_num * i, hwp_den).astype(np.float64) / float(hwp_den)
    return 2.0 * math.pi * frac + phase0


def psi_eff(psi, dpsi=None, hwp=None) -> np.ndarray:
    """Merged polarisation angle psi + dpsi_k + 2 alpha_i, shape [n_det, n_samp].

    hwp is None or a tuple (hwp_num, hwp_den, phase0).
    """
    psi = np.asarray(psi, dtype=np.float64)
    out = psi.copy()
    if dpsi is not None:
        out = out + np.asarray(dpsi, dtype=np.float64)[:, None]
    if hwp is not None:
        num, den, ph0 = hwp
        out = out + 2.0 * hwp_angle(psi.shape[1], num, den, ph0)[None, :]
    return out


def pixels(nside: int, theta, phi) -> np.ndarray:
    return ang2pix_ring(nside, theta, phi)


def weights(psi, dpsi=None, hwp=None) -> tuple[np.ndarray, np.ndarray]:
    """Polariser weights (cos 2 psi_eff, sin 2 psi_eff)."""
    a = 2.0 * psi_eff(psi, dpsi, hwp)
    return np.cos(a), np.sin(a)


def apply_pix(pix, c, s, m, gain=None) -> np.ndarray:
    """y = g_k (I[p] + c Q[p] + s U[p]), 0 where p < 0.  m is [3, npix]."""
    m = np.asarray(m, dtype=np.float64)
    ok = pix >= 0
    p = np.where(ok, pix, 0)
    y = m[0][p] + c * m[1][p] + s * m[2][p]
    if gain is not None:
        y = np.asarray(gain, dtype=np.float64)[:, None] * y
    return np.where(ok, y, 0.0)


def transpose_pix(pix, c, s, tod, npix: int, gain=None) -> np.ndarray:
    """P^T d: per-pixel sums of g_k d (1, c, s); detectors summed in index order."""
    tod = np.asarray(tod, dtype=np.float64)
    out = np.zeros((3, npix), dtype=np.float64)
    for k in range(tod.shape[0]):
        ok = pix[k] >= 0
        p = pix[k][ok]
        g = 1.0 if gain is None else float(gain[k])
        w = g * tod[k][ok]
        out[0] += np.bincount(p, weights=w, minlength=npix)
        out[1] += np.bincount(p, weights=w * c[k][ok], minlength=npix)
        out[2] += np.bincount(p, weights=w * s[k][ok], minlength=npix)
    return out


def hits(pix, npix: int) -> np.ndarray:
    """Number of unflagged samples falling in each pixel (int64)."""
    p = np.asarray(pix).ravel()
    return np.bincount(p[p >= 0], minlength=npix)


def pointing_apply(nside, theta, phi, psi, m, gain=None, dpsi=None, hwp=None) -> np.ndarray:
    """TOD = P m for detectors' pointing (theta, phi, psi) [n_det, n_samp]."""
    pix = pixels(nside, theta, phi)
    c, s = weights(psi, dpsi, hwp)
    return apply_pix(pix, c, s, m, gain)


def pointing_transpose(nside, theta, phi, psi, tod, gain=None, dpsi=None, hwp=None):
    """Map [3, npix] = P^T tod."""
    pix = pixels(nside, theta, phi)
    c, s = weights(psi, dpsi, hwp)
    return transpose_pix(pix, c, s, tod, 12 * nside * nside, gain)


def dense_matrix(pix, c, s, npix: int, gain=None) -> np.ndarray:
    """Dense P (S x 3 npix, Stokes-major columns) built one sample at a time.

    Pure-Python loops; only for tiny inputs.
    """
    nd, ns = pix.shape
    A = np.zeros((nd * ns, 3 * npix))
    for k in range(nd):
        g = 1.0 if gain is None else float(gain[k])
        for i in range(ns):
            p = int(pix[k, i])
            if p < 0:
                continue
            row = k * ns + i
            A[row, p] += g
            A[row, npix + p] += g * float(c[k, i])
            A[row, 2 * npix + p] += g * float(s[k, i])
    return A

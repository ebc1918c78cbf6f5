"""Chi-square of the data model and its analytic gradient, FP64 (oracle; test infrastructure only).

The paper's framework is differentiable (sections "Summary" and "Research
Impact Statement"); the data model is Eq. (1) with T = 0:
    d = H m + n,   H = gain * polariser * HWP * rotation * pointing.
With a per-detector gain g_k and polarisation-angle offset dpsi_k,
    s[k,i] = g_k (I[p] + Q[p] cos 2 psi_eff + U[p] sin 2 psi_eff),
    psi_eff = psi[k,i] + dpsi_k (+ 2 alpha_i with a HWP),
    r = d - s,   chi2 = r^T N^-1 r   (no factor 1/2).
Its gradient, by the chain rule (u = N^-1 r, computed once):
    d chi2 / d m     = -2 P^T (u)              (P with the gains, the adjoint)
    d chi2 / d g_k   = -2 sum_i u[k,i] (P_1 m)[k,i]    (P_1: P with unit gain)
    d chi2 / d dpsi_k = -2 sum_i u[k,i] g_k (-2 Q sin 2psi_eff + 2 U cos 2psi_eff).

Pins: central finite differences (exact up to rounding in m and g because chi2
is quadratic in them; O(h^2) in dpsi) and the dot-product test of the
vector-Jacobian product.
"""
from __future__ import annotations

import math

import numpy as np

from . import noise as _noise
from . import pointing as _pt
from . import quaternion as _quat
from .healpix import zphi2pix_ring


def chi2(nside, theta, phi, psi, d, m, gain, dpsi, noise_kind="diag", inv_var=None,
         lags=None, hwp=None) -> float:
    s = _pt.pointing_apply(nside, theta, phi, psi, m, gain, dpsi, hwp)
    r = np.asarray(d, dtype=np.float64) - s
    u = _noise.noise_apply(noise_kind, r, inv_var, lags)
    return math.fsum((r * u).ravel().tolist())


def chi2_grad(nside, theta, phi, psi, d, m, gain, dpsi, noise_kind="diag", inv_var=None,
              lags=None, hwp=None):
    """(chi2, grad_m [3, npix], grad_gain [n_det], grad_dpsi [n_det])."""
    pix = _pt.pixels(nside, theta, phi)
    c, s = _pt.weights(psi, dpsi, hwp)
    return chi2_grad_geom(nside, pix, c, s, d, m, gain, noise_kind, inv_var, lags)


def chi2_grad_quat(nside, bore_quat, det_quat, d, m, gain, dpsi, noise_kind="diag",
                   inv_var=None, lags=None, hwp=None):
    """chi2_grad with boresight-quaternion pointing (quaternion.expand gives psi)."""
    z, phi, psi = _quat.expand(bore_quat, det_quat)
    pix = zphi2pix_ring(nside, z, phi)
    c, s = _pt.weights(psi, dpsi, hwp)
    return chi2_grad_geom(nside, pix, c, s, d, m, gain, noise_kind, inv_var, lags)


def chi2_grad_geom(nside, pix, c, s, d, m, gain, noise_kind="diag", inv_var=None, lags=None):
    """chi2 and its gradient given each sample's pixel and weights at psi_eff."""
    m = np.asarray(m, dtype=np.float64)
    gain = np.asarray(gain, dtype=np.float64)
    s1 = _pt.apply_pix(pix, c, s, m)                  # unit-gain signal P_1 m
    sig = gain[:, None] * s1
    r = np.asarray(d, dtype=np.float64) - sig
    u = _noise.noise_apply(noise_kind, r, inv_var, lags)
    val = math.fsum((r * u).ravel().tolist())
    g_m = -2.0 * _pt.transpose_pix(pix, c, s, u, 12 * nside * nside, gain)
    g_g = np.array([-2.0 * math.fsum((u[k] * s1[k]).tolist()) for k in range(u.shape[0])])
    ok = pix >= 0
    p = np.where(ok, pix, 0)
    dsig = np.where(ok, -2.0 * m[1][p] * s + 2.0 * m[2][p] * c, 0.0)   # d s1 / d psi_eff
    g_d = np.array([-2.0 * gain[k] * math.fsum((u[k] * dsig[k]).tolist())
                    for k in range(u.shape[0])])
    return val, g_m, g_g, g_d

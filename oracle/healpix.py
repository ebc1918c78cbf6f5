"""HEALPix ring-scheme pixelisation, FP64, NumPy (oracle; test infrastructure only).

The paper discretises the sky with HEALPix (section "Software Design",
"Landscape types" paragraph) and does not restate the pixelisation; the
ring-scheme formulas below are the published ones of Gorski et al. (2005,
ApJ 622, 759), written out as mathematics.

Conventions fixed here (the paper is silent on all of them):
  * ring scheme, any nside >= 1;
  * phi is reduced with fmod(phi, 2 pi), plus 2 pi when negative;
  * tt = phi_reduced / (pi/2) with a true division;
  * the equatorial branch is |z| <= 2/3 with the double constant 2.0/3.0;
  * every floor is of a non-negative value;
  * theta outside [0, pi] or a non-finite angle gives pixel -1 (flagged);
    given z = cos(theta) directly (zphi2pix_ring), z outside [-1, 1] does.
  * no fused multiply-add: every product and sum is rounded on its own
    (NumPy element-wise arithmetic never fuses).

Pins: pixel-centre round trip for every pixel, the nside = 1 closed-form
centres (golden fixture), ring structure, equal area, scan continuity.
"""
from __future__ import annotations

import math

import numpy as np

TWO_PI = 2.0 * math.pi
HALF_PI = 0.5 * math.pi
TWO_THIRDS = 2.0 / 3.0


def npix(nside: int) -> int:
    return 12 * nside * nside


def ang2pix_ring(nside: int, theta, phi) -> np.ndarray:
    """Ring-scheme pixel index of each direction (theta, phi) in radians.

    Returns int64 indices in [0, 12 nside^2), or -1 where the input is
    non-finite or theta is outside [0, pi].
    """
    theta = np.asarray(theta, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    theta, phi = np.broadcast_arrays(theta, phi)
    valid = np.isfinite(theta) & np.isfinite(phi) & (theta >= 0.0) & (theta <= math.pi)
    th = np.where(valid, theta, 0.5)
    return _pix_of_z(nside, np.cos(th), np.where(valid, phi, 0.0), valid)


def zphi2pix_ring(nside: int, z, phi) -> np.ndarray:
    """Ring-scheme pixel of each direction given by z = cos(theta) and phi.

    This is the same pixelisation with the cosine already known (a direction
    vector's third component, as quaternion pointing produces it).  Returns -1
    where the input is non-finite or z is outside [-1, 1].
    """
    z = np.asarray(z, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    z, phi = np.broadcast_arrays(z, phi)
    valid = np.isfinite(z) & np.isfinite(phi) & (z >= -1.0) & (z <= 1.0)
    return _pix_of_z(nside, np.where(valid, z, 0.0), np.where(valid, phi, 0.0), valid)


def _pix_of_z(nside: int, z, ph, valid) -> np.ndarray:
    N = float(nside)
    n = int(nside)
    npx = npix(n)
    ncap = 2 * n * (n - 1)

    za = np.abs(z)
    phr = np.fmod(ph, TWO_PI)
    phr = np.where(phr < 0.0, phr + TWO_PI, phr)
    tt = phr / HALF_PI                                  # in [0, 4]

    out = np.full(z.shape, -1, dtype=np.int64)

    # Equatorial belt: |z| <= 2/3.
    eq = za <= TWO_THIRDS
    t1 = N * (0.5 + tt)
    t2 = (0.75 * N) * z
    jp = np.floor(t1 - t2).astype(np.int64)             # ascending-edge line index
    jm = np.floor(t1 + t2).astype(np.int64)             # descending-edge line index
    ir = n + 1 + jp - jm                                # ring counted from z = 2/3, in [1, 2n+1]
    kshift = 1 - (ir & 1)
    ip = (jp + jm - n + kshift + 1) // 2
    ip = np.mod(ip, 4 * n)
    pix_eq = ncap + (ir - 1) * (4 * n) + ip

    # Polar caps: |z| > 2/3.
    tp = tt - np.floor(tt)
    wpol = N * np.sqrt(3.0 * (1.0 - za))
    jp_c = np.floor(tp * wpol).astype(np.int64)
    jm_c = np.floor((1.0 - tp) * wpol).astype(np.int64)
    ir_c = jp_c + jm_c + 1                              # ring counted from the pole, in [1, n]
    ip_c = np.floor(tt * ir_c).astype(np.int64)
    ip_c = np.mod(ip_c, 4 * ir_c)
    pix_n = 2 * ir_c * (ir_c - 1) + ip_c
    pix_s = npx - 2 * ir_c * (ir_c + 1) + ip_c
    pix_cap = np.where(z > 0.0, pix_n, pix_s)

    pix = np.where(eq, pix_eq, pix_cap)
    pix = np.where((pix >= 0) & (pix < npx), pix, -1)
    out[...] = np.where(valid, pix, -1)
    return out


def _isqrt(a: np.ndarray) -> np.ndarray:
    return np.array([math.isqrt(int(v)) for v in np.ravel(a)], dtype=np.int64).reshape(np.shape(a))


def pix2ang_ring(nside: int, pix) -> tuple[np.ndarray, np.ndarray]:
    """Centre (theta, phi) of each ring-scheme pixel; used by the oracle's own tests."""
    pix = np.asarray(pix, dtype=np.int64)
    n = int(nside)
    N = float(n)
    npx = npix(n)
    ncap = 2 * n * (n - 1)
    z = np.empty(pix.shape, dtype=np.float64)
    phi = np.empty(pix.shape, dtype=np.float64)

    north = pix < ncap
    south = pix >= npx - ncap
    belt = ~(north | south)

    if north.any():
        p = pix[north]
        i = (1 + _isqrt(1 + 2 * p)) // 2
        j = p + 1 - 2 * i * (i - 1)
        z[north] = 1.0 - (i * i) / (3.0 * N * N)
        phi[north] = (j - 0.5) * math.pi / (2.0 * i)
    if belt.any():
        p = pix[belt] - ncap
        i = p // (4 * n) + n
        j = p % (4 * n) + 1
        f = np.where((i + n) % 2 == 1, 1.0, 0.5)
        z[belt] = (2 * n - i) * 2.0 / (3.0 * N)
        phi[belt] = (j - f) * math.pi / (2.0 * N)
    if south.any():
        q = npx - pix[south]
        i = (1 + _isqrt(2 * q - 1)) // 2
        j = 4 * i + 1 - (q - 2 * i * (i - 1))
        z[south] = -1.0 + (i * i) / (3.0 * N * N)
        phi[south] = (j - 0.5) * math.pi / (2.0 * i)
    return np.arccos(np.clip(z, -1.0, 1.0)), phi


def ring_of_pixel(nside: int, pix) -> np.ndarray:
    """Ring number (1 .. 4 nside - 1, from the north pole) of each pixel."""
    th, _ = pix2ang_ring(nside, pix)
    z = np.cos(th)
    n = int(nside)
    # Ring latitudes are distinct and ordered; recover the ring from the exact centre z.
    rings = np.arange(1, 4 * n)
    zr = np.where(rings < n, 1.0 - rings ** 2 / (3.0 * n * n),
                  np.where(rings <= 3 * n, (2 * n - rings) * 2.0 / (3.0 * n),
                           -1.0 + (4 * n - rings) ** 2 / (3.0 * n * n)))
    return rings[np.argmin(np.abs(z[..., None] - zr), axis=-1)]

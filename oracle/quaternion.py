"""Boresight-quaternion pointing expansion, FP64, NumPy (oracle; test infrastructure only).

What is computed (paper, section "Software Design", "Map-making classes"):
PointingOperator projects the sky onto the time-ordered data and rotates it
into the instrument frame, expanding the time-dependent pointing on the fly.
Here the time-dependent pointing is the telescope boresight attitude q_b(t),
one unit quaternion per sample, and each detector k sits at a fixed attitude
q_k relative to the boresight.  A sample's detector attitude is the
composition

    q[k, i] = q_b[i] (x) q_k          (Hamilton product),

its line of sight is d = R(q) z_hat and its polarisation-sensitive direction
is e = R(q) x_hat, where R(q) is the rotation matrix of the unit quaternion q.

Readings of points the paper leaves open (it names no attitude format):
  * quaternions are (w, x, y, z), scalar first, and are taken as given (unit
    norm is the caller's contract, nothing is renormalised);
  * the pixel comes from z = d_z (clipped to [-1, 1]) and phi = atan2(d_y, d_x)
    (healpix.zphi2pix_ring), so no cosine of a colatitude is ever formed;
  * psi is the angle of e in the tangent plane at d, measured from the local
    north (-e_theta) towards the local west (-e_phi), the HEALPix ("COSMO")
    convention:  psi = atan2(-e . e_phi, -e . e_theta), with
    e_theta = (cos th cos ph, cos th sin ph, -sin th), e_phi = (-sin ph, cos ph, 0);
    at the poles both projections vanish and psi = atan2(0, 0) = 0;
  * the merged angle, the HWP term and the polariser row are those of the
    angle-plane pointing (pointing.psi_eff / pointing.weights).

The rotation matrix is written out from the quaternion components with every
product and sum rounded on its own, so that the line of sight (hence the
pixel) is a plain IEEE evaluation of those formulas.

Pins (tests/test_oracle_quaternion.py): the product and the rotation against
scipy.spatial.transform.Rotation, closed forms for attitudes built from axis
rotations (line of sight (sin th cos ph, sin th sin ph, cos th) and
psi = chi modulo pi for q = R_z(ph) R_y(th) R_z(chi)), psi invariance under
q -> -q and under a rotation about the polar axis, psi + chi' under a turn of
the detector about its own line of sight, and orthonormality of d and e.
"""
from __future__ import annotations

import numpy as np

from .healpix import zphi2pix_ring


def quat_mul(a, b) -> np.ndarray:
    """Hamilton product a (x) b of quaternion arrays [..., 4] (w, x, y, z)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    aw, ax, ay, az = a[..., 0], a[..., 1], a[..., 2], a[..., 3]
    bw, bx, by, bz = b[..., 0], b[..., 1], b[..., 2], b[..., 3]
    return np.stack([aw * bw - ax * bx - ay * by - az * bz,
                     aw * bx + ax * bw + ay * bz - az * by,
                     aw * by - ax * bz + ay * bw + az * bx,
                     aw * bz + ax * by - ay * bx + az * bw], axis=-1)


def rotation_matrix(q) -> np.ndarray:
    """R(q) [..., 3, 3] of unit quaternions [..., 4]."""
    q = np.asarray(q, dtype=np.float64)
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    r = np.empty(q.shape[:-1] + (3, 3))
    r[..., 0, 0] = 1.0 - 2.0 * (y * y + z * z)
    r[..., 0, 1] = 2.0 * (x * y - w * z)
    r[..., 0, 2] = 2.0 * (x * z + w * y)
    r[..., 1, 0] = 2.0 * (x * y + w * z)
    r[..., 1, 1] = 1.0 - 2.0 * (x * x + z * z)
    r[..., 1, 2] = 2.0 * (y * z - w * x)
    r[..., 2, 0] = 2.0 * (x * z - w * y)
    r[..., 2, 1] = 2.0 * (y * z + w * x)
    r[..., 2, 2] = 1.0 - 2.0 * (x * x + y * y)
    return r


def detector_attitude(bore_quat, det_quat) -> np.ndarray:
    """q[k, i] = q_b[i] (x) q_k, shape [n_det, n_samp, 4]."""
    qb = np.asarray(bore_quat, dtype=np.float64)
    qd = np.asarray(det_quat, dtype=np.float64)
    return quat_mul(qb[None, :, :], qd[:, None, :])


def line_of_sight(q):
    """(d, e) = (R(q) z_hat, R(q) x_hat), each [..., 3]."""
    r = rotation_matrix(q)
    return r[..., :, 2], r[..., :, 0]


def expand(bore_quat, det_quat):
    """(z, phi, psi) of every sample, each [n_det, n_samp] float64."""
    d, e = line_of_sight(detector_attitude(bore_quat, det_quat))
    z = np.clip(d[..., 2], -1.0, 1.0)
    phi = np.arctan2(d[..., 1], d[..., 0])
    # local basis at d from (theta, phi)
    st = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    cp, sp = np.cos(phi), np.sin(phi)
    e_theta = np.stack([z * cp, z * sp, -st], axis=-1)
    e_phi = np.stack([-sp, cp, np.zeros_like(sp)], axis=-1)
    north = -np.sum(e * e_theta, axis=-1)
    west = -np.sum(e * e_phi, axis=-1)
    psi = np.arctan2(west, north)
    return z, phi, psi


def pixels(nside: int, bore_quat, det_quat) -> np.ndarray:
    """Ring pixel of every sample [n_det, n_samp] (-1 for a non-finite attitude)."""
    d, _ = line_of_sight(detector_attitude(bore_quat, det_quat))
    z = np.clip(d[..., 2], -1.0, 1.0)
    return zphi2pix_ring(nside, z, np.arctan2(d[..., 1], d[..., 0]))

"""Pins of the oracle's boresight-quaternion pointing expansion (CPU only).

The expansion is checked against scipy.spatial.transform.Rotation (an
independent implementation of quaternion composition and rotation), against
closed forms for attitudes built from axis rotations, against hand-worked
attitudes, and through invariances that any correct psi convention obeys."""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import healpix as ohp
from oracle import mapmaker as omm
from oracle import pointing as opt
from oracle import quaternion as oq


def _unit_quats(rng, n):
    q = rng.standard_normal((n, 4))
    return q / np.linalg.norm(q, axis=1, keepdims=True)


def _scipy(q):
    """scipy takes scalar-last quaternions."""
    return Rotation.from_quat(np.concatenate([q[..., 1:], q[..., :1]], axis=-1))


def _axis(axis, a):
    """Quaternion of a right-handed rotation by angle a about a coordinate axis."""
    a = np.asarray(a, dtype=np.float64)
    q = np.zeros(a.shape + (4,))
    q[..., 0] = np.cos(a / 2)
    q[..., "xyz".index(axis) + 1] = np.sin(a / 2)
    return q


def test_product_and_rotation_match_scipy():
    rng = np.random.default_rng(1)
    a, b = _unit_quats(rng, 500), _unit_quats(rng, 500)
    R = oq.rotation_matrix(oq.quat_mul(a, b))
    ref = (_scipy(a) * _scipy(b)).as_matrix()
    assert np.abs(R - ref).max() < 1e-14
    assert np.abs(oq.rotation_matrix(a) - _scipy(a).as_matrix()).max() < 1e-15
    d, e = oq.line_of_sight(a)
    assert np.abs(d - _scipy(a).apply([0.0, 0.0, 1.0])).max() < 1e-15
    assert np.abs(e - _scipy(a).apply([1.0, 0.0, 0.0])).max() < 1e-15


def test_detector_attitude_is_boresight_times_offset():
    rng = np.random.default_rng(2)
    qb, qd = _unit_quats(rng, 37), _unit_quats(rng, 5)
    q = oq.detector_attitude(qb, qd)
    assert q.shape == (5, 37, 4)
    for k in range(5):
        ref = (_scipy(qb) * _scipy(qd[k:k + 1])).as_matrix()
        assert np.abs(oq.rotation_matrix(q[k]) - ref).max() < 1e-14


def test_closed_form_zyz_attitude():
    """q = R_z(ph) R_y(th) R_z(chi): line of sight at (th, ph), psi = chi mod pi."""
    rng = np.random.default_rng(3)
    n = 4000
    th = rng.uniform(0.05, math.pi - 0.05, n)
    ph = rng.uniform(-math.pi, math.pi, n)
    chi = rng.uniform(0, 2 * math.pi, n)
    q = oq.quat_mul(oq.quat_mul(_axis("z", ph), _axis("y", th)), _axis("z", chi))
    z, phi, psi = oq.expand(q, np.array([[1.0, 0.0, 0.0, 0.0]]))
    assert np.abs(z[0] - np.cos(th)).max() < 1e-14
    assert np.abs(np.angle(np.exp(1j * (phi[0] - ph)))).max() < 1e-13
    assert np.abs(np.cos(2 * psi[0]) - np.cos(2 * chi)).max() < 1e-12
    assert np.abs(np.sin(2 * psi[0]) - np.sin(2 * chi)).max() < 1e-12


def test_hand_worked_attitudes_fix_the_psi_convention():
    """Half turn about (x + z)/sqrt 2: line of sight x_hat, polarisation z_hat
    (local north) -> psi = 0.  Then a quarter turn of the detector about its
    line of sight sends the polarisation to -y_hat, which at phi = 0 is the
    local west -> psi = +pi/2 (north through west)."""
    h = math.sqrt(0.5)
    q = np.array([[0.0, h, 0.0, h]])
    z, phi, psi = oq.expand(q, np.array([[1.0, 0.0, 0.0, 0.0]]))
    assert abs(z[0, 0]) < 1e-15 and abs(phi[0, 0]) < 1e-15 and abs(psi[0, 0]) < 1e-15
    d, e = oq.line_of_sight(oq.quat_mul(q, _axis("z", math.pi / 2)))
    assert np.abs(d[0] - [1, 0, 0]).max() < 1e-15 and np.abs(e[0] - [0, -1, 0]).max() < 1e-15
    _, _, psi2 = oq.expand(oq.quat_mul(q, _axis("z", math.pi / 2)),
                           np.array([[1.0, 0.0, 0.0, 0.0]]))
    assert abs(psi2[0, 0] - math.pi / 2) < 1e-15


def test_psi_invariances():
    rng = np.random.default_rng(4)
    qb = _unit_quats(rng, 3000)
    ident = np.array([[1.0, 0.0, 0.0, 0.0]])
    z, phi, psi = oq.expand(qb, ident)
    # q and -q are the same attitude
    _, _, psi_m = oq.expand(-qb, ident)
    assert np.abs(np.angle(np.exp(1j * (psi_m - psi)))).max() < 1e-12
    # a rotation about the polar axis moves phi and keeps psi
    g = 0.7
    z2, phi2, psi2 = oq.expand(oq.quat_mul(_axis("z", g), qb), ident)
    assert np.abs(z2 - z).max() < 1e-14
    assert np.abs(np.angle(np.exp(1j * (phi2 - phi - g)))).max() < 1e-12
    assert np.abs(np.angle(np.exp(1j * (psi2 - psi)))).max() < 1e-11
    # turning the detector about its own line of sight adds to psi
    c = 0.3
    z3, _, psi3 = oq.expand(qb, _axis("z", c)[None, :])
    assert np.abs(z3 - z).max() < 1e-14
    assert np.abs(np.angle(np.exp(2j * (psi3 - psi - c)))).max() < 1e-11


def test_line_of_sight_orthonormal():
    rng = np.random.default_rng(5)
    d, e = oq.line_of_sight(_unit_quats(rng, 10000))
    assert np.abs(np.linalg.norm(d, axis=-1) - 1).max() < 1e-15
    assert np.abs(np.linalg.norm(e, axis=-1) - 1).max() < 1e-15
    assert np.abs(np.sum(d * e, axis=-1)).max() < 1e-15


def test_zphi2pix_is_the_same_pixelisation():
    rng = np.random.default_rng(6)
    for nside in (1, 4, 64, 512):
        th = np.arccos(rng.uniform(-1, 1, 20000))
        ph = rng.uniform(-7, 7, 20000)
        assert np.array_equal(ohp.zphi2pix_ring(nside, np.cos(th), ph),
                              ohp.ang2pix_ring(nside, th, ph))
    assert list(ohp.zphi2pix_ring(8, [1.5, -1.0000001, np.nan, 0.3], [0, 0, 0, np.inf])) == \
        [-1, -1, -1, -1]
    assert ohp.zphi2pix_ring(8, 1.0, 0.0) >= 0 and ohp.zphi2pix_ring(8, -1.0, 0.0) >= 0


def test_quaternion_pixels_match_angles_up_to_boundary_rounding():
    rng = np.random.default_rng(7)
    n = 20000
    th = rng.uniform(0.01, math.pi - 0.01, n)
    ph = rng.uniform(0, 2 * math.pi, n)
    q = oq.quat_mul(_axis("z", ph), _axis("y", th))
    pq = oq.pixels(256, q, np.array([[1.0, 0.0, 0.0, 0.0]]))[0]
    pa = ohp.ang2pix_ring(256, th, ph)
    bad = np.flatnonzero(pq != pa)
    for j in bad:      # only where the direction lies within rounding of a pixel edge
        near = {int(ohp.ang2pix_ring(256, th[j] + a, ph[j] + b))
                for a in (-1e-12, 0, 1e-12) for b in (-1e-12, 0, 1e-12)}
        assert pq[j] in near
    assert len(bad) <= 2


def test_quaternion_problem_geometry():
    rng = np.random.default_rng(8)
    qb = _unit_quats(rng, 300)
    qd = np.stack([_axis("x", 0.01 * k) for k in range(3)])
    prob = omm.Problem(16, None, None, None, "diag", inv_var=np.ones(3), bore_quat=qb,
                       det_quat=qd, hwp=(2, 50, 0.1))
    pix, c, s = prob.geometry()
    z, phi, psi = oq.expand(qb, qd)
    assert np.array_equal(pix, ohp.zphi2pix_ring(16, z, phi))
    c2, s2 = opt.weights(psi, None, (2, 50, 0.1))
    assert np.array_equal(c, c2) and np.array_equal(s, s2)
    assert prob.n_det == 3 and prob.wdiag().shape == (3,)

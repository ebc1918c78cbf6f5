"""Pins of the oracle's pointing operator P and its transpose (CPU only)."""
import math
import os

import numpy as np
import pytest
import torch

from oracle import healpix as hp
from oracle import pointing as pt
from paper_2603_19600_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _tiny(nside=2, n_det=3, n_samp=300, seed=21, hwp=True):
    w = synth.WORKLOADS[2].with_(nside=nside, n_det=n_det, n_samp=n_samp, seed=seed)
    p = synth.pointing(w)
    th, ph, ps = p.theta.numpy(), p.phi.numpy(), p.psi.numpy()
    # spread samples over the whole sphere so that every pixel can be hit
    uth, uph = synth.uniform_sphere(seed, n_det * n_samp)
    th = uth.numpy().reshape(n_det, n_samp)
    ph = uph.numpy().reshape(n_det, n_samp)
    g = synth.gains(w).numpy()
    dp = synth.angle_offsets(w).numpy()
    hw = (2, 50, 0.3) if hwp else None
    return th, ph, ps, g, dp, hw


def test_worked_example_golden():
    rows = []
    with open(os.path.join(GOLD, "pointing_nside1_worked.txt")) as f:
        rows = [list(map(float, ln.split())) for ln in f if ln.strip() and not ln.startswith("#")]
    m = np.stack([np.arange(12.0), 10 + np.arange(12.0), 100 + np.arange(12.0)])
    for th, ph, ps, g, dp, al, epix, etod in rows:
        pix = hp.ang2pix_ring(1, th, ph)
        assert int(pix) == int(epix)
        y = pt.pointing_apply(1, np.array([[th]]), np.array([[ph]]), np.array([[ps]]), m,
                              gain=np.array([g]), dpsi=np.array([dp]), hwp=(0, 1, al))
        assert abs(y[0, 0] - etod) <= 1e-12 * max(1.0, abs(etod))


@pytest.mark.parametrize("nside", [1, 2, 4])
def test_dense_bruteforce(nside):
    th, ph, ps, g, dp, hw = _tiny(nside, 3, 250)
    npix = hp.npix(nside)
    pix = pt.pixels(nside, th, ph)
    pix[0, 5] = -1                                      # one flagged sample
    c, s = pt.weights(ps, dp, hw)
    A = pt.dense_matrix(pix, c, s, npix, g)
    rng = np.random.default_rng(0)
    m = rng.standard_normal((3, npix))
    d = rng.standard_normal(pix.shape)
    y = pt.apply_pix(pix, c, s, m, g)
    assert np.allclose(y.ravel(), A @ m.ravel(), rtol=0, atol=1e-15 * 50)
    mt = pt.transpose_pix(pix, c, s, d, npix, g)
    assert np.allclose(mt.ravel(), A.T @ d.ravel(), rtol=0, atol=1e-13)
    assert y[0, 5] == 0.0


def test_adjoint_identity():
    th, ph, ps, g, dp, hw = _tiny(16, 4, 5000)
    npix = hp.npix(16)
    rng = np.random.default_rng(1)
    m = rng.standard_normal((3, npix))
    d = rng.standard_normal(th.shape)
    lhs = np.sum(pt.pointing_apply(16, th, ph, ps, m, g, dp, hw) * d)
    rhs = np.sum(m * pt.pointing_transpose(16, th, ph, ps, d, g, dp, hw))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_constant_I_gives_constant_tod_bitwise():
    th, ph, ps, _, dp, hw = _tiny(8, 3, 2000)
    npix = hp.npix(8)
    m = np.zeros((3, npix))
    m[0] = 2.718281828459045
    y = pt.pointing_apply(8, th, ph, ps, m, None, dp, hw)
    assert np.all(y == 2.718281828459045)


def test_hits_sum_to_unflagged_count():
    th, ph, ps, *_ = _tiny(8, 3, 3000)
    th[1, 10:20] = np.nan
    pix = pt.pixels(8, th, ph)
    h = pt.hits(pix, hp.npix(8))
    assert h.sum() == th.size - 10
    assert h.dtype.kind == "i"


def test_psi_special_cases():
    npix = hp.npix(4)
    rng = np.random.default_rng(3)
    m = rng.standard_normal((3, npix))
    th, ph, *_ = _tiny(4, 2, 100)
    pix = pt.pixels(4, th, ph)
    y0 = pt.pointing_apply(4, th, ph, np.zeros_like(th), m)
    assert np.allclose(y0, m[0][pix] + m[1][pix], atol=1e-15)
    y45 = pt.pointing_apply(4, th, ph, np.full_like(th, math.pi / 4), m)
    assert np.allclose(y45, m[0][pix] + m[2][pix], atol=1e-15)


def _mueller_rot(a):
    """Rotation of the Stokes (I, Q, U) frame by angle a (linear polarisation rotates by 2a)."""
    c, s = math.cos(2 * a), math.sin(2 * a)
    return np.array([[1, 0, 0], [0, c, s], [0, -s, c]])


def _mueller_hwp(alpha):
    """Ideal half-wave plate with its fast axis at angle alpha: R(-alpha) diag(1, 1, -1) R(alpha)."""
    return _mueller_rot(-alpha) @ np.diag([1.0, 1.0, -1.0]) @ _mueller_rot(alpha)


def test_mueller_chain_hwp_and_rotation_merge():
    """The collapsed row (1, cos 2 psi_eff, sin 2 psi_eff) equals the explicit
    polariser * HWP * rotation Mueller chain, and rotations merge (R(a)R(b) = R(a+b)),
    and the HWP commutes with rotations as R(t) HWP = HWP R(-t)."""
    polariser = np.array([1.0, 1.0, 0.0])
    rng = np.random.default_rng(4)
    for _ in range(50):
        psi, alpha, dpsi = rng.uniform(0, 2 * math.pi, 3)
        chain = polariser @ _mueller_hwp(alpha) @ _mueller_rot(psi + dpsi)
        c, s = pt.weights(np.array([[psi]]), np.array([dpsi]), (0, 1, alpha))
        assert np.allclose(chain, [1.0, c[0, 0], s[0, 0]], atol=1e-13)
        a, b = rng.uniform(-4, 4, 2)
        assert np.allclose(_mueller_rot(a) @ _mueller_rot(b), _mueller_rot(a + b), atol=1e-14)
        assert np.allclose(_mueller_rot(a) @ _mueller_hwp(alpha),
                           _mueller_hwp(alpha) @ _mueller_rot(-a), atol=1e-14)


def test_hwp_angle_is_exact_integer_phase():
    a = pt.hwp_angle(10_000_000, 2, 50)
    assert len(np.unique(a)) == 25
    assert a[25] == a[0] and a[9_999_975] == a[0]
    assert abs(a[1] - 2 * math.pi * 2 / 50) < 1e-15

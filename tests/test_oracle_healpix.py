"""Pins of the oracle's HEALPix ring-scheme pixelisation (CPU only)."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import torch

from oracle import healpix as hp
from paper_2603_19600_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    with open(os.path.join(GOLD, name)) as f:
        return [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]


def test_nside1_centres_golden():
    for pix, z, phi_pi in _rows("healpix_nside1_centres.txt"):
        pix, z, phi = int(pix), float(z), float(phi_pi) * math.pi
        th, ph = hp.pix2ang_ring(1, np.array([pix]))
        assert abs(math.cos(th[0]) - z) < 1e-15
        assert abs(ph[0] - phi) < 1e-15
        assert hp.ang2pix_ring(1, math.acos(z), phi) == pix


def test_nside2_ring_layout_golden():
    n = 2
    allpix = np.arange(hp.npix(n))
    th, ph = hp.pix2ang_ring(n, allpix)
    for ring, first, count, zfrac, phi0 in _rows("healpix_nside2_rings.txt"):
        first, count = int(first), int(count)
        z = float(Fraction(zfrac))
        sel = np.arange(first, first + count)
        assert np.allclose(np.cos(th[sel]), z, atol=1e-15)
        assert abs(ph[first] - float(phi0) * math.pi) < 1e-15
        # equally spaced in phi around the ring
        assert np.allclose(np.diff(ph[sel]), 2 * math.pi / count, atol=1e-14)
        assert np.all(hp.ang2pix_ring(n, th[sel], ph[sel]) == sel)


@pytest.mark.parametrize("nside", [1, 2, 3, 4, 5, 8, 16, 64, 128])
def test_roundtrip_every_pixel(nside):
    pix = np.arange(hp.npix(nside))
    th, ph = hp.pix2ang_ring(nside, pix)
    assert np.array_equal(hp.ang2pix_ring(nside, th, ph), pix)


@pytest.mark.parametrize("nside", [1, 2, 4, 7, 16])
def test_ring_structure(nside):
    n = nside
    pix = np.arange(hp.npix(n))
    ring = hp.ring_of_pixel(n, pix)
    counts = np.bincount(ring)[1:]
    for i, cnt in enumerate(counts, start=1):
        expect = 4 * i if i < n else (4 * n if i <= 3 * n else 4 * (4 * n - i))
        assert cnt == expect
    for i in range(1, n):
        assert pix[ring == i][0] == 2 * i * (i - 1)
    assert 2 * n * (n - 1) == np.sum(counts[: n - 1])


def test_equal_area():
    n = 8
    th, ph = synth.uniform_sphere(11, 400_000)
    pix = hp.ang2pix_ring(n, th.numpy(), ph.numpy())
    counts = np.bincount(pix, minlength=hp.npix(n))
    e = len(pix) / hp.npix(n)
    chi2 = np.sum((counts - e) ** 2 / e) / (hp.npix(n) - 1)
    assert 0.85 < chi2 < 1.15


def test_perturbed_centres_stay_inside():
    for n in (1, 4, 32):
        pix = np.arange(hp.npix(n))
        th, ph = hp.pix2ang_ring(n, pix)
        eps = 1e-3 / n
        for dth, dph in ((eps, 0), (-eps, 0), (0, eps), (0, -eps)):
            t = np.clip(th + dth, 0, math.pi)
            got = hp.ang2pix_ring(n, t, ph + dph / np.maximum(np.sin(th), 1e-3))
            assert np.array_equal(got, pix)


def test_phi_periodicity_and_invalid():
    n = 16
    th, ph = synth.uniform_sphere(5, 10_000)
    th, ph = th.numpy(), ph.numpy()
    a = hp.ang2pix_ring(n, th, ph)
    assert np.array_equal(a, hp.ang2pix_ring(n, th, ph + 2 * math.pi))
    assert np.array_equal(a, hp.ang2pix_ring(n, th, ph - 2 * math.pi))
    bad = hp.ang2pix_ring(n, np.array([-0.1, math.pi + 0.1, np.nan, 0.3, np.inf]),
                          np.array([0.0, 0.0, 0.0, np.nan, 1.0]))
    assert np.all(bad == -1)
    poles = hp.ang2pix_ring(n, np.array([0.0, math.pi]), np.array([0.0, 0.0]))
    assert poles[0] in range(0, 4) and poles[1] in range(hp.npix(n) - 4, hp.npix(n))


def test_scan_continuity():
    w = synth.WORKLOADS[2].with_(nside=256, n_det=2, n_samp=20_000)
    pt = synth.pointing(w)
    pix = hp.ang2pix_ring(w.nside, pt.theta.numpy(), pt.phi.numpy())
    assert np.all(pix >= 0)
    th, ph = hp.pix2ang_ring(w.nside, pix)
    v = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], -1)
    dist = np.arccos(np.clip(np.sum(v[:, 1:] * v[:, :-1], -1), -1, 1))
    pixsize = math.sqrt(4 * math.pi / hp.npix(w.nside))
    # the scan moves ~0.09 deg per sample; consecutive pixel centres are neighbours
    assert dist.max() < 2.5 * pixsize + math.radians(0.1)


def test_pixel_mismatch_check_accepts_only_the_ulp_band():
    """The GPU tests' pixel comparison accepts a disagreement only where a
    one-ulp change of the cosine moves the pixel (resolved with mpmath's
    correctly rounded cosine); a wrong pixel anywhere else fails."""
    from tests.gpu_util import check_pixel_mismatches

    nside = 64
    # directions whose cosine lies within an ulp of an equatorial pixel edge:
    # at phi = 0.3, floor(N (0.5 + tt) - 0.75 N z) steps at z = (N (0.5 + tt) - 40) / (0.75 N)
    ph0 = 0.3
    z_edge = (nside * (0.5 + ph0 / (math.pi / 2)) - 40.0) / (0.75 * nside)
    z = z_edge + np.arange(-200, 201) * np.spacing(z_edge)
    ph = np.full(z.size, ph0)
    th = np.arccos(z)                      # unused when the cosine is given
    ref = hp.zphi2pix_ring(nside, z, ph)
    lo = hp.zphi2pix_ring(nside, np.nextafter(z, -2.0), ph)
    hi = hp.zphi2pix_ring(nside, np.nextafter(z, 2.0), ph)
    flipped = 0
    for i in np.flatnonzero(lo != hi):
        for a in (lo[i], hi[i]):
            if a != ref[i]:
                got = ref.copy()
                got[i] = a
                assert check_pixel_mismatches(nside, th, ph, got, ref, z=z) == 1
                flipped += 1
    # two ulps away from the edge the same substitution is rejected
    i = int(np.flatnonzero(lo != hi)[0])
    far = i - 3 if ref[i - 3] == ref[i] else i + 3
    got = ref.copy()
    got[far] = lo[i] if lo[i] != ref[far] else hi[i]
    with pytest.raises(AssertionError):
        check_pixel_mismatches(nside, th, ph, got, ref, z=z)
    assert flipped >= 1
    # a planted wrong pixel away from every edge is rejected
    rng = np.random.default_rng(5)
    th2 = np.arccos(rng.uniform(-0.5, 0.5, 100))
    ph2 = rng.uniform(0, 2 * math.pi, 100)
    ref2 = hp.ang2pix_ring(nside, th2, ph2)
    bad = ref2.copy()
    bad[17] += 1
    with pytest.raises(AssertionError):
        check_pixel_mismatches(nside, th2, ph2, bad, ref2)
    assert check_pixel_mismatches(nside, th2, ph2, ref2, ref2) == 0

"""Pins of the oracle's chi-square gradient (CPU only)."""
import math

import numpy as np

from oracle import chi2 as oc
from oracle import healpix as hp
from paper_2603_19600_amd import synth


def _setup(kind="diag", seed=6, hwp=None):
    nside, nd, ns = 4, 3, 400
    w = synth.WORKLOADS[4].with_(nside=nside, n_det=nd, n_samp=ns, seed=seed)
    uth, uph = synth.uniform_sphere(seed, nd * ns)
    th = uth.numpy().reshape(nd, ns)
    ph = uph.numpy().reshape(nd, ns)
    ps = synth.pointing(w).psi.numpy().astype(np.float64)
    rng = np.random.default_rng(seed)
    m = rng.standard_normal((3, hp.npix(nside)))
    g = 1 + 0.05 * rng.standard_normal(nd)
    dp = 0.01 * rng.standard_normal(nd)
    d = rng.standard_normal((nd, ns))
    kw = dict(noise_kind=kind, inv_var=np.array([1.0, 0.5, 2.0]),
              lags=np.array([1.2, -0.3, 0.1]), hwp=hwp)
    return nside, th, ph, ps, d, m, g, dp, kw


def _fd(f, x, i, h):
    xp, xm = x.copy(), x.copy()
    xp.flat[i] += h
    xm.flat[i] -= h
    return (f(xp) - f(xm)) / (2 * h)


def test_gradient_matches_central_differences():
    for kind, hwp in (("diag", None), ("band", (2, 50, 0.0))):
        nside, th, ph, ps, d, m, g, dp, kw = _setup(kind, hwp=hwp)
        kw["noise_kind"] = kind
        val, gm, gg, gd = oc.chi2_grad(nside, th, ph, ps, d, m, g, dp, **kw)
        assert abs(val - oc.chi2(nside, th, ph, ps, d, m, g, dp, **kw)) < 1e-12 * abs(val)
        h = 1e-4
        for i in np.flatnonzero(np.abs(gm).ravel() > 0)[:6]:
            fd = _fd(lambda x: oc.chi2(nside, th, ph, ps, d, x, g, dp, **kw), m, i, h)
            assert abs(fd - gm.flat[i]) <= 1e-7 * max(1.0, abs(gm.flat[i]))
        for k in range(3):
            fd = _fd(lambda x: oc.chi2(nside, th, ph, ps, d, m, x, dp, **kw), g, k, h)
            assert abs(fd - gg[k]) <= 1e-7 * max(1.0, abs(gg[k]))
            fd = _fd(lambda x: oc.chi2(nside, th, ph, ps, d, m, g, x, **kw), dp, k, h)
            assert abs(fd - gd[k]) <= 1e-6 * max(1.0, abs(gd[k]))


def test_vjp_dot_product_identity():
    """<J v, u> = <v, J^T u> for the linear map m -> P m (gain included)."""
    from oracle import pointing as pt
    nside, th, ph, ps, d, m, g, dp, kw = _setup()
    rng = np.random.default_rng(9)
    u = rng.standard_normal(th.shape)
    v = rng.standard_normal(m.shape)
    Jv = pt.pointing_apply(nside, th, ph, ps, v, g, dp)
    JTu = pt.pointing_transpose(nside, th, ph, ps, u, g, dp)
    assert abs(np.sum(Jv * u) - np.sum(v * JTu)) < 1e-12 * abs(np.sum(Jv * u))

"""Pins of the oracle's block-Jacobi PCG map-maker (CPU only)."""
import math

import numpy as np
import pytest

from oracle import healpix as hp
from oracle import mapmaker as mm
from oracle import noise as nz
from oracle import pointing as pt
from paper_2603_19600_amd import synth


def _problem(nside=2, n_det=3, n_samp=400, kind="diag", b=8, seed=3, hwp=True, gain=True):
    w = synth.WORKLOADS[2].with_(nside=nside, n_det=n_det, n_samp=n_samp, seed=seed)
    p = synth.pointing(w)
    uth, uph = synth.uniform_sphere(seed, n_det * n_samp)
    th = uth.numpy().reshape(n_det, n_samp)
    ph = uph.numpy().reshape(n_det, n_samp)
    kw = {}
    if kind == "diag":
        kw["inv_var"] = np.linspace(0.5, 2.0, n_det)
    else:
        kw["lags"] = synth.toeplitz_lags(w.with_(f_knee=2.0), b)
    return mm.Problem(nside, th, ph, p.psi.numpy(), kind,
                      gain=synth.gains(w, scale=0.1).numpy() if gain else None,
                      dpsi=synth.angle_offsets(w).numpy(),
                      hwp=(2, 50, 0.1) if hwp else None, **kw)


def test_bj_inverse_and_rcond_vs_numpy():
    rng = np.random.default_rng(0)
    X = rng.standard_normal((200, 5, 3))
    Ms = np.einsum("nki,nkj->nij", X, X)
    Ms[0] = np.diag([1.0, 1e-9, 1.0])          # nearly singular
    M6 = np.stack([Ms[:, 0, 0], Ms[:, 0, 1], Ms[:, 0, 2], Ms[:, 1, 1], Ms[:, 1, 2], Ms[:, 2, 2]])
    hits = np.full(200, 5)
    inv, valid, rcond = mm.bj_invert(M6, hits, 1e-3, 3)
    ref = np.linalg.inv(Ms)
    assert np.allclose(mm.sym3(inv)[1:], ref[1:], rtol=1e-10, atol=1e-12)
    assert np.allclose(rcond, 1.0 / np.linalg.cond(Ms, 1), rtol=1e-9)
    assert not valid[0] and valid[1:].all()
    _, v2, _ = mm.bj_invert(M6, np.full(200, 2), 1e-3, 3)
    assert not v2.any()


def test_bj_invert_closed_forms():
    """A block inverted by hand and diagonal blocks.

    M = [[4,1,0],[1,3,1],[0,1,2]]: det 18, adjugate [[5,-2,1],[-2,8,-4],[1,-4,11]],
    so M^-1 = adj/18, ||M||_1 = 5, ||M^-1||_1 = 16/18 and rcond = 18/80.
    diag(a, b, c): M^-1 = diag(1/a, 1/b, 1/c), rcond = min/max of (a, b, c).
    A zero block (unobserved pixel) has rcond 0 and inverse 0."""
    M6 = np.array([[4.0, 2.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 0.0], [3.0, 5.0, 0.0],
                   [1.0, 0.0, 0.0], [2.0, 0.5, 0.0]])
    inv, valid, rcond = mm.bj_invert(M6, np.array([5, 5, 5]), 1e-3, 3)
    np.testing.assert_allclose(inv[:, 0], np.array([5, -2, 1, 8, -4, 11]) / 18.0, rtol=1e-14)
    np.testing.assert_allclose(rcond[0], 18.0 / 80.0, rtol=1e-14)
    np.testing.assert_allclose(inv[:, 1], [0.5, 0, 0, 0.2, 0, 2.0], rtol=1e-15)
    np.testing.assert_allclose(rcond[1], 0.5 / 5.0, rtol=1e-15)
    assert valid[0] and valid[1] and not valid[2]
    assert rcond[2] == 0.0 and np.all(inv[:, 2] == 0.0)


def test_bj_rank_deficient_blocks_are_invalid():
    """Blocks singular in exact arithmetic -- every sample at one polariser angle
    (rank 1), or at two angles pi/2 apart (rank 2) -- must come out invalid with
    a tiny rcond, as numpy's condition number of the same matrices says."""
    rng = np.random.default_rng(3)
    blocks = []
    for _ in range(300):
        n = int(rng.integers(3, 9))
        ang = np.full(n, rng.uniform(0, 2 * np.pi))               # one angle: rank 1
        if rng.random() < 0.5:                                    # two angles pi/2 apart
            ang = ang + (np.pi / 2) * rng.integers(0, 2, n)
        w = rng.uniform(0.5, 2.0, n)
        v = np.stack([np.ones(n), np.cos(2 * ang), np.sin(2 * ang)], 1)
        blocks.append(np.einsum("k,ki,kj->ij", w, v, v))
    Ms = np.array(blocks)
    M6 = np.stack([Ms[:, 0, 0], Ms[:, 0, 1], Ms[:, 0, 2], Ms[:, 1, 1], Ms[:, 1, 2], Ms[:, 2, 2]])
    inv, valid, rcond = mm.bj_invert(M6, np.full(len(Ms), 8), 1e-3, 3)
    assert not valid.any()
    assert (rcond < 1e-10).all()
    assert (1.0 / np.linalg.cond(Ms, 1) < 1e-10).all()
    assert (inv == 0).all()


def test_bj_well_conditioned_psd_blocks_match_numpy():
    """Blocks made the way the method makes them (sums of w (1,c,s)^T (1,c,s))."""
    rng = np.random.default_rng(4)
    n = 400
    k = rng.integers(3, 12, n)
    Ms = np.zeros((n, 3, 3))
    for j in range(n):
        ang = rng.uniform(0, 2 * np.pi, k[j])
        v = np.stack([np.ones(k[j]), np.cos(2 * ang), np.sin(2 * ang)], 1)
        Ms[j] = np.einsum("k,ki,kj->ij", rng.uniform(0.5, 2, k[j]), v, v)
    M6 = np.stack([Ms[:, 0, 0], Ms[:, 0, 1], Ms[:, 0, 2], Ms[:, 1, 1], Ms[:, 1, 2], Ms[:, 2, 2]])
    inv, valid, rcond = mm.bj_invert(M6, k, 0.0, 3)
    ref_rc = 1.0 / np.linalg.cond(Ms, 1)
    good = ref_rc > 1e-6
    assert good.sum() > 300
    assert np.allclose(rcond[good], ref_rc[good], rtol=1e-8)
    assert np.allclose(mm.sym3(inv)[good], np.linalg.inv(Ms[good]), rtol=1e-8, atol=1e-10)


def test_diag_noise_converges_in_one_iteration_to_binned_map():
    prob = _problem(nside=4, n_det=4, n_samp=600, kind="diag")
    rng = np.random.default_rng(1)
    d = rng.standard_normal(prob.theta.shape)
    res = mm.pcg_mapmake(prob, d, max_iter=5, keep_iterates=True)
    # binned map by an independent per-pixel dense solve
    pix, c, s = prob.geometry()
    pixv = mm.flag_invalid(pix, res.valid)
    x_ref = np.zeros((3, prob.npix))
    A = pt.dense_matrix(pixv, c, s, prob.npix, prob.gain)
    W = np.repeat(prob.inv_var, prob.theta.shape[1])
    rhs = A.T @ (W * d.ravel())
    for q in np.flatnonzero(res.valid):
        idx = [q, prob.npix + q, 2 * prob.npix + q]
        Mq = (A[:, idx].T * W) @ A[:, idx]
        x_ref[:, q] = np.linalg.solve(Mq, rhs[idx])
    x1 = res.iterates[0]
    assert np.max(np.abs(x1 - x_ref)) <= 1e-10 * np.max(np.abs(x_ref))
    assert res.resid_history[1] < 1e-12
    binned, _ = mm.binned_map(prob, d)
    assert np.allclose(binned, x_ref, atol=1e-10 * np.max(np.abs(x_ref)))


def test_band_noise_equals_dense_solve():
    prob = _problem(nside=2, n_det=2, n_samp=500, kind="band", b=40)
    rng = np.random.default_rng(2)
    d = rng.standard_normal(prob.theta.shape)
    res = mm.pcg_mapmake(prob, d, max_iter=200, rtol=1e-14)
    assert res.stop_reason in (mm.STOP_RTOL, mm.STOP_MAXITER)
    pix, c, s = prob.geometry()
    pixv = mm.flag_invalid(pix, res.valid)
    A = pt.dense_matrix(pixv, c, s, prob.npix, prob.gain)
    nd, ns = prob.theta.shape
    Ninv = np.zeros((nd * ns, nd * ns))
    for k in range(nd):
        Ninv[k * ns:(k + 1) * ns, k * ns:(k + 1) * ns] = nz.toeplitz_dense(ns, prob.lags)
    keep = np.concatenate([res.valid] * 3)
    Av = A[:, keep]
    x = np.linalg.solve(Av.T @ Ninv @ Av, Av.T @ Ninv @ d.ravel())
    got = res.x.reshape(-1)[keep]
    assert np.max(np.abs(got - x)) <= 1e-10 * np.max(np.abs(x))
    assert np.all(res.x.reshape(-1)[~keep] == 0)


@pytest.mark.parametrize("kind", ["diag", "band"])
def test_noiseless_exact_recovery_and_monotone_error(kind):
    prob = _problem(nside=4, n_det=4, n_samp=1500, kind=kind, b=30)
    pix, c, s = prob.geometry()
    _, hits = mm.bj_build(pix, c, s, prob.wdiag(), prob.npix, prob.gain)
    m_true = np.random.default_rng(3).standard_normal((3, prob.npix))
    M, h = mm.bj_build(pix, c, s, prob.wdiag(), prob.npix, prob.gain)
    _, valid, _ = mm.bj_invert(M, h)
    m_true[:, ~valid] = 0.0
    d = pt.apply_pix(mm.flag_invalid(pix, valid), c, s, m_true, prob.gain)
    res = mm.pcg_mapmake(prob, d, max_iter=300, rtol=1e-13, keep_iterates=True)
    err = np.linalg.norm(res.x - m_true) / np.linalg.norm(m_true)
    assert err <= 1e-10
    # A-norm of the error decreases monotonically (CG optimality)
    pixv = mm.flag_invalid(pix, res.valid)
    anorm = []
    for xk in res.iterates:
        e = xk - m_true
        anorm.append(np.sum(e * mm.normal_apply(prob, pixv, c, s, e)))
    anorm = np.array(anorm)
    assert np.all(np.diff(anorm) <= 1e-12 * anorm[0])


def test_detector_split_sum_equals_unsplit():
    prob = _problem(nside=4, n_det=4, n_samp=800, kind="band", b=20)
    pix, c, s = prob.geometry()
    x = np.random.default_rng(4).standard_normal((3, prob.npix))
    full = mm.normal_apply(prob, pix, c, s, x)
    part = np.zeros_like(full)
    for sl in (slice(0, 1), slice(1, 3), slice(3, 4)):
        sub = mm.Problem(prob.nside, prob.theta[sl], prob.phi[sl], prob.psi[sl], "band",
                         lags=prob.lags, gain=prob.gain[sl], dpsi=prob.dpsi[sl], hwp=prob.hwp)
        ps, cs, ss = sub.geometry()
        part += mm.normal_apply(sub, ps, cs, ss, x)
    assert np.allclose(part, full, rtol=0, atol=1e-12 * np.abs(full).max())


def test_breakdown_on_nan_data():
    prob = _problem(nside=2, n_det=2, n_samp=300, kind="diag")
    d = np.ones(prob.theta.shape)
    d[0, 3] = np.nan
    res = mm.pcg_mapmake(prob, d, max_iter=10)
    assert res.stop_reason == mm.STOP_BREAKDOWN
    assert res.iters == 0 and np.all(res.x == 0)


def test_indefinite_noise_breaks_down():
    """A negative-definite kernel makes every block negative definite: no pixel
    passes the (Cholesky) validity test, and with every pixel forced valid the
    first <r, z> is not positive, which is a breakdown."""
    prob = _problem(nside=2, n_det=2, n_samp=300, kind="band", b=4)
    prob.lags = np.array([-1.0, 0.1, 0.0, 0.0])       # negative-definite kernel
    d = np.random.default_rng(0).standard_normal(prob.theta.shape)
    M6, hits = mm.bj_build(*prob.geometry(), prob.wdiag(), prob.npix, prob.gain)
    assert not mm.bj_invert(M6, hits)[1].any()
    res = mm.pcg_mapmake(prob, d, max_iter=10, valid_in=np.ones(prob.npix, bool))
    assert res.stop_reason == mm.STOP_BREAKDOWN

"""Pins of the oracle's template deprojection F_T (Eq. (3)) (CPU only)."""
import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

from oracle import mapmaker as mm
from oracle import pointing as pt
from oracle import templates as tp
from paper_2603_19600_amd import synth


def test_basis_is_numpys_legendre_series():
    for length, order in ((1, 0), (7, 3), (1000, 5), (33, 7)):
        B = tp.legendre_basis(length, order)
        x = (2.0 * np.arange(length) + 1.0) / length - 1.0
        for j in range(order + 1):
            c = np.zeros(j + 1)
            c[j] = 1.0
            assert np.allclose(B[:, j], npleg.legval(x, c), rtol=0, atol=1e-13)


def _stream(n_det=3, n_samp=1000, seed=0):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n_det, n_samp)), rng.uniform(0.5, 2.0, n_det)


@pytest.mark.parametrize("seg_len,order", [(100, 0), (128, 3), (333, 2), (1000, 5)])
def test_templates_are_projected_out(seg_len, order):
    y, w = _stream()
    n = y.shape[1]
    nseg = len(tp.segments(n, seg_len))
    amp = np.random.default_rng(1).standard_normal((3, nseg, order + 1))
    Tt = tp.template_signal(amp, n, seg_len, order)
    assert np.abs(tp.deproject_apply(Tt, w, seg_len, order)).max() < 1e-11 * np.abs(Tt).max()
    # T^T F_T y = 0: what is left has no template component
    Fy = tp.deproject_apply(y, w, seg_len, order)
    for k in range(3):
        T = tp.template_matrix(n, seg_len, order)
        assert np.abs(T.T @ Fy[k]).max() < 1e-11 * np.abs(y).max() * seg_len
    # amplitude estimate of pure template data returns the amplitudes
    assert np.allclose(tp.template_amplitudes(Tt, w, seg_len, order), amp, rtol=0, atol=1e-10)


def test_symmetric_psd_and_projector():
    u, w = _stream(seed=2)
    v, _ = _stream(seed=3)
    seg_len, order = 150, 3
    Fu = tp.deproject_apply(u, w, seg_len, order)
    Fv = tp.deproject_apply(v, w, seg_len, order)
    a, b = float((u * Fv).sum()), float((Fu * v).sum())
    assert abs(a - b) <= 1e-12 * abs(a)
    assert float((v * Fv).sum()) > 0.0
    # F_T W^-1 F_T = F_T
    FWF = tp.deproject_apply(Fv / w[:, None], w, seg_len, order)
    assert np.allclose(FWF, Fv, rtol=0, atol=1e-12 * np.abs(Fv).max())


def test_segmentwise_equals_dense_eq3():
    """F_T = W - W T (T^T W T)^-1 T^T W built densely from the whole stream's T."""
    y, w = _stream(n_det=2, n_samp=257, seed=4)
    seg_len, order = 64, 2
    T = tp.template_matrix(257, seg_len, order)
    got = tp.deproject_apply(y, w, seg_len, order)
    for k in range(2):
        W = w[k] * np.eye(257)
        F = W - W @ T @ np.linalg.inv(T.T @ W @ T) @ T.T @ W
        assert np.allclose(got[k], F @ y[k], rtol=0, atol=1e-12)


def _tiny_problem(seed=5):
    w = synth.WORKLOADS[2].with_(nside=2, n_det=4, n_samp=3000, seed=seed)
    p = synth.pointing(w)
    uth, uph = synth.uniform_sphere(seed, 4 * 3000)
    return mm.Problem(2, uth.numpy().reshape(4, 3000), uph.numpy().reshape(4, 3000), p.psi.numpy(),
                      "deproj", inv_var=np.array([1.0, 0.5, 2.0, 1.5]), hwp=(2, 50, 0.1),
                      tmpl=(500, 2))


def test_segments_cover_the_stream():
    assert tp.segments(1000, 333) == [(0, 333), (333, 666), (666, 1000)]
    assert tp.segments(100, 333) == [(0, 100)]
    assert tp.segments(666, 333) == [(0, 333), (333, 666)]


def test_map_recovered_from_data_with_template_signals():
    """d = P m + T t exactly: the deprojected GLS map is m up to the I monopole
    (a constant sky is itself an offset template in every segment, so P^T F_T P
    cannot see it), while the plain weighting W leaves a biased map."""
    prob = _tiny_problem()
    rng = np.random.default_rng(6)
    m = rng.standard_normal((3, prob.npix))
    pix, c, s = prob.geometry()
    nseg = len(tp.segments(3000, 500))
    amp = 5.0 * rng.standard_normal((4, nseg, 3))
    d = pt.apply_pix(pix, c, s, m) + tp.template_signal(amp, 3000, 500, 2)
    res = mm.pcg_mapmake(prob, d, max_iter=200, rtol=1e-13)
    assert res.valid.all()
    err = res.x - m
    mono = err[0].mean()
    assert np.abs(err[0] - mono).max() < 1e-9 and np.abs(err[1:]).max() < 1e-9
    plain = mm.Problem(prob.nside, prob.theta, prob.phi, prob.psi, "diag", inv_var=prob.inv_var,
                       hwp=prob.hwp)
    biased = mm.pcg_mapmake(plain, d, max_iter=200, rtol=1e-13)
    eb = biased.x - m
    assert np.abs(eb[0] - eb[0].mean()).max() > 0.1
    # and the template amplitudes come back from the residual (the monopole
    # moves into the offsets)
    m_fix = res.x.copy()
    m_fix[0] -= mono
    t_hat = tp.template_amplitudes(d - pt.apply_pix(pix, c, s, m_fix), prob.inv_var, 500, 2)
    assert np.allclose(t_hat, amp, rtol=0, atol=1e-8)

"""Pins of the oracle's gap filling by constrained Gaussian realisations (CPU only)."""
import numpy as np

from oracle import gapfill as gf
from oracle import noise as nz
from paper_2603_19600_amd import synth


def _case(n=300, b=20, seed=0):
    w = synth.WORKLOADS[2].with_(n_samp=n, n_det=3, seed=seed)
    c = synth.covariance_lags(w.with_(f_knee=2.0), b)
    rng = np.random.default_rng(seed)
    L = np.linalg.cholesky(nz.toeplitz_dense(n, c))
    d = (L @ rng.standard_normal((n, 3))).T
    nr = (L @ rng.standard_normal((n, 3))).T
    gaps = np.zeros((3, n), dtype=bool)
    gaps[0, 40:90] = True
    gaps[1, :7] = True
    gaps[1, 200:203] = True
    gaps[2, -30:] = True
    gaps[2, 100] = True
    return d, nr, gaps, c


def test_covariance_lags_positive_definite():
    w = synth.WORKLOADS[2]
    for b in (1, 65, 4096):
        c = synth.covariance_lags(w, b)
        assert nz.symbol_min(c) > 0.0


def test_valid_untouched_and_trivial_cases():
    d, nr, gaps, c = _case()
    out = gf.gap_fill(d, gaps, nr, c)
    assert np.array_equal(out[~gaps], d[~gaps])
    assert np.array_equal(gf.gap_fill(d, np.zeros_like(gaps), nr, c), d)
    # white covariance: the gaps get the unconstrained realisation itself
    outw = gf.gap_fill(d, gaps, nr, np.array([2.0]))
    assert np.allclose(outw[gaps], nr[gaps], rtol=0, atol=1e-14)
    # data equal to the realisation: nothing to constrain
    assert np.allclose(gf.gap_fill(nr, gaps, nr, c), nr, rtol=0, atol=1e-12)


def test_conditional_mean_against_precision_form():
    d, nr, gaps, c = _case(seed=1)
    out = gf.gap_fill(d, gaps, np.zeros_like(d), c)
    N = nz.toeplitz_dense(d.shape[1], c)
    Q = np.linalg.inv(N)
    for k in range(3):
        g, v = gaps[k], ~gaps[k]
        ref = -np.linalg.solve(Q[np.ix_(g, g)], Q[np.ix_(g, v)] @ d[k, v])
        assert np.allclose(out[k, g], ref, rtol=1e-9, atol=1e-9)


def test_constrained_realisations_have_the_conditional_covariance():
    n, b = 40, 8
    c = synth.covariance_lags(synth.WORKLOADS[2].with_(f_knee=5.0), b)
    N = nz.toeplitz_dense(n, c)
    L = np.linalg.cholesky(N)
    rng = np.random.default_rng(3)
    gaps = np.zeros((1, n), dtype=bool)
    gaps[0, 15:25] = True
    d = (L @ rng.standard_normal(n))[None, :]
    R = 20000
    nr = (L @ rng.standard_normal((n, R))).T                  # R realisations
    filled = np.array([gf.gap_fill(d, gaps, nr[r:r + 1], c)[0, 15:25] for r in range(R)])
    g, v = gaps[0], ~gaps[0]
    cond = N[np.ix_(g, g)] - N[np.ix_(g, v)] @ np.linalg.solve(N[np.ix_(v, v)], N[np.ix_(v, g)])
    mean = N[np.ix_(g, v)] @ np.linalg.solve(N[np.ix_(v, v)], d[0, v])
    emp = np.cov(filled.T)
    assert np.abs(filled.mean(0) - mean).max() < 5 * np.sqrt(cond.diagonal().max() / R)
    assert np.abs(emp - cond).max() < 0.05 * cond.diagonal().max()

"""Pins of the oracle's inverse-noise weighting (CPU only)."""
import numpy as np
import pytest

from oracle import noise as nz
from paper_2603_19600_amd import synth


@pytest.mark.parametrize("n,b", [(1, 1), (7, 3), (100, 1), (257, 64), (300, 300), (1000, 999),
                                 (4096, 512)])
def test_direct_dense_fft_agree(n, b):
    rng = np.random.default_rng(n * 31 + b)
    t = rng.standard_normal(b)
    y = rng.standard_normal(n)
    dense = nz.toeplitz_dense(n, t) @ y
    direct = nz.toeplitz_direct_row(y, t)
    fft = nz.toeplitz_fft_row(y, t)
    scale = np.abs(t).sum() * np.abs(y).max()
    assert np.max(np.abs(direct - dense)) <= 1e-13 * scale
    assert np.max(np.abs(fft - dense)) <= 1e-13 * scale


def test_one_over_f_lags_symmetric_positive_definite():
    w = synth.WORKLOADS[2]
    t = synth.toeplitz_lags(w, 512)
    n = 2000
    T = nz.toeplitz_dense(n, t)
    rng = np.random.default_rng(0)
    x, y = rng.standard_normal(n), rng.standard_normal(n)
    assert abs(np.dot(nz.toeplitz_direct_row(x, t), y) - np.dot(x, nz.toeplitz_direct_row(y, t))) \
        < 1e-12 * n
    assert np.linalg.eigvalsh(T).min() > 0
    assert np.dot(x, nz.toeplitz_direct_row(x, t)) > 0


@pytest.mark.parametrize("b", [4096, 8192])
def test_symbol_positive(b):
    t = synth.toeplitz_lags(synth.WORKLOADS[2], b)
    assert nz.symbol_min(t) > 0


def test_b1_reduces_to_diagonal():
    rng = np.random.default_rng(2)
    y = rng.standard_normal((3, 500))
    t = np.array([1.7])
    assert np.array_equal(nz.band_apply(y, t), nz.diag_apply(y, np.full(3, 1.7)))


def test_white_limit():
    w = synth.WORKLOADS[2].with_(f_knee=1e-12, sigma=2.0)
    t = synth.toeplitz_lags(w, 16)
    assert abs(t[0] - 0.25) < 1e-9
    assert np.max(np.abs(t[1:])) < 1e-9


def test_per_detector_kernels():
    rng = np.random.default_rng(5)
    y = rng.standard_normal((2, 400))
    t = rng.standard_normal((2, 9))
    out = nz.band_apply(y, t)
    for k in range(2):
        assert np.allclose(out[k], nz.toeplitz_dense(400, t[k]) @ y[k], atol=1e-12)

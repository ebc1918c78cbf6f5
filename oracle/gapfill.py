"""Gap filling by constrained Gaussian realisations, FP64, NumPy (oracle; test
infrastructure only).

What is computed (paper, the paragraph after Table 2: the symmetric
band-Toeplitz operator is central to correlated-noise modelling and to
gap-filling by constrained Gaussian realisations): a detector's stream d has
missing samples G and valid samples V, and its noise is Gaussian with the
stationary covariance N, a symmetric band-Toeplitz matrix of autocorrelation
lags c[0..b-1].  Given an unconstrained realisation n ~ N(0, N) (an input:
the random numbers are drawn by the caller), the constrained realisation

    d_G = n_G + N_GV N_VV^-1 (d_V - n_V),     d_V unchanged,

has the conditional distribution of the missing samples given the valid
ones; with n = 0 it is the conditional mean (Wiener interpolation).

Readings of the open points: the covariance is the truncated linear
convolution of the band (zero outside the stream), as for the weights; each
detector is filled independently; white covariance (b = 1) gives d_G = n_G.

Pins (tests/test_oracle_gapfill.py): valid samples untouched; no gaps
returns d; white covariance returns n on the gaps; d = n returns n; the
conditional mean against the precision-matrix form -(Q_GG)^-1 Q_GV d_V with
Q = N^-1 (an independent formula for the same Gaussian conditional); the
sample covariance of many constrained realisations against the conditional
covariance N_GG - N_GV N_VV^-1 N_VG.
"""
from __future__ import annotations

import numpy as np

from .noise import toeplitz_dense


def gap_fill(tod, gaps, noise_real, c) -> np.ndarray:
    """Constrained realisation for tod [n_det, n_samp] with gaps [n_det, n_samp]
    (True = missing), an unconstrained realisation noise_real of the same shape
    and covariance lags c ([b] or [n_det, b]).  Dense: small streams only."""
    tod = np.asarray(tod, dtype=np.float64)
    nr = np.asarray(noise_real, dtype=np.float64)
    gaps = np.asarray(gaps, dtype=bool)
    c = np.asarray(c, dtype=np.float64)
    out = tod.copy()
    n = tod.shape[1]
    for k in range(tod.shape[0]):
        g = gaps[k]
        if not g.any():
            continue
        v = ~g
        ck = c if c.ndim == 1 else c[k]
        Nk = toeplitz_dense(n, ck)
        x = np.linalg.solve(Nk[np.ix_(v, v)], tod[k, v] - nr[k, v])
        out[k, g] = nr[k, g] + Nk[np.ix_(g, v)] @ x
    return out

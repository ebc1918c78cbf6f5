"""Template deprojection, FP64, NumPy (oracle; test infrastructure only).

What is computed (paper, Eq. (1)-(3) and the TemplateOperator of Table 3):
the data model d = H m + T t + n carries unwanted additive signals T t, and
the generalised least-squares estimator weights the data with

    F_T = W - W T (T^T W T)^-1 T^T W                          (Eq. (3))

for positive-definite weights W, which removes every component of the data
that the templates T can represent.  The map is then
m = (P^T F_T P)^-1 P^T F_T d (Eq. (2), F_T in the role of the weight, as
with T = 0 the weight is W = N^-1).

Readings of points the paper leaves open (it names neither T nor W):
  * W is diagonal per detector, w_k I (the white-noise weights);
  * T is block-diagonal over detectors and over consecutive segments of
    seg_len samples, the last segment absorbing the remainder (so segments
    have seg_len to 2 seg_len - 1 samples, or the whole stream when it is
    shorter than seg_len; a stream needs at least order + 1 samples): on each
    segment, the Legendre polynomials P_0 .. P_order of the sample's position
    x_i = (2 (i - i0) + 1) / len - 1 (cell centres in (-1, 1)), i.e. slowly
    varying baselines per detector and segment;
  * so T^T W T is one (order+1) x (order+1) block per (detector, segment)
    and F_T acts on each segment independently:
        F_T y = w (y - T_s G_s^-1 T_s^T y),   G_s = T_s^T T_s.

Pins (tests/test_oracle_templates.py): the basis against numpy's Legendre
series; F_T T = 0 and T^T F_T = 0; symmetry and positive semi-definiteness;
F_T W^-1 F_T = F_T; the segment-wise application against F_T built densely
from the full T of a tiny stream; exact recovery of a map from noiseless
data that carries template signals, and of the template amplitudes.
"""
from __future__ import annotations

import numpy as np


def legendre_basis(length: int, order: int) -> np.ndarray:
    """[length, order + 1]: P_j(x_i) at x_i = (2 i + 1) / length - 1."""
    x = (2.0 * np.arange(length, dtype=np.float64) + 1.0) / length - 1.0
    B = np.empty((length, order + 1))
    B[:, 0] = 1.0
    if order >= 1:
        B[:, 1] = x
    for j in range(1, order):                       # (j+1) P_{j+1} = (2j+1) x P_j - j P_{j-1}
        B[:, j + 1] = ((2 * j + 1) * x * B[:, j] - j * B[:, j - 1]) / (j + 1)
    return B


def segments(n_samp: int, seg_len: int):
    """[(i0, i1)] of the segments: n_samp // seg_len of them (at least one), the
    last one running to the end of the stream."""
    nseg = max(1, n_samp // seg_len)
    return [(s * seg_len, (s + 1) * seg_len if s + 1 < nseg else n_samp) for s in range(nseg)]


def template_matrix(n_samp: int, seg_len: int, order: int) -> np.ndarray:
    """One detector's dense T [n_samp, n_seg (order + 1)] (for small streams)."""
    segs = segments(n_samp, seg_len)
    T = np.zeros((n_samp, len(segs) * (order + 1)))
    for s, (i0, i1) in enumerate(segs):
        T[i0:i1, s * (order + 1):(s + 1) * (order + 1)] = legendre_basis(i1 - i0, order)
    return T


def deproject_apply(tod, w, seg_len: int, order: int) -> np.ndarray:
    """F_T y for tod [n_det, n_samp] with W = diag(w_k), Eq. (3) per segment."""
    tod = np.asarray(tod, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    out = np.empty_like(tod)
    n = tod.shape[1]
    for k in range(tod.shape[0]):
        for i0, i1 in segments(n, seg_len):
            Ts = legendre_basis(i1 - i0, order)
            Wy = w[k] * tod[k, i0:i1]
            WT = w[k] * Ts
            amp = np.linalg.solve(Ts.T @ WT, Ts.T @ Wy)      # (T^T W T)^-1 T^T W y
            out[k, i0:i1] = Wy - WT @ amp
    return out


def template_amplitudes(tod, w, seg_len: int, order: int) -> np.ndarray:
    """(T^T W T)^-1 T^T W y: [n_det, n_seg, order + 1], the template fit."""
    tod = np.asarray(tod, dtype=np.float64)
    segs = segments(tod.shape[1], seg_len)
    out = np.empty((tod.shape[0], len(segs), order + 1))
    for k in range(tod.shape[0]):
        for s, (i0, i1) in enumerate(segs):
            Ts = legendre_basis(i1 - i0, order)
            out[k, s] = np.linalg.solve(Ts.T @ (w[k] * Ts), Ts.T @ (w[k] * tod[k, i0:i1]))
    return out


def template_signal(amp, n_samp: int, seg_len: int, order: int) -> np.ndarray:
    """T t for amplitudes [n_det, n_seg, order + 1]: tod [n_det, n_samp]."""
    amp = np.asarray(amp, dtype=np.float64)
    out = np.zeros((amp.shape[0], n_samp))
    for s, (i0, i1) in enumerate(segments(n_samp, seg_len)):
        out[:, i0:i1] = amp[:, s, :] @ legendre_basis(i1 - i0, order).T
    return out

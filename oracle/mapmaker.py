"""Block-Jacobi preconditioned CG map-maker, FP64, NumPy (oracle; test infrastructure only).

What is computed:
  * the GLS / maximum-likelihood map of Eq. (2) with no templates (T = 0),
    so the weighting is W = N^-1 and the estimator is
        m_hat = (P^T N^-1 P)^-1 P^T N^-1 d,
    as the listing's estimator (H.T @ N.I @ H).I @ H.T @ N.I states it
    (section "Software Design");
  * the inverse is taken iteratively (Table 1, "A.I(solver=...,
    preconditioner=...)") by preconditioned conjugate gradients;
  * the preconditioner is block Jacobi ("BJPreconditioner", paragraph
    "Map-making classes"): one 3x3 block per pixel, the pixel's diagonal
    block of P^T diag(N^-1) P;
  * the binned estimator of the same paragraph is that preconditioner applied
    to P^T N^-1 d.

Readings of points the paper leaves open:
  * a pixel is solved for ("valid") iff it has at least 3 hits and the
    1-norm reciprocal condition number of its 3x3 block is >= 1e-3; samples
    that fall in other pixels are flagged (pixel := -1) in both P and P^T,
    which makes the operator SPD on the valid set; invalid pixels output 0;
  * PCG in textbook (Hestenes-Stiefel) form from x0 = 0; dot products over
    all 3 npix unknowns (invalid ones are identically zero) with math.fsum;
    stop when ||r|| / ||b|| <= rtol or after max_iter iterations; breakdown if
    <p, q> <= 0, <r, z> <= 0 or either is non-finite, returning the last
    good iterate.

Pins: with diagonal N the block-Jacobi preconditioner IS the inverse, so PCG
reaches the per-pixel np.linalg.solve binned map in one iteration; with band
N on tiny inputs the result equals np.linalg.solve of the dense normal
matrix; noiseless data recover the input map exactly; the A-norm of the
error decreases monotonically; the 3x3 inverse and rcond match a block
inverted by hand (adjugate over determinant) and diagonal blocks, and blocks
singular in exact arithmetic come out invalid; a detector-split sum equals the
unsplit one.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import noise as _noise
from . import pointing as _pt
from . import quaternion as _quat
from .healpix import zphi2pix_ring

STOP_MAXITER = 0
STOP_RTOL = 1
STOP_BREAKDOWN = 2


def bj_build(pix, c, s, wdiag, npix: int, gain=None):
    """Per-pixel 3x3 blocks M_p = sum g_k^2 w_k (1,c,s)^T (1,c,s).

    Returns (M [6, npix] as II, IQ, IU, QQ, QU, UU; hits [npix] int64).
    """
    M = np.zeros((6, npix))
    hits = np.zeros(npix, dtype=np.int64)
    for k in range(pix.shape[0]):
        ok = pix[k] >= 0
        p = pix[k][ok]
        g = 1.0 if gain is None else float(gain[k])
        w = g * g * float(wdiag[k])
        ck, sk = c[k][ok], s[k][ok]
        wv = np.full(p.shape, w)
        M[0] += np.bincount(p, weights=wv, minlength=npix)
        M[1] += np.bincount(p, weights=wv * ck, minlength=npix)
        M[2] += np.bincount(p, weights=wv * sk, minlength=npix)
        M[3] += np.bincount(p, weights=wv * ck * ck, minlength=npix)
        M[4] += np.bincount(p, weights=wv * ck * sk, minlength=npix)
        M[5] += np.bincount(p, weights=wv * sk * sk, minlength=npix)
        hits += np.bincount(p, minlength=npix)
    return M, hits


def sym3(M6) -> np.ndarray:
    """[6, n] unique entries -> [n, 3, 3] symmetric matrices."""
    a, b, c, d, e, f = M6
    return np.stack([np.stack([a, b, c], -1), np.stack([b, d, e], -1),
                     np.stack([c, e, f], -1)], -2)


def bj_invert(M6, hits, rcond_min: float = 1e-3, min_hits: int = 3):
    """Inverse and 1-norm reciprocal condition number of each 3x3 block, by definition.

    For each pixel's block M (sym3 of M6):
      * rcond = 1 / (||M||_1 ||M^-1||_1), i.e. 1 / numpy.linalg.cond(M, 1), for a
        block that is positive definite (every eigenvalue > 0, numpy.linalg.eigvalsh)
        with a finite condition number; rcond = 0 for any other block (singular,
        indefinite, non-finite).  The blocks of the method are sums of
        w (1, c, s)^T (1, c, s) with w > 0, so they are positive semi-definite,
        and one that is singular in exact arithmetic (all of a pixel's samples at
        one polariser angle, or at two angles pi/2 apart) has a tiny rcond, or 0;
      * M^-1 = numpy.linalg.inv(M) on the blocks with rcond > 0, 0 elsewhere;
      * valid = hits >= min_hits and rcond >= rcond_min; Minv is 0 on invalid pixels.

    Returns (Minv [6, npix] as II, IQ, IU, QQ, QU, UU; valid [npix] bool; rcond [npix]).
    """
    Ms = sym3(np.asarray(M6, dtype=np.float64))
    n = Ms.shape[0]
    rcond = np.zeros(n)
    inv = np.zeros((6, n))
    # an all-zero block (unobserved pixel) is singular: rcond 0, inverse 0
    fin = np.isfinite(Ms).all(axis=(1, 2)) & (Ms != 0.0).any(axis=(1, 2))
    if fin.any():
        Mf = Ms[fin]
        with np.errstate(all="ignore"):
            cond = np.linalg.cond(Mf, 1)              # inf for a singular block
        pd = np.linalg.eigvalsh(Mf)[:, 0] > 0.0
        ok = pd & np.isfinite(cond)
        rc = np.zeros(len(Mf))
        rc[ok] = 1.0 / cond[ok]
        rcond[fin] = rc
        idx = np.flatnonzero(fin)[ok]
        if idx.size:
            Mi = np.linalg.inv(Ms[idx])
            inv[:, idx] = np.stack([Mi[:, 0, 0], Mi[:, 0, 1], Mi[:, 0, 2],
                                    Mi[:, 1, 1], Mi[:, 1, 2], Mi[:, 2, 2]])
    valid = (np.asarray(hits) >= min_hits) & (rcond >= rcond_min)
    inv = np.where(valid[None, :], inv, 0.0)
    return inv, valid, rcond


def bj_apply(Minv6, r) -> np.ndarray:
    """z_p = M_p^-1 r_p for r [3, npix]."""
    a, b, c, d, e, f = Minv6
    return np.stack([a * r[0] + b * r[1] + c * r[2],
                     b * r[0] + d * r[1] + e * r[2],
                     c * r[0] + e * r[1] + f * r[2]])


def dot(u, v) -> float:
    """sum_j u_j v_j, each product rounded once and the sum exactly rounded
    (math.fsum); zero products (unobserved unknowns) are left out, which does
    not change an exact sum."""
    prod = (np.asarray(u) * np.asarray(v)).ravel()
    return math.fsum(prod[prod != 0.0].tolist())


@dataclass
class Problem:
    """A map-making problem: pointing, noise model and data."""
    nside: int
    theta: np.ndarray
    phi: np.ndarray
    psi: np.ndarray
    noise_kind: str                     # "diag", "band" or "deproj" (templates)
    inv_var: np.ndarray | None = None   # [n_det] for "diag"
    lags: np.ndarray | None = None      # [b] or [n_det, b] for "band"
    gain: np.ndarray | None = None
    dpsi: np.ndarray | None = None
    hwp: tuple | None = None            # (num, den, phase0)
    bore_quat: np.ndarray | None = None # [n_samp, 4]: quaternion pointing (theta/phi/psi None)
    det_quat: np.ndarray | None = None  # [n_det, 4]
    tmpl: tuple | None = None           # (seg_len, order) for noise_kind "deproj" (Eq. (3))

    @property
    def npix(self):
        return 12 * self.nside * self.nside

    @property
    def n_det(self):
        return self.det_quat.shape[0] if self.bore_quat is not None else self.theta.shape[0]

    def geometry(self):
        if self.bore_quat is not None:
            z, phi, psi = _quat.expand(self.bore_quat, self.det_quat)
            pix = zphi2pix_ring(self.nside, z, phi)
        else:
            pix = _pt.pixels(self.nside, self.theta, self.phi)
            psi = self.psi
        c, s = _pt.weights(psi, self.dpsi, self.hwp)
        return pix, c, s

    def ninv(self, y):
        return _noise.noise_apply(self.noise_kind, y, self.inv_var, self.lags, tmpl=self.tmpl)

    def wdiag(self):
        return _noise.diag_of_inverse(self.noise_kind, self.n_det, self.inv_var, self.lags)


def flag_invalid(pix, valid) -> np.ndarray:
    ok = pix >= 0
    keep = np.zeros_like(ok)
    keep[ok] = valid[pix[ok]]
    return np.where(keep, pix, -1)


def normal_apply(prob: Problem, pix, c, s, x) -> np.ndarray:
    """A x = P^T N^-1 P x on the (flagged) pixel set."""
    y = _pt.apply_pix(pix, c, s, x, prob.gain)
    z = prob.ninv(y)
    return _pt.transpose_pix(pix, c, s, z, prob.npix, prob.gain)


@dataclass
class PCGResult:
    x: np.ndarray
    valid: np.ndarray
    iters: int
    stop_reason: int
    rel_resid: float
    resid_history: list = field(default_factory=list)
    iterates: list = field(default_factory=list)


def pcg_mapmake(prob: Problem, d, max_iter: int = 50, rtol: float = 0.0,
                rcond_min: float = 1e-3, min_hits: int = 3, valid_in=None,
                keep_iterates: bool = False) -> PCGResult:
    """Solve (P^T N^-1 P) x = P^T N^-1 d by block-Jacobi PCG."""
    pix, c, s = prob.geometry()
    npix = prob.npix
    M, hits = bj_build(pix, c, s, prob.wdiag(), npix, prob.gain)
    Minv, valid, _ = bj_invert(M, hits, rcond_min, min_hits)
    if valid_in is not None:
        valid = np.asarray(valid_in, dtype=bool)
        Minv = np.where(valid[None, :], bj_invert(M, hits, -np.inf, 0)[0], 0.0)
    pixv = flag_invalid(pix, valid)

    b = _pt.transpose_pix(pixv, c, s, prob.ninv(np.asarray(d, dtype=np.float64)), npix, prob.gain)
    x = np.zeros((3, npix))
    r = b.copy()
    z = bj_apply(Minv, r)
    p = z.copy()
    rz = dot(r, z)
    bnorm = math.sqrt(dot(b, b))
    hist = [1.0 if bnorm > 0 else 0.0]
    iterates = []
    stop = STOP_MAXITER
    k = 0
    if bnorm == 0.0:
        return PCGResult(x, valid, 0, STOP_RTOL, 0.0, hist, iterates)
    if not (math.isfinite(rz) and rz > 0.0):
        return PCGResult(x, valid, 0, STOP_BREAKDOWN, 1.0, hist, iterates)
    while k < max_iter:
        q = normal_apply(prob, pixv, c, s, p)
        pq = dot(p, q)
        if not (math.isfinite(pq) and pq > 0.0):
            stop = STOP_BREAKDOWN
            break
        alpha = rz / pq
        x = x + alpha * p
        r = r - alpha * q
        k += 1
        rel = math.sqrt(dot(r, r)) / bnorm
        hist.append(rel)
        if keep_iterates:
            iterates.append(x.copy())
        if rel <= rtol:
            stop = STOP_RTOL
            break
        z = bj_apply(Minv, r)
        rz_new = dot(r, z)
        if not (math.isfinite(rz_new) and rz_new > 0.0):
            stop = STOP_BREAKDOWN
            break
        beta = rz_new / rz
        rz = rz_new
        p = z + beta * p
    return PCGResult(x, valid, k, stop, hist[-1], hist, iterates)


def binned_map(prob: Problem, d, rcond_min: float = 1e-3, min_hits: int = 3):
    """Binned estimator: the block-Jacobi preconditioner applied to P^T N^-1 d."""
    pix, c, s = prob.geometry()
    M, hits = bj_build(pix, c, s, prob.wdiag(), prob.npix, prob.gain)
    Minv, valid, _ = bj_invert(M, hits, rcond_min, min_hits)
    pixv = flag_invalid(pix, valid)
    b = _pt.transpose_pix(pixv, c, s, prob.ninv(np.asarray(d, dtype=np.float64)), prob.npix,
                          prob.gain)
    return bj_apply(Minv, b), valid

"""Helpers shared by the GPU parity tests: seeded inputs on both sides."""
import math

import numpy as np
import torch

from paper_2603_19600_amd import synth


def dev():
    return torch.device("cuda:0")


def case(nside=16, n_det=3, n_samp=5000, seed=7, hwp=True, gains=True, dpsi=True, dtype="f64",
         sphere=False, offsets_deg=1.0):
    """A small seeded workload: (Workload, host pointing dict (float64 numpy), device tensors)."""
    w = synth.WORKLOADS[2].with_(nside=nside, n_det=n_det, n_samp=n_samp, seed=seed,
                                 dtype=dtype, hwp=hwp, offsets_deg=offsets_deg)
    pt = synth.pointing(w)
    th, ph, ps = pt.theta, pt.phi, pt.psi
    if sphere:
        uth, uph = synth.uniform_sphere(seed, n_det * n_samp)
        tdt = th.dtype
        th = uth.reshape(n_det, n_samp).to(tdt)
        ph = uph.reshape(n_det, n_samp).to(tdt)
    g = synth.gains(w, scale=0.05) if gains else None
    d = synth.angle_offsets(w) if dpsi else None
    hw = (w.hwp_num, w.hwp_den, 0.25) if hwp else None
    host = dict(theta=th.double().numpy(), phi=ph.double().numpy(), psi=ps.double().numpy(),
                gain=None if g is None else g.numpy(), dpsi=None if d is None else d.numpy(),
                hwp=hw)
    return w, host, dict(theta=th, phi=ph, psi=ps, gain=g, dpsi=d, hwp=hw)


def to_pointing(nside, t):
    from paper_2603_19600_amd import furax as fx
    D = dev()
    return fx.Pointing(nside, t["theta"].to(D).contiguous(), t["phi"].to(D).contiguous(),
                       t["psi"].to(D).contiguous(),
                       None if t["gain"] is None else t["gain"].to(D),
                       None if t["dpsi"] is None else t["dpsi"].to(D), t["hwp"])


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (den if den > 0 else 1.0))


def check_pixel_mismatches(nside, theta, phi, got, ref, z=None):
    """Every pixel where the device (got) and the oracle (ref) disagree must be
    explained by a one-ulp difference of the cosine: with z_cr the correctly
    rounded cos(theta) (mpmath at 40 digits; or the given z, for directions
    whose cosine is known), the pixel must change between z_cr - 1 ulp and
    z_cr + 1 ulp (the direction lies in the ulp band of a ring or pixel edge),
    got must be the pixel of one of z_cr - 1 ulp, z_cr, z_cr + 1 ulp, and the
    oracle's answer too.  No other mismatch is allowed.  Returns the number of
    explained mismatches."""
    import mpmath

    from oracle import healpix as ohp

    got = np.asarray(got).ravel()
    ref = np.asarray(ref).ravel()
    theta = np.asarray(theta, dtype=np.float64).ravel()
    phi = np.asarray(phi, dtype=np.float64).ravel()
    mism = np.flatnonzero(got != ref)
    for i in mism:
        if z is None:
            with mpmath.workdps(40):
                zc = float(mpmath.cos(mpmath.mpf(float(theta[i]))))
        else:
            zc = float(np.asarray(z).ravel()[i])
        cand = np.array([np.nextafter(zc, -2.0), zc, np.nextafter(zc, 2.0)])
        pc = ohp.zphi2pix_ring(nside, cand, np.full(3, phi[i]))
        band = len(set(pc.tolist())) > 1
        assert band, (f"pixel mismatch outside the ulp band: theta={theta[i]!r} phi={phi[i]!r} "
                      f"got {got[i]} oracle {ref[i]} (cos band pixels {pc.tolist()})")
        assert int(got[i]) in pc.tolist() and int(ref[i]) in pc.tolist(), (
            f"theta={theta[i]!r} phi={phi[i]!r}: got {got[i]}, oracle {ref[i]}, "
            f"pixels within one ulp of the correctly rounded cosine {pc.tolist()}")
    return len(mism)

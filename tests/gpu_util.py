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

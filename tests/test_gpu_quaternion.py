"""GPU parity of boresight-quaternion pointing against the FP64 oracle.

Pixels are read back exactly: P applied to the map I = pixel + 1, Q = U = 0
returns pixel + 1 per sample (exact in FP64, and in FP32 below 2^24 pixels).
They must equal the oracle's except where the device and host atan2 differ by
one ulp at a pixel edge (checked by moving phi by one ulp on the host).
Operators: P, P^T (LDS-hash tiles), the normal operator with band N (the
superpixel transpose), block-Jacobi blocks, PCG and the chi-square gradient,
at sizes spanning many tiles with ragged tails, and rows of the full
nside-512 / 256 x 2^20 quaternion workload."""
import math

import numpy as np
import pytest
import torch

from oracle import chi2 as och
from oracle import healpix as ohp
from oracle import mapmaker as omm
from oracle import pointing as opt
from oracle import quaternion as oq
from paper_2603_19600_amd import synth
from tests.gpu_util import dev, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fx():
    from paper_2603_19600_amd import furax
    return furax


def _qcase(fx, nside, n_det, n_samp, dtype=torch.float64, hwp=True, gains=True, dpsi=True,
           seed=7, kind="band", b=65):
    w = synth.WORKLOADS[2].with_(nside=nside, n_det=n_det, n_samp=n_samp, seed=seed, hwp=hwp,
                                 pointing="quat")
    qb = synth.boresight_quaternions(w)
    qd = synth.detector_quaternions(w)
    g = synth.gains(w, scale=0.05) if gains else None
    dp = synth.angle_offsets(w) if dpsi else None
    hw = (w.hwp_num, w.hwp_den, 0.25) if hwp else None
    D = dev()
    P = fx.QuatPointing(nside, qb.to(D), qd.to(D), dtype,
                        None if g is None else g.to(D), None if dp is None else dp.to(D), hw)
    if kind == "diag":
        iv = np.linspace(0.5, 2.0, n_det)
        N = fx.Noise("diag", n_det, n_samp, inv_var=torch.from_numpy(iv).to(D))
        prob = omm.Problem(nside, None, None, None, "diag", inv_var=iv,
                           gain=None if g is None else g.numpy(),
                           dpsi=None if dp is None else dp.numpy(), hwp=hw,
                           bore_quat=qb.numpy(), det_quat=qd.numpy())
    else:
        lags = synth.toeplitz_lags(w, b)
        N = fx.Noise("band", n_det, n_samp, lags=torch.from_numpy(lags).to(D))
        prob = omm.Problem(nside, None, None, None, "band", lags=lags,
                           gain=None if g is None else g.numpy(),
                           dpsi=None if dp is None else dp.numpy(), hwp=hw,
                           bore_quat=qb.numpy(), det_quat=qd.numpy())
    return w, P, N, prob


def _pixels_via_P(fx, P):
    m = torch.zeros(3, P.npix, dtype=torch.float64, device=P.device)
    m[0] = torch.arange(1, P.npix + 1, dtype=torch.float64, device=P.device)
    Pp = P.with_(gain=None)
    y = fx.pointing_apply(Pp, m if P.dtype == torch.float64 else m.float())
    return y.double().cpu().numpy().astype(np.int64) - 1


def _check_pixels(nside, got, qb, qd):
    ref = oq.pixels(nside, qb, qd)
    bad = np.argwhere(got != ref)
    if len(bad):
        d, _ = oq.line_of_sight(oq.detector_attitude(qb, qd))
        for k, i in bad:
            z = np.clip(d[k, i, 2], -1.0, 1.0)
            ph = math.atan2(d[k, i, 1], d[k, i, 0])
            near = {int(ohp.zphi2pix_ring(nside, z, p))
                    for p in (np.nextafter(ph, -4), ph, np.nextafter(ph, 4))}
            assert got[k, i] in near, (k, i, got[k, i], ref[k, i])
    assert len(bad) <= max(2, got.size // 10 ** 7)


@pytest.mark.parametrize("nside,n_det,n_samp", [(64, 4, 50000), (512, 8, 1 << 16),
                                                (1, 3, 4097), (8192, 2, 30001)])
def test_quaternion_pixels_bitexact(fx, nside, n_det, n_samp):
    w, P, N, prob = _qcase(fx, nside, n_det, n_samp, kind="diag")
    got = _pixels_via_P(fx, P)
    _check_pixels(nside, got, prob.bore_quat, prob.det_quat)


def test_quaternion_pixels_bitexact_fp32_path(fx):
    w, P, N, prob = _qcase(fx, 256, 5, 40001, dtype=torch.float32, kind="diag")
    got = _pixels_via_P(fx, P)
    _check_pixels(256, got, prob.bore_quat, prob.det_quat)


@pytest.mark.parametrize("dpsi", [True, False])   # False: the tabulated HWP turn
@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 2e-6)])
def test_quaternion_P_and_PT(fx, dtype, tol, dpsi):
    w, P, N, prob = _qcase(fx, 32, 5, 30001, dtype=dtype, kind="diag", dpsi=dpsi)
    m = synth.sky_map(w).numpy()
    pix, c, s = prob.geometry()
    y_ref = opt.apply_pix(pix, c, s, m, prob.gain)
    mt = torch.from_numpy(m).to(dev())
    y = fx.pointing_apply(P, mt if dtype == torch.float64 else mt.float())
    assert rel_err(y.double().cpu().numpy(), y_ref) <= tol
    d = torch.from_numpy(y_ref).to(dev()).to(dtype)
    q = fx.pointing_transpose(P, d)
    q_ref = opt.transpose_pix(pix, c, s, d.double().cpu().numpy(), prob.npix, prob.gain)
    assert rel_err(q.cpu().numpy(), q_ref) <= tol


@pytest.mark.parametrize("dpsi", [True, False])
@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 2e-6)])
def test_quaternion_normal_operator_band(fx, dtype, tol, dpsi):
    """Band N with a power-of-two nside: the superpixel transpose path."""
    w, P, N, prob = _qcase(fx, 64, 6, 40000, dtype=dtype, kind="band", b=129, dpsi=dpsi)
    g = torch.Generator(device=dev()).manual_seed(3)
    x = torch.randn(3, P.npix, dtype=torch.float64, device=dev(), generator=g)
    got = fx.normal_apply(P, N, x).cpu().numpy()
    pix, c, s = prob.geometry()
    ref = omm.normal_apply(prob, pix, c, s, x.cpu().numpy())
    assert rel_err(got, ref) <= tol


def test_quaternion_bj_blocks(fx):
    w, P, N, prob = _qcase(fx, 32, 4, 30000, kind="diag")
    M6, hits = fx.bj_build(P, N)
    pix, c, s = prob.geometry()
    M_ref, h_ref = omm.bj_build(pix, c, s, prob.wdiag(), prob.npix, prob.gain)
    assert np.array_equal(hits.cpu().numpy(), h_ref)
    assert rel_err(M6.cpu().numpy(), M_ref) <= 1e-12


@pytest.mark.parametrize("kind,dpsi", [("diag", True), ("band", True), ("band", False)])
def test_quaternion_pcg_matches_oracle(fx, kind, dpsi):
    w, P, N, prob = _qcase(fx, 32, 4, 40000, kind=kind, b=65, dpsi=dpsi)
    m = synth.sky_map(w).numpy()
    n = synth.noise(w.with_(noise="diag")).numpy()
    pix, c, s = prob.geometry()
    d = opt.apply_pix(pix, c, s, m, prob.gain) + n
    # diagonal N is solved exactly at the first iteration; the iterations after
    # it act on rounding-level residuals that shrink until they underflow, so
    # where each side stops there is noise: compare the first three
    iters = 3 if kind == "diag" else 15
    ref = omm.pcg_mapmake(prob, d, max_iter=iters, rtol=0.0)
    x, valid, info, _ = fx.pcg_mapmake(P, N, torch.from_numpy(d).to(dev()), max_iter=iters,
                                       rtol=0.0, valid_in=torch.from_numpy(
                                           ref.valid.astype(np.uint8)).to(dev()))
    assert info.iters == ref.iters
    assert rel_err(x.cpu().numpy(), ref.x) <= 1e-10


def test_quaternion_chi2_gradient(fx):
    w, P, N, prob = _qcase(fx, 32, 4, 20000, kind="diag", gains=False, dpsi=False)
    m0 = synth.sky_map(w).numpy()
    pix, c, s = prob.geometry()
    d = opt.apply_pix(pix, c, s, m0, None) + synth.noise(w.with_(noise="diag")).numpy()
    rng = np.random.default_rng(5)
    mm = m0 + 0.1 * rng.standard_normal(m0.shape)
    g0 = 1.0 + 0.02 * np.arange(4)
    d0 = 0.01 * np.arange(4)
    m = torch.tensor(mm, device=dev(), requires_grad=True)
    g = torch.tensor(g0, device=dev(), requires_grad=True)
    dp = torch.tensor(d0, device=dev(), requires_grad=True)
    loss = fx.chi2_loss(P, N, torch.from_numpy(d).to(dev()), m, g, dp)
    loss.backward()
    val, gm, gg, gd = och.chi2_grad_quat(32, prob.bore_quat, prob.det_quat, d, mm, g0, d0,
                                         "diag", inv_var=prob.inv_var, hwp=prob.hwp)
    assert abs(loss.item() - val) <= 1e-12 * abs(val)
    assert rel_err(m.grad.cpu().numpy(), gm) <= 1e-12
    assert rel_err(g.grad.cpu().numpy(), gg) <= 1e-12
    assert rel_err(dp.grad.cpu().numpy(), gd) <= 1e-12


def test_quaternion_argument_errors(fx):
    w, P, N, prob = _qcase(fx, 16, 2, 100, kind="diag")
    m = torch.zeros(3, P.npix, dtype=torch.float64, device=dev())
    cp = P.c()
    # both representations at once
    cp.theta = P.bore_quat.data_ptr()
    out = torch.empty(2, 100, dtype=torch.float64, device=dev())
    st = fx._lib.furax_pointing_apply(fx.C.byref(cp), fx.F64, fx._ptr(m), fx.F64,
                                      fx._ptr(out), None)
    assert st == fx.EINVAL
    # misaligned quaternion array
    cp = P.c()
    cp.bore_quat = P.bore_quat.data_ptr() + 8
    st = fx._lib.furax_pointing_apply(fx.C.byref(cp), fx.F64, fx._ptr(m), fx.F64,
                                      fx._ptr(out), None)
    assert st == fx.EINVAL
    # missing detector attitudes
    cp = P.c()
    cp.det_quat = None
    st = fx._lib.furax_pointing_apply(fx.C.byref(cp), fx.F64, fx._ptr(m), fx.F64,
                                      fx._ptr(out), None)
    assert st == fx.EINVAL


@pytest.fixture(scope="module")
def full(fx):
    w = synth.WORKLOADS[3].with_(pointing="quat")
    D = dev()
    qb = synth.boresight_quaternions(w, device=D)
    qd = synth.detector_quaternions(w, device=D)
    hwp = (w.hwp_num, w.hwp_den, 0.0)
    P32 = fx.QuatPointing(w.nside, qb, qd, torch.float32, hwp=hwp)
    P64 = fx.QuatPointing(w.nside, qb, qd, torch.float64, hwp=hwp)
    lags = synth.toeplitz_lags(w)
    N = fx.Noise("band", w.n_det, w.n_samp, lags=torch.from_numpy(lags).to(D))
    return dict(w=w, P32=P32, P64=P64, N=N, lags=lags, hwp=hwp, qb=qb.cpu().numpy(),
                qd=qd.cpu().numpy(), m=synth.sky_map(w, device=D))


ROWS = (0, 91, 255)


def test_full_quaternion_rows(fx, full):
    """Pixels and P rows of the full nside-512 / 256 x 2^20 stream against the oracle."""
    w = full["w"]
    qd_rows = full["qd"][list(ROWS)]
    got = _pixels_via_P(fx, full["P64"])[list(ROWS)]
    _check_pixels(w.nside, got, full["qb"], qd_rows)
    z, phi, psi = oq.expand(full["qb"], qd_rows)
    pix = ohp.zphi2pix_ring(w.nside, z, phi)
    c, s = opt.weights(psi, None, full["hwp"])
    mh = full["m"].cpu().numpy()
    y_ref = opt.apply_pix(pix, c, s, mh)
    for P, tol in ((full["P64"], 1e-12), (full["P32"], 2e-6)):
        m = full["m"] if P.dtype == torch.float64 else full["m"].float()
        y = fx.pointing_apply(P, m)[list(ROWS)].double().cpu().numpy()
        assert rel_err(y, y_ref) <= tol


def test_full_quaternion_pcg_f32_within_1e6_of_f64(fx, full):
    w, N = full["w"], full["N"]
    D = dev()
    y = fx.pointing_apply(full["P32"], full["m"].float())
    d32 = y + synth.noise(w.with_(noise="diag"), device=D).float()
    x64, valid, i64, _ = fx.pcg_mapmake(full["P64"], N, d32.double(), max_iter=400, rtol=1e-10)
    x32, _, i32, _ = fx.pcg_mapmake(full["P32"], N, d32, max_iter=400, rtol=1e-8,
                                    valid_in=valid)
    err = rel_err(x32.cpu().numpy(), x64.cpu().numpy())
    print(f"quaternion full size: FP32 map vs FP64 map {err:.3e}; iterations "
          f"{i32.iters} / {i64.iters}")
    assert err <= 1e-6


def _axis_quat(axis, ang):
    """Rotation by ang about coordinate axis 0, 1 or 2, as (w, x, y, z) quaternions."""
    ang = np.asarray(ang, dtype=np.float64)
    q = np.zeros(ang.shape + (4,))
    q[..., 0] = np.cos(0.5 * ang)
    q[..., 1 + axis] = np.sin(0.5 * ang)
    return q


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 2e-5)])
def test_quaternion_normal_operator_with_many_chunk_groups(fx, dtype, tol):
    """Quaternion pointing on a raster over a ~5 degree patch at nside 1024: each
    superpixel holds dozens of chunks, which the superpixel P^T takes in groups
    (one partial per group); A x must still equal the oracle's."""
    nside, nd, ns, b = 1024, 48, 150_000, 33
    t = np.arange(ns, dtype=np.float64)
    th = 1.1 + np.deg2rad(2.5) * np.sin(2 * np.pi * t / 5003.0)
    ph = 2.3 + np.deg2rad(5.0) * ((t * 0.0113) % 1.0)
    roll = 0.37 * t
    # boresight R = Rz(phi) Ry(theta) Rz(roll): line of sight at (theta, phi)
    qb = oq.quat_mul(oq.quat_mul(_axis_quat(2, ph), _axis_quat(1, th)), _axis_quat(2, roll))
    rng = np.random.default_rng(5)
    qd = oq.quat_mul(_axis_quat(0, np.deg2rad(rng.uniform(-0.3, 0.3, nd))),
                     _axis_quat(1, np.deg2rad(rng.uniform(-0.3, 0.3, nd))))
    w = synth.WORKLOADS[2].with_(nside=nside, n_det=nd, n_samp=ns)
    lags = synth.toeplitz_lags(w, b)
    hwp = (w.hwp_num, w.hwp_den, 0.3)
    prob = omm.Problem(nside, None, None, None, "band", lags=lags, hwp=hwp,
                       bore_quat=qb, det_quat=qd)
    pix, c, s = prob.geometry()
    hit = np.unique(pix[pix >= 0])
    assert hit.size < 20_000 and pix.min() >= 0
    D = dev()
    P = fx.QuatPointing(nside, torch.from_numpy(qb).to(D), torch.from_numpy(qd).to(D), dtype,
                        None, None, hwp)
    N = fx.Noise("band", nd, ns, lags=torch.from_numpy(lags).to(D))
    x = np.zeros((3, 12 * nside * nside))
    x[:, hit] = np.random.default_rng(11).standard_normal((3, hit.size))
    got = fx.normal_apply(P, N, torch.from_numpy(x).to(D)).cpu().numpy()
    ref = omm.normal_apply(prob, pix, c, s, x)
    assert rel_err(got, ref) <= tol

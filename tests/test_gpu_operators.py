"""GPU parity: ang2pix, P, P^T, N^-1 and the normal operator against the FP64 oracle.

Tolerances: pixel indices and hit counts bit-exact; FP64 operators <= 1e-12
relative (norm-wise); FP32 operators <= 2e-6 relative (FP32 products and
FFT arithmetic, FP64 sums: a few FP32 roundings per sample)."""
import math

import numpy as np
import pytest
import torch

from oracle import healpix as ohp
from oracle import mapmaker as omm
from oracle import noise as onz
from oracle import pointing as opt
from paper_2603_19600_amd import synth
from tests.gpu_util import case, check_pixel_mismatches, dev, rel_err, to_pointing

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fx():
    from paper_2603_19600_amd import furax
    return furax


# ---------------------------------------------------------------- ang2pix
@pytest.mark.parametrize("nside", [1, 2, 3, 4, 64, 512, 1024])
def test_ang2pix_pixel_centres_bitexact(fx, nside):
    pix = np.arange(ohp.npix(nside))
    th, ph = ohp.pix2ang_ring(nside, pix)
    got = fx.ang2pix(nside, torch.from_numpy(th).to(dev()), torch.from_numpy(ph).to(dev()))
    assert np.array_equal(got.cpu().numpy(), pix)


@pytest.mark.parametrize("nside", [1, 7, 64, 1024, 8192])
def test_ang2pix_random_points_bitexact(fx, nside):
    th, ph = synth.uniform_sphere(nside, 2_000_000)
    ref = ohp.ang2pix_ring(nside, th.numpy(), ph.numpy())
    got = fx.ang2pix(nside, th.to(dev()), ph.to(dev())).cpu().numpy()
    # bit-exact except where a one-ulp cosine difference is resolved by mpmath
    check_pixel_mismatches(nside, th.numpy(), ph.numpy(), got, ref)


@pytest.mark.parametrize("nside", [4, 64, 1024])
def test_ang2pix_ring_boundaries_ulp_neighbourhood(fx, nside):
    """Directions within a few ulp of every ring boundary latitude, and phi
    within a few ulp of pixel-edge longitudes on the equatorial / polar split."""
    n = nside
    zs = [2.0 / 3.0, -2.0 / 3.0]
    zs += [1.0 - (i * i) / (3.0 * n * n) for i in range(1, n)]
    zs += [(2 * n - i) * 2.0 / (3.0 * n) for i in range(n, 3 * n + 1)]
    th0 = np.arccos(np.clip(np.array(zs), -1, 1))
    rng = np.random.default_rng(nside)
    th = np.concatenate([np.nextafter(th0, th0 + s) if s else th0 for s in (-1, 0, 1)]
                        + [th0 + k * np.spacing(th0) for k in (-3, -2, 2, 3)])
    th = np.clip(th, 0, math.pi)
    th = np.repeat(th, 16)
    ph = rng.uniform(0, 2 * math.pi, th.size)
    ph[::4] = np.round(ph[::4] / (math.pi / (2 * n))) * (math.pi / (2 * n))
    ref = ohp.ang2pix_ring(n, th, ph)
    got = fx.ang2pix(n, torch.from_numpy(th).to(dev()), torch.from_numpy(ph).to(dev()))
    # a mismatch is only acceptable where the device cosine differs by 1 ulp:
    # then z sits within 1 ulp of a boundary, and mpmath's correctly rounded
    # cosine decides between the two adjacent pixels
    check_pixel_mismatches(n, th, ph, got.cpu().numpy(), ref)


def test_ang2pix_f32_inputs_and_invalid(fx):
    th, ph = synth.uniform_sphere(3, 100_000)
    th32, ph32 = th.float(), ph.float()
    ref = ohp.ang2pix_ring(256, th32.double().numpy(), ph32.double().numpy())
    got = fx.ang2pix(256, th32.to(dev()), ph32.to(dev())).cpu().numpy()
    check_pixel_mismatches(256, th32.double().numpy(), ph32.double().numpy(), got, ref)
    bad_t = torch.tensor([-0.1, math.pi + 0.1, float("nan"), 0.3, 1.0, 0.0, math.pi],
                         dtype=torch.float64)
    bad_p = torch.tensor([0.0, 0.0, 0.0, float("nan"), float("inf"), 7.0, -7.0],
                         dtype=torch.float64)
    got = fx.ang2pix(16, bad_t.to(dev()), bad_p.to(dev())).cpu().numpy()
    assert np.array_equal(got, ohp.ang2pix_ring(16, bad_t.numpy(), bad_p.numpy()))
    assert np.all(got[:5] == -1)


@pytest.mark.parametrize("nside", [1, 4, 64, 1024, 8192])
def test_ang2pix_every_fp32_theta_matches_the_fp64_path(fx, nside):
    """Every FP32 theta in [0, pi] (all 1.08e9 of them, plus the FP32 value just
    above pi), each with a random FP32 phi: the pixel of the FP32 inputs equals
    the pixel of their exact FP64 promotion bit for bit (the FP32 path promotes
    before any arithmetic).  The FP64 path itself is pinned to the oracle by
    the tests above."""
    D = dev()
    hi = int(np.array([np.pi], dtype=np.float32).view(np.int32)[0])
    g = torch.Generator(device=D).manual_seed(nside)
    step = 1 << 27
    for a in range(0, hi + 1, step):
        b = min(a + step, hi + 1)
        th = torch.arange(a, b, dtype=torch.int32, device=D).view(torch.float32)
        ph = torch.rand(b - a, generator=g, device=D, dtype=torch.float32) * float(2 * np.pi)
        p32 = fx.ang2pix(nside, th, ph)
        p64 = fx.ang2pix(nside, th.double(), ph.double())
        bad = torch.nonzero(p32 != p64).flatten()
        assert bad.numel() == 0, (nside, th[bad[:4]].tolist(), ph[bad[:4]].tolist())


def test_ang2pix_empty(fx):
    e = torch.empty(0, dtype=torch.float64, device=dev())
    assert fx.ang2pix(8, e, e).numel() == 0


# ---------------------------------------------------------------- P and P^T
@pytest.mark.parametrize("nside,n_det,n_samp,hwp", [(16, 3, 5000, True), (64, 2, 3333, False),
                                                     (4, 1, 1, True), (512, 4, 70001, True)])
def test_pointing_apply_f64(fx, nside, n_det, n_samp, hwp):
    w, h, t = case(nside, n_det, n_samp, hwp=hwp, sphere=nside <= 16)
    P = to_pointing(nside, t)
    m = synth.sky_map(w.with_(nside=nside))
    ref = opt.pointing_apply(nside, h["theta"], h["phi"], h["psi"], m.numpy(), h["gain"],
                             h["dpsi"], h["hwp"])
    got = fx.pointing_apply(P, m.to(dev())).cpu().numpy()
    assert rel_err(got, ref) <= 1e-12
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_pointing_apply_f32(fx):
    w, h, t = case(64, 3, 20000, dtype="f32")
    P = to_pointing(64, t)
    m = synth.sky_map(w)
    ref = opt.pointing_apply(64, h["theta"], h["phi"], h["psi"], m.numpy(), h["gain"], h["dpsi"],
                             h["hwp"])
    got = fx.pointing_apply(P, m.to(dev())).cpu().numpy()
    assert rel_err(got, ref) <= 2e-6
    got32 = fx.pointing_apply(P, m.float().to(dev())).cpu().numpy()
    assert rel_err(got32, ref) <= 2e-6


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_constant_I_tod_bitwise(fx, dtype):
    w, h, t = case(32, 2, 7000, dtype=dtype, gains=False)
    P = to_pointing(32, t)
    m = torch.zeros(3, w.npix, dtype=torch.float64)
    m[0] = 1.6180339887498949 if dtype == "f64" else float(np.float32(1.618034))
    got = fx.pointing_apply(P, m.to(dev())).cpu().numpy()
    assert np.all(got == m[0, 0].item())


@pytest.mark.parametrize("nside,n_det,n_samp,dtype", [(16, 3, 5000, "f64"), (64, 2, 3333, "f64"),
                                                       (256, 5, 40000, "f64"),
                                                       (64, 3, 20000, "f32")])
def test_pointing_transpose(fx, nside, n_det, n_samp, dtype):
    w, h, t = case(nside, n_det, n_samp, dtype=dtype, sphere=nside <= 16)
    P = to_pointing(nside, t)
    d = synth.noise(w.with_(noise="diag"))
    dd = d.to(P.dtype)
    ref = opt.pointing_transpose(nside, h["theta"], h["phi"], h["psi"], dd.double().numpy(),
                                 h["gain"], h["dpsi"], h["hwp"])
    got = fx.pointing_transpose(P, dd.to(dev()).contiguous()).cpu().numpy()
    tol = 1e-12 if dtype == "f64" else 2e-6
    assert rel_err(got, ref) <= tol
    # accumulate = 1 adds on top
    base = torch.ones(3, w.npix, dtype=torch.float64, device=dev())
    acc = fx.pointing_transpose(P, dd.to(dev()).contiguous(), out=base, accumulate=True)
    assert rel_err(acc.cpu().numpy() - 1.0, ref) <= tol


def test_adjoint_identity_gpu(fx):
    w, h, t = case(128, 4, 50000)
    P = to_pointing(128, t)
    m = synth.sky_map(w).to(dev())
    d = synth.noise(w.with_(noise="diag")).to(dev())
    lhs = torch.sum(fx.pointing_apply(P, m) * d).item()
    rhs = torch.sum(m * fx.pointing_transpose(P, d)).item()
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_hits_bitexact_and_sum(fx):
    w, h, t = case(64, 3, 30000, dtype="f32")
    t["theta"][1, 100:150] = float("nan")
    h["theta"][1, 100:150] = np.nan
    P = to_pointing(64, t)
    N = fx.Noise("diag", 3, 30000, inv_var=torch.tensor([1.0, 2.0, 0.5], dtype=torch.float64, device=dev()))
    M6, hits = fx.bj_build(P, N)
    pix = opt.pixels(64, h["theta"], h["phi"])
    ref_hits = opt.hits(pix, w.npix)
    assert np.array_equal(hits.cpu().numpy(), ref_hits)
    assert hits.sum().item() == 3 * 30000 - 50
    c, s = opt.weights(h["psi"], h["dpsi"], h["hwp"])
    M_ref, _ = omm.bj_build(pix, c, s, np.array([1.0, 2.0, 0.5]), w.npix, h["gain"])
    assert rel_err(M6.cpu().numpy(), M_ref) <= 1e-6


# ---------------------------------------------------------------- N^-1
@pytest.mark.parametrize("n_samp,b", [(1, 1), (100, 1), (5000, 7), (40000, 129), (70001, 4096),
                                      (16384, 4096), (200_000, 1000), (50_001, 2500),
                                      (8194, 4096), (100_000, 8192), (60_001, 6000),
                                      (24_579, 4097), (5000, 4096), (9000, 8192),
                                      (40_003, 3072), (70_001, 3073), (26_625, 3500),
                                      (26_624, 3073), (26_625, 3073), (5000, 5000),
                                      (30_002, 2560), (30_002, 2561), (30_001, 2500),
                                      (30_001, 3000)])
def test_band_noise_f64(fx, n_samp, b):
    rng = np.random.default_rng(n_samp + b)
    y = rng.standard_normal((2, n_samp))
    t = synth.toeplitz_lags(synth.WORKLOADS[2], b)
    ref = onz.band_apply(y, t, "fft" if n_samp * b > 1 << 26 else "auto")
    N = fx.Noise("band", 2, n_samp, lags=torch.from_numpy(t).to(dev()))
    got = fx.noise_apply(N, torch.from_numpy(y).to(dev())).cpu().numpy()
    assert rel_err(got, ref) <= 1e-12


@pytest.mark.parametrize("n_samp,b", [(5000, 7), (70001, 4096), (100_000, 8192), (3, 2),
                                      (50_001, 2500), (5000, 4096), (9000, 8192), (40_000, 4097),
                                      (40_003, 3072), (70_001, 3073), (8192, 8192),
                                      (16_386, 8192), (16_387, 8192), (32_772, 8192)])
def test_band_noise_f32(fx, n_samp, b):
    rng = np.random.default_rng(n_samp + b)
    y = rng.standard_normal((3, n_samp)).astype(np.float32)
    t = synth.toeplitz_lags(synth.WORKLOADS[2], b)
    ref = onz.band_apply(y.astype(np.float64), t, "fft")
    N = fx.Noise("band", 3, n_samp, lags=torch.from_numpy(t).to(dev()))
    got = fx.noise_apply(N, torch.from_numpy(y).to(dev())).cpu().numpy()
    assert rel_err(got, ref) <= 2e-6


@pytest.mark.parametrize("dtype,b,wl,tol", [(np.float64, 4096, 2, 1e-12),
                                             (np.float32, 4096, 3, 2e-6),
                                             (np.float32, 8192, 5, 2e-6)])
def test_band_noise_full_stream(fx, dtype, b, wl, tol):
    """Whole 2^20-sample streams with the benchmark workloads' lags: the same
    kernel and launch shape per detector as the timed iteration."""
    n = synth.WORKLOADS[wl].n_samp
    rng = np.random.default_rng(b + wl)
    y = rng.standard_normal((3, n)).astype(dtype)
    t = synth.toeplitz_lags(synth.WORKLOADS[wl], b)
    ref = onz.band_apply(y.astype(np.float64), t, "fft")
    N = fx.Noise("band", 3, n, lags=torch.from_numpy(t).to(dev()))
    got = fx.noise_apply(N, torch.from_numpy(y).to(dev())).cpu().numpy()
    assert rel_err(got, ref) <= tol


@pytest.mark.parametrize("b", [2500, 3000, 4096, 6000, 8192])
@pytest.mark.parametrize("dtype,tol", [(np.float64, 1e-12), (np.float32, 2e-6)])
def test_band_noise_per_detector_long_kernels(fx, dtype, tol, b):
    """Per-detector lags wide enough for the register-resident blocks (8192-
    and 16384-point packed transforms), up to the widest band."""
    rng = np.random.default_rng(3)
    y = rng.standard_normal((3, 30001)).astype(dtype)
    base = synth.toeplitz_lags(synth.WORKLOADS[2], b)
    t = np.stack([base, 0.5 * base, 2.0 * base]) + 1e-3 * rng.standard_normal((3, b))
    t[:, 0] = np.abs(t[:, 0]) + 1.0
    ref = onz.band_apply(y.astype(np.float64), t, "fft")
    N = fx.Noise("band", 3, 30001, lags=torch.from_numpy(t).to(dev()))
    got = fx.noise_apply(N, torch.from_numpy(y).to(dev())).cpu().numpy()
    assert rel_err(got, ref) <= tol


@pytest.mark.parametrize("dtype,b,tol", [(np.float64, 4096, 1e-12), (np.float32, 4096, 2e-6),
                                          (np.float64, 2500, 1e-12), (np.float32, 8192, 2e-6)])
def test_band_noise_rows_off_16_byte_alignment(fx, dtype, b, tol):
    """Streams of even length whose data starts one element past an aligned
    address (a view into a larger buffer): the kernels' sample-pair accesses
    then sit at half-pair alignment and must give the same result."""
    n = 40_000
    rng = np.random.default_rng(b + 7)
    y = rng.standard_normal((2, n)).astype(dtype)
    t = synth.toeplitz_lags(synth.WORKLOADS[2], b)
    ref = onz.band_apply(y.astype(np.float64), t, "fft")
    buf = torch.zeros(2 * n + 1, dtype=torch.from_numpy(y).dtype, device=dev())
    yv = buf[1:].view(2, n)
    yv.copy_(torch.from_numpy(y).to(dev()))
    obuf = torch.zeros_like(buf)
    zv = obuf[1:].view(2, n)
    N = fx.Noise("band", 2, n, lags=torch.from_numpy(t).to(dev()))
    fx.noise_apply(N, yv, out=zv)
    assert rel_err(zv.cpu().numpy(), ref) <= tol
    assert float(obuf[0]) == 0.0


def test_band_noise_per_detector_kernels(fx):
    rng = np.random.default_rng(1)
    y = rng.standard_normal((3, 9000))
    t = rng.standard_normal((3, 33)) * np.array([[1.0], [0.5], [2.0]])
    ref = onz.band_apply(y, t)
    N = fx.Noise("band", 3, 9000, lags=torch.from_numpy(t).to(dev()))
    got = fx.noise_apply(N, torch.from_numpy(y).to(dev())).cpu().numpy()
    assert rel_err(got, ref) <= 1e-12


def test_diag_noise(fx):
    rng = np.random.default_rng(2)
    y = rng.standard_normal((4, 1234))
    w = np.array([1.0, 0.25, 3.0, 2.0])
    N = fx.Noise("diag", 4, 1234, inv_var=torch.from_numpy(w).to(dev()))
    got = fx.noise_apply(N, torch.from_numpy(y).to(dev())).cpu().numpy()
    assert np.array_equal(got, w[:, None] * y)


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 3e-6)])
def test_superpixel_paths_at_nside_1024(fx, dtype, tol):
    """Angle pointing at nside 1024: the superpixel P^T and block-Jacobi build
    use 1024-run chunks there (runs are shorter than at nside 512)."""
    nside, nd, ns, b = 1024, 3, 30011, 257
    w, h, t = case(nside, nd, ns, dtype=dtype)
    P = to_pointing(nside, t)
    lags = synth.toeplitz_lags(w, b)
    N = fx.Noise("band", nd, ns, lags=torch.from_numpy(lags).to(dev()))
    prob = omm.Problem(nside, h["theta"], h["phi"], h["psi"], "band", lags=lags,
                       gain=h["gain"], dpsi=h["dpsi"], hwp=h["hwp"])
    x = synth.sky_map(w)
    pix, c, s = prob.geometry()
    ref = omm.normal_apply(prob, pix, c, s, x.numpy())
    got = fx.normal_apply(P, N, x.to(dev())).cpu().numpy()
    assert rel_err(got, ref) <= tol
    M6, hits = fx.bj_build(P, N)
    M_ref, h_ref = omm.bj_build(pix, c, s, prob.wdiag(), prob.npix, prob.gain)
    assert np.array_equal(hits.cpu().numpy(), h_ref)
    assert rel_err(M6.cpu().numpy(), M_ref) <= (1e-12 if dtype == "f64" else 1e-6)


# ---------------------------------------------------------------- normal operator
@pytest.mark.parametrize("kind,dtype", [("diag", "f64"), ("band", "f64"), ("diag", "f32"),
                                        ("band", "f32")])
def test_normal_apply(fx, kind, dtype):
    nside, nd, ns, b = 64, 3, 30011, 257
    w, h, t = case(nside, nd, ns, dtype=dtype)
    P = to_pointing(nside, t)
    if kind == "diag":
        iv = np.array([1.0, 0.5, 2.0])
        N = fx.Noise("diag", nd, ns, inv_var=torch.from_numpy(iv).to(dev()))
        prob = omm.Problem(nside, h["theta"], h["phi"], h["psi"], "diag", inv_var=iv,
                           gain=h["gain"], dpsi=h["dpsi"], hwp=h["hwp"])
    else:
        lags = synth.toeplitz_lags(w, b)
        N = fx.Noise("band", nd, ns, lags=torch.from_numpy(lags).to(dev()))
        prob = omm.Problem(nside, h["theta"], h["phi"], h["psi"], "band", lags=lags,
                           gain=h["gain"], dpsi=h["dpsi"], hwp=h["hwp"])
    x = synth.sky_map(w)
    pix, c, s = prob.geometry()
    ref = omm.normal_apply(prob, pix, c, s, x.numpy())
    got = fx.normal_apply(P, N, x.to(dev())).cpu().numpy()
    assert rel_err(got, ref) <= (1e-12 if dtype == "f64" else 3e-6)
    # flagged pixels: a validity mask removes their samples from both P and P^T
    valid = np.ones(w.npix, dtype=np.uint8)
    valid[::3] = 0
    pixv = omm.flag_invalid(pix, valid.astype(bool))
    ref_v = omm.normal_apply(prob, pixv, c, s, x.numpy())
    got_v = fx.normal_apply(P, N, x.to(dev()), valid=torch.from_numpy(valid).to(dev()))
    assert rel_err(got_v.cpu().numpy(), ref_v) <= (1e-12 if dtype == "f64" else 3e-6)

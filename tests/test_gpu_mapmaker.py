"""GPU parity: block-Jacobi preconditioner, PCG map-maker and the chi-square
gradient against the FP64 oracle.

Tolerances: FP64 solved maps after identical iteration counts <= 1e-10
relative (Krylov recurrences amplify the 1e-16 reordering of sums);
FP32-path solved maps <= 1e-6 relative to the FP64 oracle."""
import math

import numpy as np
import pytest
import torch

from oracle import chi2 as och
from oracle import mapmaker as omm
from oracle import pointing as opt
from paper_2603_19600_amd import synth
from tests.gpu_util import case, dev, rel_err, to_pointing

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fx():
    from paper_2603_19600_amd import furax
    return furax


def _problem(fx, nside, nd, ns, kind, dtype="f64", b=65, seed=7, hwp=True, gains=True):
    w, h, t = case(nside, nd, ns, dtype=dtype, seed=seed, hwp=hwp, gains=gains)
    P = to_pointing(nside, t)
    if kind == "diag":
        iv = np.linspace(0.5, 2.0, nd)
        N = fx.Noise("diag", nd, ns, inv_var=torch.from_numpy(iv).to(dev()))
        prob = omm.Problem(nside, h["theta"], h["phi"], h["psi"], "diag", inv_var=iv,
                           gain=h["gain"], dpsi=h["dpsi"], hwp=h["hwp"])
    else:
        lags = synth.toeplitz_lags(w, b)
        N = fx.Noise("band", nd, ns, lags=torch.from_numpy(lags).to(dev()))
        prob = omm.Problem(nside, h["theta"], h["phi"], h["psi"], "band", lags=lags,
                           gain=h["gain"], dpsi=h["dpsi"], hwp=h["hwp"])
    return w, P, N, prob


def _tod(w, prob, P, with_signal=True):
    """d = P m_true + n, built with the ORACLE's P (never the HIP path)."""
    m = synth.sky_map(w).numpy()
    n = synth.noise(w.with_(noise="diag")).numpy()
    pix, c, s = prob.geometry()
    d = (opt.apply_pix(pix, c, s, m, prob.gain) if with_signal else 0.0) + n
    return d, m


def test_bj_invert_matches_oracle(fx):
    w, P, N, prob = _problem(fx, 32, 3, 20000, "diag")
    M6, hits = fx.bj_build(P, N)
    Minv, valid, rcond = fx.bj_invert(M6, hits, 1e-3, 3)
    pix, c, s = prob.geometry()
    M_ref, h_ref = omm.bj_build(pix, c, s, prob.wdiag(), prob.npix, prob.gain)
    inv_ref, v_ref, rc_ref = omm.bj_invert(M_ref, h_ref)
    assert np.array_equal(hits.cpu().numpy(), h_ref)
    assert rel_err(M6.cpu().numpy(), M_ref) <= 1e-12
    v = valid.cpu().numpy().astype(bool)
    near = np.abs(rc_ref - 1e-3) <= 1e-9
    assert np.all((v == v_ref) | near)
    both = v & v_ref
    assert rel_err(Minv.cpu().numpy()[:, both], inv_ref[:, both]) <= 1e-10


def test_pcg_diag_is_binned_after_one_iteration(fx):
    # the small workload: nside 64, 4 detectors at boresight, white noise
    w = synth.WORKLOADS[1].with_(n_samp=65536)
    pt = synth.pointing(w)
    iv = np.ones(w.n_det)
    D = dev()
    P = fx.Pointing(w.nside, pt.theta.to(D), pt.phi.to(D), pt.psi.to(D))
    N = fx.Noise("diag", w.n_det, w.n_samp, inv_var=torch.from_numpy(iv).to(D))
    prob = omm.Problem(w.nside, pt.theta.numpy(), pt.phi.numpy(), pt.psi.numpy(), "diag",
                       inv_var=iv)
    d, _ = _tod(w, prob, P)
    binned, v_ref = omm.binned_map(prob, d)
    x1, valid, info, st = fx.pcg_mapmake(P, N, torch.from_numpy(d).to(D), max_iter=1,
                                         valid_in=torch.from_numpy(v_ref.astype(np.uint8)).to(D))
    assert info.iters == 1 and st == fx.OK
    assert rel_err(x1.cpu().numpy(), binned) <= 1e-10
    assert info.resid_history[1] < 1e-10
    # 20 iterations (the workload's count) stay at the binned map
    x20, _, info20, _ = fx.pcg_mapmake(P, N, torch.from_numpy(d).to(D), max_iter=20,
                                       valid_in=torch.from_numpy(v_ref.astype(np.uint8)).to(D))
    assert rel_err(x20.cpu().numpy(), binned) <= 1e-9


@pytest.mark.parametrize("kind,iters", [("band", 25), ("diag", 3)])
def test_pcg_matches_oracle_f64(fx, kind, iters):
    w, P, N, prob = _problem(fx, 32, 4, 30000, kind, b=300)
    d, _ = _tod(w, prob, P)
    res = omm.pcg_mapmake(prob, d, max_iter=iters)
    x, valid, info, st = fx.pcg_mapmake(
        P, N, torch.from_numpy(d).to(dev()), max_iter=iters,
        valid_in=torch.from_numpy(res.valid.astype(np.uint8)).to(dev()))
    assert info.iters == res.iters
    assert np.array_equal(valid.cpu().numpy().astype(bool), res.valid)
    assert info.n_valid == int(res.valid.sum())
    assert rel_err(x.cpu().numpy(), res.x) <= 1e-10
    h_ref = np.array(res.resid_history)
    h_got = np.array(info.resid_history)
    # residuals at rounding level (after exact convergence) are noise on both sides
    live = h_ref > 1e-10
    assert np.allclose(h_got[live], h_ref[live], rtol=1e-8)
    assert np.all(h_got[~live] < 1e-10)


def test_pcg_own_mask_matches_oracle_mask(fx):
    w, P, N, prob = _problem(fx, 32, 3, 20000, "band", b=100)
    d, _ = _tod(w, prob, P)
    res = omm.pcg_mapmake(prob, d, max_iter=5)
    x, valid, info, _ = fx.pcg_mapmake(P, N, torch.from_numpy(d).to(dev()), max_iter=5)
    pix, c, s = prob.geometry()
    M, h = omm.bj_build(pix, c, s, prob.wdiag(), prob.npix, prob.gain)
    _, _, rc = omm.bj_invert(M, h)
    v = valid.cpu().numpy().astype(bool)
    assert np.all((v == res.valid) | (np.abs(rc - 1e-3) <= 1e-9))


def test_pcg_noiseless_exact_recovery_f64(fx):
    w, P, N, prob = _problem(fx, 16, 4, 40000, "band", b=200)
    pix, c, s = prob.geometry()
    M, h = omm.bj_build(pix, c, s, prob.wdiag(), prob.npix, prob.gain)
    _, valid, _ = omm.bj_invert(M, h)
    m = synth.sky_map(w).numpy()
    m[:, ~valid] = 0
    d = opt.apply_pix(omm.flag_invalid(pix, valid), c, s, m, prob.gain)
    x, _, info, st = fx.pcg_mapmake(P, N, torch.from_numpy(d).to(dev()), max_iter=200,
                                    rtol=1e-13)
    assert st == fx.OK and info.stop_reason == fx.STOP_RTOL
    assert rel_err(x.cpu().numpy(), m) <= 1e-10


def test_pcg_f32_path_within_1e6_of_f64_oracle(fx):
    w, P, N, prob = _problem(fx, 32, 4, 40000, "band", dtype="f32", b=400)
    d, _ = _tod(w, prob, P)
    d32 = d.astype(np.float32)
    res = omm.pcg_mapmake(prob, d32.astype(np.float64), max_iter=300, rtol=1e-12)
    x, valid, info, st = fx.pcg_mapmake(
        P, N, torch.from_numpy(d32).to(dev()), max_iter=300, rtol=1e-9,
        valid_in=torch.from_numpy(res.valid.astype(np.uint8)).to(dev()))
    err = rel_err(x.cpu().numpy(), res.x)
    per = [rel_err(x.cpu().numpy()[i], res.x[i]) for i in range(3)]
    print(f"FP32 path solved-map error vs FP64 oracle: {err:.3e} (I,Q,U: {per})")
    assert err <= 1e-6


def test_pcg_session_resume_equals_straight(fx):
    w, P, N, prob = _problem(fx, 32, 3, 20000, "band", b=100)
    d, _ = _tod(w, prob, P)
    dt = torch.from_numpy(d).to(dev())
    s1 = fx.PCGSession(P, N, dt, max_iter=10, no_early_exit=True)
    s1.iterate(5)
    s1.iterate(5)
    xa, _, ia, _ = s1.finish()
    s1.close()
    xb, _, ib, _ = fx.pcg_mapmake(P, N, dt, max_iter=10)
    assert ia.iters == ib.iters == 10
    assert rel_err(xa.cpu().numpy(), xb.cpu().numpy()) <= 1e-12


def test_pcg_breakdown_and_invalid_args(fx):
    w, P, N, prob = _problem(fx, 16, 2, 5000, "diag")
    d, _ = _tod(w, prob, P)
    d[0, 10] = np.nan
    x, _, info, st = fx.pcg_mapmake(P, N, torch.from_numpy(d).to(dev()), max_iter=5)
    assert st == fx.EBREAKDOWN and info.stop_reason == fx.STOP_BREAKDOWN and info.iters == 0
    assert torch.all(x == 0)
    bad = fx.Noise("band", 2, 5000, lags=torch.tensor([-1.0, 0.1], dtype=torch.float64,
                                                       device=dev()))
    d2, _ = _tod(w, prob, P)
    # a negative-definite kernel: no block passes the Cholesky validity test ...
    _, v0, info0, _ = fx.pcg_mapmake(P, bad, torch.from_numpy(d2).to(dev()), max_iter=5)
    assert info0.n_valid == 0 and int(v0.sum()) == 0
    # ... and with every pixel forced valid the first <r, z> is not positive
    allv = torch.ones(P.npix, dtype=torch.uint8, device=dev())
    _, _, info2, st2 = fx.pcg_mapmake(P, bad, torch.from_numpy(d2).to(dev()), max_iter=5,
                                      valid_in=allv)
    assert st2 == fx.EBREAKDOWN
    with pytest.raises(fx.FuraxError) as e:
        fx.pcg_mapmake(P, fx.Noise("diag", 3, 5000, inv_var=torch.ones(3, dtype=torch.float64,
                                                                         device=dev())),
                       torch.from_numpy(d2).to(dev()))
    assert e.value.status == fx.EINVAL
    too_wide = fx.Noise("band", 2, 9000, lags=torch.ones(8193, dtype=torch.float64, device=dev()))
    with pytest.raises(fx.FuraxError) as e:
        fx.noise_apply(too_wide, torch.zeros(2, 9000, dtype=torch.float64, device=dev()))
    assert e.value.status == fx.EUNSUPPORTED


# ---------------------------------------------------------------- chi2 and its VJP
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_chi2_and_vjp_match_oracle(fx, dtype):
    w, h, t = case(32, 4, 20000, dtype=dtype, hwp=False)
    P = to_pointing(32, t)
    iv = np.array([1.0, 0.5, 2.0, 1.5])
    N = fx.Noise("diag", 4, 20000, inv_var=torch.from_numpy(iv).to(dev()))
    m = synth.sky_map(w).numpy()
    d = synth.noise(w.with_(noise="diag")).numpy().astype(np.float32 if dtype == "f32" else
                                                          np.float64)
    val, gm, gg, gd = och.chi2_grad(32, h["theta"], h["phi"], h["psi"], d.astype(np.float64), m,
                                    h["gain"], h["dpsi"], "diag", inv_var=iv)
    c2, u = fx.chi2(P, N, torch.from_numpy(m).to(dev()), torch.from_numpy(d).to(dev()),
                    want_resid=True)
    tol = 1e-12 if dtype == "f64" else 3e-6
    assert abs(c2.item() - val) <= tol * abs(val)
    gmap, ggain, gdpsi = fx.pointing_vjp(P, torch.from_numpy(m).to(dev()), u)
    assert rel_err(-2 * gmap.cpu().numpy(), gm) <= tol
    assert rel_err(-2 * ggain.cpu().numpy(), gg) <= tol
    assert rel_err(-2 * gdpsi.cpu().numpy(), gd) <= (tol if dtype == "f64" else 1e-5)


def _patch_scan(n_det, n_samp, seed):
    """A raster over a ~5 degree patch at nside 1024 (the 1.8 degree 32 x 32
    superpixels crossed every ~30 samples): a dozen or so superpixels each
    hold tens of thousands of short runs -- dozens of chunks, and several
    chunk groups, per superpixel."""
    rng = np.random.default_rng(seed)
    t = np.arange(n_samp, dtype=np.float64)
    th0, ph0 = 1.1, 2.3
    dth = np.deg2rad(rng.uniform(-0.3, 0.3, n_det))[:, None]
    dph = np.deg2rad(rng.uniform(-0.3, 0.3, n_det))[:, None]
    theta = th0 + dth + np.deg2rad(2.5) * np.sin(2 * np.pi * t / 5003.0)[None, :]
    phi = ph0 + dph + np.deg2rad(5.0) * ((t * 0.0113) % 1.0)[None, :]
    psi = rng.uniform(-np.pi, np.pi, (n_det, n_samp))
    return theta, phi, psi


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_normal_apply_with_many_chunk_groups_per_superpixel(fx, dtype):
    """The superpixel P^T sums a superpixel's chunks in groups, one partial per
    group, and the reduction adds the groups: a dense patch scan puts dozens of
    chunks in each superpixel; A x must still equal the oracle's."""
    nside, nd, ns, b = 1024, 64, 150_000, 33
    theta, phi, psi = _patch_scan(nd, ns, 5)
    if dtype == "f32":
        theta, phi, psi = (a.astype(np.float32).astype(np.float64) for a in (theta, phi, psi))
    w = synth.WORKLOADS[2].with_(nside=nside, n_det=nd, n_samp=ns)
    lags = synth.toeplitz_lags(w, b)
    hwp = (w.hwp_num, w.hwp_den, 0.3)
    prob = omm.Problem(nside, theta, phi, psi, "band", lags=lags, hwp=hwp)
    pix, c, s = prob.geometry()
    npix = 12 * nside * nside
    hit = np.unique(pix[pix >= 0])
    # 9.6e6 samples on a patch of < 2e4 pixels (~20 superpixels' worth):
    # every superpixel holds thousands of runs of a few tens of samples
    assert hit.size < 20_000 and pix.min() >= 0
    D = dev()
    tt = torch.float32 if dtype == "f32" else torch.float64
    P = fx.Pointing(nside, torch.from_numpy(theta).to(D, tt).contiguous(),
                    torch.from_numpy(phi).to(D, tt).contiguous(),
                    torch.from_numpy(psi).to(D, tt).contiguous(), hwp=hwp)
    N = fx.Noise("band", nd, ns, lags=torch.from_numpy(lags).to(D))
    rng = np.random.default_rng(11)
    x = np.zeros((3, npix))
    x[:, hit] = rng.standard_normal((3, hit.size))
    got = fx.normal_apply(P, N, torch.from_numpy(x).to(D)).cpu().numpy()
    ref = omm.normal_apply(prob, pix, c, s, x)
    assert rel_err(got, ref) <= (1e-12 if dtype == "f64" else 2e-5)



@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("ns", [40000, 40001])
def test_normal_apply_long_band_with_invalid_pointing(fx, dtype, ns):
    """Above 3072 lags (2560 in FP64) N^-1 takes the transform of 32768-sample
    blocks; with samples that no superpixel run holds (invalid pointing) and
    on even and odd stream lengths (paired and single-value row accesses),
    A x must equal the oracle's."""
    nside, nd, b = 32, 3, 3500
    w, h, t = case(nside, nd, ns, dtype=dtype, seed=5)
    t["theta"][1, 100:150] = float("nan")
    h["theta"][1, 100:150] = np.nan
    P = to_pointing(nside, t)
    lags = synth.toeplitz_lags(w, b)
    N = fx.Noise("band", nd, ns, lags=torch.from_numpy(lags).to(dev()))
    prob = omm.Problem(nside, h["theta"], h["phi"], h["psi"], "band", lags=lags,
                       gain=h["gain"], dpsi=h["dpsi"], hwp=h["hwp"])
    pix, c, s = prob.geometry()
    assert (pix < 0).sum() == 50
    x = np.random.default_rng(3).standard_normal((3, 12 * nside * nside))
    got = fx.normal_apply(P, N, torch.from_numpy(x).to(dev())).cpu().numpy()
    ref = omm.normal_apply(prob, pix, c, s, x)
    assert rel_err(got, ref) <= (1e-12 if dtype == "f64" else 2e-5)

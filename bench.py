"""Benchmark: TOD samples/s per PCG iteration of P^T N^-1 P on one MI355X.

A step is one block-Jacobi PCG iteration of the map-maker: q = P^T N^-1 P p
(pointing expanded on the fly, overlap-save band-Toeplitz N^-1, scatter-add
P^T) plus the FP64 vector updates and dot products.  Inputs are synthetic,
seeded and resident in HBM before the timed region.

Default workload (the largest single-GPU one): HEALPix nside 1024, 1024
detectors x 2^20 samples (1.07e9 samples), 1/f noise weighted by a
band-Toeplitz of 8192 lags, ideal HWP at 2 Hz, 100 PCG iterations.  The
headline is the FP32 path (FP32 pointing, TOD and FFT arithmetic; FP64
binning, vectors, dot products and 3x3 inversion); the plain FP64 path of the
same workload is measured beside it, and the line reports the relative
difference of the two solved maps after the 100 iterations.  Also measured:
the same workload with boresight-quaternion pointing, with template
deprojection (the weight F_T of Eq. (3)) in place of N^-1, the chi-square
gradient of the differentiation workload (nside 256, 64 x 2^20 FP32), gap
filling, a device copy (the achievable bandwidth), and the FP64 oracle's
P^T N^-1 P on a 16-detector prefix of the workload on the host's cores.

The headline iterations are timed with HIP events around the timed steps
only; the per-phase times come from a separate pass of the same number of
iterations with the library's phase events on.

Prints one JSON line (rank 0).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "TOD samples/s per PCG iter of P^T N^-1 P (FP32 vs FP64) + % HBM peak"
HBM_PEAK_GBS = 8000.0
TARGET_FRAC = 0.60


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_inputs(w, dev, prec):
    """Pointing, noise model and data of workload w (FP32 canonical inputs) for
    the path of precision prec: the FP32 path reads the FP32 arrays, the FP64
    path their exact FP64 promotion, and both solve the same data (the FP32
    path's signal plus white noise)."""
    import torch

    from paper_2603_19600_amd import furax as fx
    from paper_2603_19600_amd import synth

    t0 = time.time()
    hwp = (w.hwp_num, w.hwp_den, 0.0) if w.hwp else None
    tdt = torch.float64 if prec == "f64" else torch.float32
    m_true = synth.sky_map(w, device=dev)
    if w.pointing == "quat":
        P = fx.QuatPointing(w.nside, synth.boresight_quaternions(w, device=dev),
                            synth.detector_quaternions(w, device=dev), torch.float32, hwp=hwp)
        d = fx.pointing_apply(P, m_true.float())
        if prec == "f64":
            P = P.with_(dtype=torch.float64)
    else:
        pt = synth.pointing(w, device=dev, det_chunk=8)          # canonical dtype of w
        P = fx.Pointing(w.nside, pt.theta, pt.phi, pt.psi, hwp=hwp)
        d = fx.pointing_apply(P, m_true.to(pt.theta.dtype))
        if prec != w.dtype:
            P = P.with_(theta=pt.theta.to(tdt), phi=pt.phi.to(tdt), psi=pt.psi.to(tdt))
        del pt
    if w.noise == "band":
        lags = torch.from_numpy(synth.toeplitz_lags(w)).to(dev)
        N = fx.Noise("band", w.n_det, w.n_samp, lags=lags)
    elif w.noise == "deproj":
        N = fx.Noise("deproj", w.n_det, w.n_samp,
                     inv_var=torch.full((w.n_det,), 1.0 / w.sigma ** 2, dtype=torch.float64,
                                        device=dev),
                     seg_len=w.tmpl_seg_len, order=w.tmpl_order)
    else:
        N = fx.Noise("diag", w.n_det, w.n_samp,
                     inv_var=torch.full((w.n_det,), 1.0 / w.sigma ** 2, dtype=torch.float64,
                                        device=dev))
    # white noise streams: the 1/f model enters through the band-Toeplitz
    # weights, and no operator's cost depends on the data values
    d = (d + synth.noise(w, device=dev, shape_1f=False).to(d.dtype)).to(tdt)
    torch.cuda.synchronize()
    log(f"{w.name} ({prec} path): inputs generated in {time.time() - t0:.1f} s")
    return P, N, d


def kernel_bytes(w):
    """Algorithmic HBM bytes per launch of each phase of one PCG iteration.

    P: the pointing stream once and the map read once (what the operator
    needs; its TOD output is the decomposition's intermediate, not counted).
    N^-1: its TOD in and out.  P^T: what it reads (the angle psi and the
    2-byte pixel offset of every sample, from the plan's run-sorted copies,
    and the weighted TOD) and the FP64 map written once."""
    e = 8 if w.dtype == "f64" else 4
    S = w.n_det * w.n_samp
    if w.pointing == "quat":
        pt_p, pt_t = 32 * (w.n_samp + w.n_det), 32 * (w.n_samp + w.n_det) + S * 2
    else:
        pt_p, pt_t = S * 3 * e, S * (e + 2)
    return {
        "apply": pt_p + 3 * w.npix * e,
        "noise": S * 2 * e,
        "transpose": pt_t + S * e + 3 * w.npix * 8,
    }


def operator_bytes(w):
    """B_alg of a whole PCG iteration: the pointing stream once plus the
    map-domain vectors (p, q, x, r, z and the preconditioner: ~52 FP64 values
    per pixel).  The TOD never has to reach HBM when P, N^-1 and P^T are fused."""
    e = 8 if w.dtype == "f64" else 4
    pt = w.n_det * w.n_samp * 3 * e if w.pointing != "quat" else 32 * (w.n_samp + w.n_det)
    return pt + 52 * 8 * w.npix


def traffic_file(w):
    tag = w.name.replace("^", "p").replace("_hwp", "").replace("_f32", "").replace("_f64", "")
    return os.path.join(ROOT, "profiles", f"traffic_{tag}.txt")


# kernels making up each phase, by rocprofv3 kernel name ({T}: double or float)
PHASE_KERNELS = {
    "apply": ["fx::k_apply<{T}, {T}, true, false>"],
    "noise": ["fx::k_os_r32x<{T}", "fx::k_os_r32<{T}", "fx::k_overlap_save<{T}, "],
    "transpose": ["fx::k_sp_accum<{T}, 0, false", "fx::k_sp_reduce"],
}


def source_fingerprint():
    """sha256 of the HIP sources and the C header (the counters go stale with them)."""
    import hashlib

    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2603_19600_amd", "csrc")
    for f in sorted(os.listdir(csrc)) + ["../../include/furax.h"]:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode())
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(w, phase):
    """HBM bytes per launch of a phase from the committed rocprofv3 record:
    FETCH_SIZE and WRITE_SIZE, each scaled by what it reads for the library's
    non-temporal device copy of known size (the cache policy of the kernels'
    streams).  None when the record is missing, the kernels changed since it
    was taken, or the read counter falls below the bytes the phase must read
    (then it is not measuring them)."""
    try:
        with open(traffic_file(w)) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != source_fingerprint():
        return None
    cal = rec["calibration"]["nontemporal"]
    cb = rec["calibration"]["bytes"]
    sf, sw = cb / (cal["FETCH_SIZE"] * 1024.0), cb / (cal["WRITE_SIZE"] * 1024.0)
    T = "double" if w.dtype == "f64" else "float"
    rd, wr, found = 0.0, 0.0, 0
    for pat in PHASE_KERNELS[phase]:
        pat = pat.format(T=T)
        for name, v in rec["kernels"].items():
            if name.startswith(pat):
                rd += v["FETCH_SIZE"] * 1024.0 * sf
                wr += v["WRITE_SIZE"] * 1024.0 * sw
                found += 1
    if not found:
        return None
    e = 8 if w.dtype == "f64" else 4
    S = w.n_det * w.n_samp
    must_read = {"apply": S * 3 * e, "noise": S * e, "transpose": S * (2 * e + 2)}[phase]
    if rd < 0.98 * must_read:
        return None            # the read counter does not see all of the stream's requests
    return {"read": rd, "write": wr, "total": rd + wr, "must_read": must_read}


def run_pcg(fx, P, N, d, steps, warmup, iters):
    """warmup iterations, `steps` timed with no phase events, `steps` more with
    the phase events on, then the rest up to `iters`; returns the timed ms per
    iteration, the phase sums, the final map and the session's info."""
    import torch

    total = max(iters, warmup + 2 * steps)
    sess = fx.PCGSession(P, N, d, max_iter=total, rtol=0.0, no_early_exit=True)
    sess.iterate(warmup)
    torch.cuda.synchronize()
    # the library launches on torch's current stream, where these events go too
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    sess.iterate(steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    sess.set_timing(True)
    sess.read_timing()
    sess.iterate(steps)
    phases = sess.read_timing()
    sess.set_timing(False)
    rest = total - warmup - 2 * steps
    if rest > 0:
        sess.iterate(rest)
    x, valid, info, st = sess.finish()
    sess.close()
    return ms, phases, x, valid, info


def measure(w, dev, steps, warmup, prec, keep_map=False):
    import torch

    from paper_2603_19600_amd import furax as fx

    P, N, d = make_inputs(w, dev, prec)
    w = w.with_(dtype=prec)
    ms, phases, x, valid, info = run_pcg(fx, P, N, d, steps, warmup, w.iters)
    S = w.n_det * w.n_samp
    res = {"workload": w.name.replace("_f32", "_" + prec), "ms_per_step": ms, "value": S / (ms * 1e-3), "iters": info.iters,
           "rel_resid": info.rel_resid, "n_valid": info.n_valid}
    kb = kernel_bytes(w)
    n = max(phases["iters"], 1)
    res["kernels"] = {}
    for k in ("apply", "noise", "transpose", "update"):
        t = phases[k] / n
        row = {"ms": t}
        if k in kb and t > 0:
            row["alg_bytes"] = kb[k]
            row["GB_s"] = kb[k] / (t * 1e-3) / 1e9
            row["frac"] = row["GB_s"] / HBM_PEAK_GBS
        res["kernels"][k] = row
    ob = operator_bytes(w)
    res["operator"] = {"alg_bytes_per_iter": ob, "B_alg_per_sample": ob / S,
                       "GB_s": ob / (ms * 1e-3) / 1e9,
                       "frac_hbm_peak": ob / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                       "target_frac": TARGET_FRAC}
    log(f"{res['workload']}: {ms:.3f} ms/iter, {res['value']:.4g} samples/s; after {info.iters} "
        f"iterations rel resid {info.rel_resid:.3e}")
    log("phases: " + ", ".join(f"{k} {v['ms']:.3f} ms" + (f" {v['GB_s']:.0f} GB/s" if "GB_s" in v else "")
                               for k, v in res["kernels"].items()))
    del P, N, d
    if not keep_map:
        del x, valid
        x = None
    torch.cuda.empty_cache()
    return res, x


def measure_copy(dev, gib=4):
    """Device copy of `gib` GiB by the library's stream copy, plain and
    non-temporal: read + write GB/s, the achievable-bandwidth ceiling."""
    import torch

    from paper_2603_19600_amd import furax as fx

    nb = gib << 30
    src = torch.ones(nb // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    out = {"bytes_copied": nb}
    for name, nt in (("plain", False), ("nontemporal", True)):
        fx.stream_copy(src, dst, nt)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 5
        e0.record()
        for _ in range(reps):
            fx.stream_copy(src, dst, nt)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[name] = {"ms": ms, "GB_s": 2 * nb / (ms * 1e-3) / 1e9,
                     "frac": 2 * nb / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    assert torch.equal(src[:1024], dst[:1024])
    del src, dst
    torch.cuda.empty_cache()
    log(f"device copy: plain {out['plain']['GB_s']:.0f} GB/s, non-temporal "
        f"{out['nontemporal']['GB_s']:.0f} GB/s (read + write)")
    return out


def measure_chi2(w, dev, steps=5):
    """The differentiation workload: chi2 forward (furax_chi2) plus the gradient
    with respect to the map, the gains and the angle offsets (furax_chi2_grad,
    pointing recomputed), through the torch.autograd.Function; samples/s of one
    forward + backward and each pass's algorithmic GB/s (pointing and data
    read once per pass, the map read, the FP64 map gradient written)."""
    import torch

    from paper_2603_19600_amd import furax as fx
    from paper_2603_19600_amd import synth

    pt = synth.pointing(w, device=dev, det_chunk=8)
    P = fx.Pointing(w.nside, pt.theta, pt.phi, pt.psi)
    iv = torch.full((w.n_det,), 1.0 / w.sigma ** 2, dtype=torch.float64, device=dev)
    N = fx.Noise("diag", w.n_det, w.n_samp, inv_var=iv)
    m_true = synth.sky_map(w, device=dev)
    d = (fx.pointing_apply(P, m_true).double() + synth.noise(w, device=dev)).float()
    m = (m_true + 0.1).requires_grad_(True)
    g = torch.ones(w.n_det, dtype=torch.float64, device=dev, requires_grad=True)
    dp = torch.zeros(w.n_det, dtype=torch.float64, device=dev, requires_grad=True)

    def step():
        m.grad = g.grad = dp.grad = None
        fx.chi2_loss(P, N, d, m, g, dp).backward()

    step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    # the two passes alone
    tf = _time(lambda: fx.chi2(P, N, m.detach(), d), steps)
    tb = _time(lambda: fx.chi2_grad(P, N, m.detach(), d), steps)
    S = w.n_det * w.n_samp
    fwd_bytes = S * (3 * 4 + 4) + 3 * w.npix * 8
    bwd_bytes = S * (3 * 4 + 4) + 3 * w.npix * 8 * 2
    res = {"workload": w.name, "ms_fwd_bwd": ms, "samples_per_s": S / (ms * 1e-3),
           "ms_forward": tf, "ms_gradient": tb,
           "forward": {"alg_bytes": fwd_bytes, "GB_s": fwd_bytes / (tf * 1e-3) / 1e9,
                       "frac": fwd_bytes / (tf * 1e-3) / 1e9 / HBM_PEAK_GBS},
           "gradient": {"alg_bytes": bwd_bytes, "GB_s": bwd_bytes / (tb * 1e-3) / 1e9,
                        "frac": bwd_bytes / (tb * 1e-3) / 1e9 / HBM_PEAK_GBS}}
    log(f"chi2 {w.name}: forward + gradient {ms:.3f} ms ({res['samples_per_s']:.4g} samples/s); "
        f"forward {tf:.3f} ms, gradient {tb:.3f} ms")
    del P, N, d, m, pt
    torch.cuda.empty_cache()
    return res


def _time(fn, reps):
    import torch

    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def measure_gapfill(w, dev, frac=0.01, rtol=1e-10):
    """Constrained-realisation gap filling of the workload's streams (1 % of the
    samples missing in gaps of 1-399 samples, band-Toeplitz covariance of the
    workload's bandwidth): wall time of the whole call (CG to rtol on every
    detector, set-up and output), its CG iterations, and samples/s per CG
    iteration."""
    import numpy as np
    import torch

    from paper_2603_19600_amd import furax as fx
    from paper_2603_19600_amd import synth

    C = fx.Noise("band", w.n_det, w.n_samp,
                 lags=torch.from_numpy(synth.covariance_lags(w)).to(dev))
    d = synth.noise(w, device=dev, shape_1f=True)
    nr = synth.noise(w.with_(seed=w.seed + 1), device=dev, shape_1f=True)
    gaps = torch.from_numpy(synth.gap_mask(w, frac=frac).astype(np.uint8)).to(dev)
    fx.gap_fill(C, gaps, d, nr, max_iter=2, rtol=0.0)       # warm-up (plans, caches)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out, iters, rel, st = fx.gap_fill(C, gaps, d, nr, max_iter=500, rtol=rtol)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    S = w.n_det * w.n_samp
    log(f"gap fill: {iters} CG iterations in {dt * 1e3:.1f} ms ({dt * 1e3 / max(iters, 1):.3f} ms "
        f"per iteration), worst |r|/|b| {rel:.2e}")
    res = {"workload": w.name.replace(f"band{w.bandwidth}", f"gapfill{w.bandwidth}"),
           "missing_fraction": float(gaps.double().mean()), "cg_iters": iters,
           "rel_resid": rel, "ms_total": dt * 1e3, "ms_per_cg_iter": dt * 1e3 / max(iters, 1),
           "samples_per_s_per_cg_iter": S / (dt / max(iters, 1))}
    del C, d, nr, gaps, out
    torch.cuda.empty_cache()
    return res


# ---------------------------------------------------------------------------
# CPU baseline: the FP64 oracle's P^T N^-1 P on a detector prefix.
# ---------------------------------------------------------------------------
def _oracle_inputs(cfg, k0, k1):
    """The oracle's problem for detectors [k0, k1) of workload cfg, and the map."""
    from oracle import mapmaker as omm
    from paper_2603_19600_amd import synth

    w = synth.WORKLOADS[cfg]
    pt = synth.pointing(w, det0=k0, n_det=k1 - k0)
    hwp = (w.hwp_num, w.hwp_den, 0.0) if w.hwp else None
    prob = omm.Problem(w.nside, pt.theta.double().numpy(), pt.phi.double().numpy(),
                       pt.psi.double().numpy(), "band", lags=synth.toeplitz_lags(w), hwp=hwp)
    return prob, synth.sky_map(w).numpy()


def _oracle_apply(prob, x):
    """One application of A x = sum_k P_k^T N_k^-1 P_k x by the oracle, the
    pointing expanded first (as at every application); returns the touched
    pixels and their three Stokes sums."""
    import numpy as np

    from oracle import mapmaker as omm

    pix, c, s = prob.geometry()
    q = omm.normal_apply(prob, pix, c, s, x)
    nz = np.flatnonzero(np.any(q != 0.0, axis=0))
    return nz, q[:, nz]


def _oracle_worker(cfg, k0, k1, ready, go, out):
    from threadpoolctl import threadpool_limits

    with threadpool_limits(limits=1):
        prob, x = _oracle_inputs(cfg, k0, k1)
        ready.put(k0)
        go.wait()
        out.put(_oracle_apply(prob, x))


def cpu_baseline(cfg, n_det, workers):
    """The FP64 NumPy oracle's P^T N^-1 P on an n_det-detector prefix of the
    workload: on one host core, and over `workers` processes each applying it
    to its own shard of the detectors (the paper's decomposition
    sum_k P_k^T N_k^-1 P_k), summed here.  Inputs are generated before the
    timed regions."""
    import multiprocessing as mp

    import numpy as np
    from threadpoolctl import threadpool_limits

    from paper_2603_19600_amd import synth

    w = synth.WORKLOADS[cfg]
    S = n_det * w.n_samp
    with threadpool_limits(limits=1):
        prob, x = _oracle_inputs(cfg, 0, n_det)
        t0 = time.perf_counter()
        c0 = time.process_time()
        nz1, q1 = _oracle_apply(prob, x)
        one = time.perf_counter() - t0
        cpu1 = time.process_time() - c0
    del prob
    bounds = np.linspace(0, n_det, workers + 1).round().astype(int)
    shards = [(int(a), int(b)) for a, b in zip(bounds[:-1], bounds[1:]) if b > a]
    ctx = mp.get_context("spawn")
    ready, out, go = ctx.Queue(), ctx.Queue(), ctx.Event()
    procs = [ctx.Process(target=_oracle_worker, args=(cfg, a, b, ready, go, out), daemon=True)
             for a, b in shards]
    for p in procs:
        p.start()
    for _ in procs:
        ready.get(timeout=600)
    t0 = time.perf_counter()
    go.set()
    q = np.zeros((3, w.npix))
    for _ in procs:
        nz, vals = out.get(timeout=600)
        q[:, nz] += vals
    many = time.perf_counter() - t0
    for p in procs:
        p.join(timeout=60)
    ref = np.zeros_like(q)
    ref[:, nz1] = q1
    agree = float(np.abs(q - ref).max() / max(np.abs(ref).max(), 1e-300))
    log(f"cpu baseline: {n_det} detectors, 1 core {S / one:.4g} samples/s ({one:.1f} s); "
        f"{len(shards)} processes {S / many:.4g} samples/s ({many:.1f} s); shards vs whole "
        f"{agree:.1e}")
    return {"value": S / many, "unit": "samples/s", "cores": len(shards), "kind": "oracle",
            "sample": f"one application of P^T N^-1 P by the FP64 NumPy oracle (pointing "
                      f"expanded, single-FFT band-Toeplitz, bincount binning) on the first "
                      f"{n_det} detectors x {w.n_samp} samples of {w.name}, split by detector "
                      f"over {len(shards)} worker processes (one thread each) and summed; "
                      f"{many:.1f} s wall",
            "seconds": many,
            "one_core": {"value": S / one, "cores": 1, "seconds": one, "cpu_seconds": cpu1},
            "shards_vs_whole_max_rel": agree}


def host_info():
    info = {"nproc": os.cpu_count(), "machine": platform.machine()}
    try:
        info["affinity"] = len(os.sched_getaffinity(0))
    except Exception:
        pass
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True).stdout
        for ln in out.splitlines():
            if ln.startswith("Model name"):
                info["cpu"] = ln.split(":", 1)[1].strip()
    except Exception:
        pass
    for k in ("OMP_NUM_THREADS", "MKL_NUM_THREADS", "OPENBLAS_NUM_THREADS"):
        if k in os.environ:
            info[k] = os.environ[k]
    return info


# ---------------------------------------------------------------------------
# Profile records (run on the rocprofv3 output of this script; nothing below
# is used by the measurement itself).
# ---------------------------------------------------------------------------
def _rocpd_dbs(d):
    import glob

    return sorted(glob.glob(os.path.join(d, "**", "*.db"), recursive=True))


def _short_kernel(name):
    import re

    return re.sub(r"\(.*", "", name).replace("void ", "")


def summarize_trace(db_dir, out, command, title):
    """Markdown table of a rocprofv3 --kernel-trace run: per-kernel calls and
    durations with the launch resources, the library's kernels only."""
    import sqlite3

    rows = []
    for db in _rocpd_dbs(db_dir):
        con = sqlite3.connect(db)
        rows += list(con.execute(
            "select name, count(*), avg(duration), sum(duration), min(duration), max(duration), "
            "max(vgpr_count), max(accum_vgpr_count), max(sgpr_count), max(lds_size), "
            "max(scratch_size), max(workgroup_x), max(grid_x) from kernels group by name"))
    rows = sorted((r for r in rows if "fx::" in r[0]), key=lambda r: -r[3])
    lines = [f"# {title}", "", "Command (run from the repository root on one MI355X):", "",
             "```", command, "```", "", "Durations in microseconds (rocprofv3 kernel trace).", "",
             "| kernel | calls | avg us | total us | min us | max us | VGPR | AGPR | SGPR | LDS B "
             "| scratch B | wg | grid |", "|---|---|---|---|---|---|---|---|---|---|---|---|---|"]
    for r in rows:
        lines.append(f"| `{_short_kernel(r[0])}` | {r[1]} | {r[2] / 1000:.1f} | {r[3] / 1000:.1f} | "
                     f"{r[4] / 1000:.1f} | {r[5] / 1000:.1f} | {r[6]} | {r[7]} | {r[8]} | {r[9]} | "
                     f"{r[10]} | {r[11]} | {r[12]} |")
    lines += _marker_summary(db_dir)
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def _marker_summary(db_dir):
    """Host-side roctx ranges (P, N^-1, P^T, pcg_iteration, pcg_update) of a
    run taken with --marker-trace: count and mean duration per range.  The
    database records each range as a region of the roctx API with its
    message in the region's extdata (JSON)."""
    import sqlite3

    wanted = ("pcg_iteration", "P", "N^-1", "P^T", "pcg_update")
    agg = {}
    for db in _rocpd_dbs(db_dir):
        con = sqlite3.connect(db)
        try:
            rows = list(con.execute(
                "select extdata, \"end\" - start from regions where name like 'roctx%'"))
        except sqlite3.Error:
            continue
        for ext, dur in rows:
            try:
                name = json.loads(ext or "{}").get("message")
            except ValueError:
                continue
            if name in wanted:
                a = agg.setdefault(name, [0, 0.0])
                a[0] += 1
                a[1] += dur
    if not agg:
        return []
    out = ["", "Host-side roctx ranges (time to enqueue each phase on the host thread, not GPU "
           "time):", "", "| range | count | mean us |", "|---|---|---|"]
    for name in wanted:
        if name in agg:
            n, tot = agg[name]
            out.append(f"| `{name}` | {n} | {tot / max(n, 1) / 1000:.1f} |")
    return out


def traffic_record(dirs, out, commands):
    """The traffic record measured_traffic() reads, from rocprofv3 --pmc runs of
    this script (one counter group per run: FETCH_SIZE; WRITE_SIZE; optionally
    the request-size counters TCC_EA0_RDREQ_32B/64B/128B): the mean per
    dispatch of every counter of every library kernel, the same counters of
    the two 1 GiB calibration copies (the first dispatch of each kind), and
    the fingerprint of the sources they were taken on."""
    import collections
    import sqlite3

    vals = collections.defaultdict(lambda: collections.defaultdict(list))
    calib = {"plain": {}, "nontemporal": {}}
    for d in dirs:
        for db in _rocpd_dbs(d):
            con = sqlite3.connect(db)
            first = {}
            for name, cname, v, disp in con.execute(
                    "select kernel_name, counter_name, value, dispatch_id from counters_collection "
                    "order by dispatch_id"):
                if "k_stream_copy" in name:
                    kind = "nontemporal" if "<true>" in name else "plain"
                    first.setdefault(kind, disp)
                    if disp == first[kind]:
                        calib[kind][cname] = v
                elif "fx::" in name:
                    vals[_short_kernel(name)][cname].append(v)
    rec = {"calibration": {"bytes": 1 << 30, **calib}, "commands": commands,
           "source_sha256": source_fingerprint(), "kernels": {}}
    for k, d in vals.items():
        rec["kernels"][k] = {c: sum(v) / len(v) for c, v in d.items()}
        rec["kernels"][k]["dispatches"] = max(len(v) for v in d.values())
    with open(out, "w") as fh:
        json.dump(rec, fh, indent=1, sort_keys=True)


def calibration_copies(dev):
    """One plain and one non-temporal 1 GiB copy (2^30 bytes read, 2^30
    written) by the library's stream copy: the dispatches of known traffic
    that the profiler's counters are scaled by."""
    import torch

    from paper_2603_19600_amd import furax as fx

    src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    fx.stream_copy(src, dst, False)
    fx.stream_copy(src, dst, True)
    torch.cuda.synchronize()
    del src, dst
    torch.cuda.empty_cache()


def counter_summary(dirs, out, commands, title):
    """Markdown table of rocprofv3 --pmc runs: per library kernel, dispatches,
    mean duration and the mean of each counter per dispatch; with
    SQ_INSTS_VALU, the VALU busy fraction (a wave64 VALU instruction occupies
    a 16-lane SIMD for 4 cycles; 1024 SIMDs at 2.4 GHz)."""
    import collections
    import sqlite3

    rows = collections.defaultdict(lambda: collections.defaultdict(list))
    for d in dirs:
        for db in _rocpd_dbs(d):
            con = sqlite3.connect(db)
            for name, cname, v, dur in con.execute(
                    "select kernel_name, counter_name, value, duration from counters_collection"):
                if "fx::" in name:
                    r = rows[_short_kernel(name)]
                    r[cname].append(v)
                    r["_dur"].append(dur / 1000.0)
    cnames = sorted({c for r in rows.values() for c in r if c != "_dur"})
    busy = "SQ_INSTS_VALU" in cnames
    head = ["kernel", "dispatches", "mean us"] + cnames + (["VALU busy"] if busy else [])
    lines = [f"# {title}", "", "Commands (run from the repository root on one MI355X, one "
             "counter group per run):", "", "```"] + commands + ["```", "",
             "Counter values are means per dispatch over the profiled run (set-up and "
             "iterations); FETCH_SIZE / WRITE_SIZE in KiB.", "",
             "| " + " | ".join(head) + " |", "|" + "---|" * len(head)]
    for k in sorted(rows, key=lambda k: -sum(rows[k]["_dur"])):
        r = rows[k]
        dur = sum(r["_dur"]) / len(r["_dur"])
        cells = [f"`{k}`", str(max(len(v) for c, v in r.items() if c != "_dur")), f"{dur:.1f}"]
        for c in cnames:
            cells.append(f"{sum(r[c]) / len(r[c]):.4g}" if r.get(c) else "")
        if busy:
            v = r.get("SQ_INSTS_VALU")
            cells.append(f"{100 * (sum(v) / len(v)) * 4 / (1024 * 2400.0) / dur:.0f} %" if v else "")
        lines.append("| " + " | ".join(cells) + " |")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=5,
                    help="workload number: 5 (default, nside 1024) or 3 (nside 512); the FP32 "
                         "path is the headline and the FP64 path runs beside it")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 path")
    ap.add_argument("--no-quat", action="store_true",
                    help="skip the boresight-quaternion pointing variant")
    ap.add_argument("--no-deproj", action="store_true",
                    help="skip the template-deprojection variant")
    ap.add_argument("--no-chi2", action="store_true", help="skip the chi-square gradient")
    ap.add_argument("--no-gapfill", action="store_true",
                    help="skip the gap-filling measurement")
    ap.add_argument("--no-copy", action="store_true", help="skip the device-copy ceiling")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--iters", type=int, default=0,
                    help="PCG iterations per solve (0: the workload's own count); profiling "
                         "runs shorten the solves with it")
    ap.add_argument("--cpu-dets", type=int, default=64)
    ap.add_argument("--cpu-workers", type=int, default=16,
                    help="worker processes of the CPU baseline (capped by the host's CPUs)")
    ap.add_argument("--summarize-trace", metavar="DIR",
                    help="write the kernel-trace summary of a rocprofv3 output directory to --out")
    ap.add_argument("--traffic-record", nargs="+", metavar="DIR",
                    help="write the traffic record of rocprofv3 --pmc runs (FETCH_SIZE, "
                         "WRITE_SIZE, ...) to --out")
    ap.add_argument("--counter-summary", nargs="+", metavar="DIR",
                    help="write the per-kernel counter table of rocprofv3 --pmc outputs to --out")
    ap.add_argument("--calibrate", action="store_true",
                    help="only run the 1 GiB device copies the traffic counters are scaled by")
    ap.add_argument("--out")
    ap.add_argument("--command", action="append", default=[],
                    help="the profiling command(s) to record in the summary")
    ap.add_argument("--title", default="rocprofv3 kernel summary")
    args = ap.parse_args()
    if args.summarize_trace:
        summarize_trace(args.summarize_trace, args.out, "\n".join(args.command), args.title)
        return
    if args.counter_summary:
        counter_summary(args.counter_summary, args.out, args.command, args.title)
        return
    if args.traffic_record:
        traffic_record(args.traffic_record, args.out, args.command)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the map-making path runs on a single MI355X "
              "(sharding the detectors over several GPUs is described, not implemented).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2603_19600_amd import synth

    dev = torch.device("cuda:0")
    calibration_copies(dev)
    if args.calibrate:
        return
    w = synth.WORKLOADS[args.config]
    if args.iters > 0:
        w = w.with_(iters=args.iters)
    if w.dtype != "f32" or w.noise != "band":
        raise SystemExit("--config must name an FP32 band-noise workload (3 or 5)")
    primary, x32 = measure(w, dev, args.steps, args.warmup, "f32", keep_map=not args.no_fp64)
    fp64 = None
    map_err = None
    if not args.no_fp64:
        fp64, x64 = measure(w, dev, args.steps, args.warmup, "f64", keep_map=True)
        # both paths ran the workload's iterations from the same data; the FP64
        # path is pinned to the oracle by the parity tests
        num = float(torch.linalg.vector_norm(x32 - x64))
        den = float(torch.linalg.vector_norm(x64))
        per = [float(torch.linalg.vector_norm(x32[i] - x64[i]) / torch.linalg.vector_norm(x64[i]))
               for i in range(3)]
        map_err = {"rel": num / den, "I": per[0], "Q": per[1], "U": per[2],
                   "iterations": primary["iters"],
                   "rel_resid_f32": primary["rel_resid"], "rel_resid_f64": fp64["rel_resid"]}
        log(f"solved maps after {primary['iters']} iterations: FP32 vs FP64 {num / den:.3e} "
            f"(I {per[0]:.2e}, Q {per[1]:.2e}, U {per[2]:.2e})")
        del x32, x64
        torch.cuda.empty_cache()

    variants = {}
    if not args.no_quat:
        r, _ = measure(w.with_(pointing="quat", name=w.name + "_quat"), dev, args.steps,
                       args.warmup, "f32")
        variants["quat"] = {k: r[k] for k in ("workload", "value", "ms_per_step", "kernels",
                                              "operator")}
    if not args.no_deproj:
        wd = w.with_(noise="deproj", name=w.name.replace(
            f"band{w.bandwidth}", f"deproj{w.tmpl_seg_len}o{w.tmpl_order}"))
        r, _ = measure(wd, dev, args.steps, args.warmup, "f32")
        variants["deproj"] = {k: r[k] for k in ("workload", "value", "ms_per_step", "kernels",
                                                "operator")}
    chi2 = None if args.no_chi2 else measure_chi2(synth.WORKLOADS[4], dev)
    gapfill = None if args.no_gapfill else measure_gapfill(synth.WORKLOADS[2], dev)
    copy = None if args.no_copy else measure_copy(dev)

    # the dominant kernel of the headline iteration
    name, k = max(((n, v) for n, v in primary["kernels"].items() if "alg_bytes" in v),
                  key=lambda kv: kv[1]["ms"])
    traffic = measured_traffic(w, name)
    roofline = {"bound": "hbm", "kernel": name, "achieved": k["GB_s"], "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": k["GB_s"] / HBM_PEAK_GBS,
                "traffic": None if traffic is None else traffic["total"],
                "traffic_read_write": traffic,
                "alg_bytes_per_launch": k["alg_bytes"], "ms_per_launch": k["ms"],
                "iteration_frac": primary["operator"]["frac_hbm_peak"],
                "iteration_target_frac": TARGET_FRAC}
    if copy is not None:
        roofline["copy_ceiling_GB_s"] = copy["nontemporal"]["GB_s"]

    cpu = None
    if not args.no_cpu_baseline:
        try:
            ncpu = len(os.sched_getaffinity(0))
        except Exception:
            ncpu = os.cpu_count() or 1
        cpu = cpu_baseline(args.config, args.cpu_dets, max(1, min(args.cpu_workers, ncpu)))

    S = w.n_det * w.n_samp
    line = {
        "metric": METRIC,
        "value": primary["value"],
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": primary["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded spin+precession scan, random IQU sky, white noise data, "
                "1/f band-Toeplitz weights)",
        "config": {"workload": w.name, "nside": w.nside, "n_det": w.n_det, "n_samp": w.n_samp,
                   "samples": S, "noise": w.noise, "bandwidth": w.bandwidth, "hwp": w.hwp,
                   "pcg_iterations": w.iters, "pcg_precision": "f32 operator, f64 vectors/dots",
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernels": primary["kernels"],
        "operator": primary["operator"],
        "rel_resid": primary["rel_resid"],
        "fp64": None if fp64 is None else {
            "workload": fp64["workload"], "value": fp64["value"],
            "ms_per_step": fp64["ms_per_step"], "kernels": fp64["kernels"],
            "operator": fp64["operator"], "rel_resid": fp64["rel_resid"],
            "fp32_speedup": primary["value"] / fp64["value"]},
        "map_error_fp32_vs_fp64": map_err,
        "variants": variants or None,
        "chi2_grad": chi2,
        "gapfill": gapfill,
        "copy": copy,
        "host": host_info(),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

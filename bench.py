"""Benchmark: TOD samples/s per PCG iteration of P^T N^-1 P on one MI355X.

A step is one block-Jacobi PCG iteration of the map-maker: q = P^T N^-1 P p
(pointing expanded on the fly, overlap-save band-Toeplitz N^-1, scatter-add
P^T) plus the FP64 vector updates and dot products.  Inputs are synthetic,
seeded and resident in HBM before the timed region.

Default workload: HEALPix nside 512, 256 detectors x 2^20 samples, FP64
pointing/TOD, 1/f noise weighted by a band-Toeplitz of 4096 lags, ideal HWP at
2 Hz.  The FP32 variant of the same workload (FP32 pointing, TOD and FFT,
FP64 accumulation, dots and preconditioner) is measured beside it, and both
again with boresight-quaternion pointing (the same scan given as one attitude
per time sample and one per detector, expanded per sample in the kernels).

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


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_inputs(w, dev):
    import torch

    from paper_2603_19600_amd import furax as fx
    from paper_2603_19600_amd import synth

    t0 = time.time()
    hwp = (w.hwp_num, w.hwp_den, 0.0) if w.hwp else None
    if w.pointing == "quat":
        P = fx.QuatPointing(w.nside, synth.boresight_quaternions(w, device=dev),
                            synth.detector_quaternions(w, device=dev),
                            torch.float64 if w.dtype == "f64" else torch.float32, hwp=hwp)
    else:
        pt = synth.pointing(w, device=dev, det_chunk=8)
        P = fx.Pointing(w.nside, pt.theta, pt.phi, pt.psi, hwp=hwp)
    if w.noise == "band":
        lags = torch.from_numpy(synth.toeplitz_lags(w)).to(dev)
        N = fx.Noise("band", w.n_det, w.n_samp, lags=lags)
    else:
        N = fx.Noise("diag", w.n_det, w.n_samp,
                     inv_var=torch.full((w.n_det,), 1.0 / w.sigma ** 2, dtype=torch.float64,
                                        device=dev))
    m_true = synth.sky_map(w, device=dev)
    d = fx.pointing_apply(P, m_true)                       # signal (HIP path; bench only)
    # white noise streams: the 1/f model enters through the band-Toeplitz
    # weights, and no operator's cost depends on the data values (this also
    # keeps library FFTs, which the counter profiler cannot follow, out of it)
    d += synth.noise(w, device=dev, shape_1f=False).to(d.dtype)
    torch.cuda.synchronize()
    log(f"{w.name}: inputs generated in {time.time() - t0:.1f} s")
    return P, N, d


def kernel_bytes(w):
    """Algorithmic HBM bytes per launch of each phase of one PCG iteration (what
    the operator must move as the method defines it, whatever the kernel reads)."""
    e = 8 if w.dtype == "f64" else 4
    S = w.n_det * w.n_samp
    # pointing stream per phase: theta, phi, psi planes, or (quaternion
    # pointing) one boresight attitude per time sample and one per detector
    pt = S * 3 * e if w.pointing != "quat" else 32 * (w.n_samp + w.n_det)
    return {
        # P: pointing in, TOD out, the map read once
        "apply": pt + S * e + 3 * w.npix * e,
        # N^-1: TOD in, TOD out
        "noise": S * 2 * e,
        # P^T: pointing and TOD in, the FP64 map written once
        "transpose": pt + S * e + 3 * w.npix * 8,
    }


def operator_bytes(w):
    """Algorithmic bytes of a whole PCG iteration: the pointing stream once plus
    the map-domain vectors (p, q, x, r, z, preconditioner: ~52 FP64 per pixel).
    The TOD itself never has to reach HBM when P, N^-1 and P^T are fused."""
    e = 8 if w.dtype == "f64" else 4
    pt = w.n_det * w.n_samp * 3 * e if w.pointing != "quat" else 32 * (w.n_samp + w.n_det)
    return pt + 52 * 8 * w.npix


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_nside512_256x2p20_band4096.txt")
# kernels making up each phase, by rocprofv3 kernel name ({T}: double or float)
PHASE_KERNELS = {
    "apply": ["fx::k_apply<{T}, {T}, true, false>"],
    "noise": ["fx::k_overlap_save<{T}, "],
    "transpose": ["fx::k_sp_accum<{T}, 0, false>", "fx::k_sp_reduce"],
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


def measured_traffic(phase, dtype):
    """HBM bytes per launch of a phase from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE record, each counter scaled by what it reads for a plain 1 GiB
    device copy; None when the record is missing or the kernels changed since."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != source_fingerprint():
        return None
    cal = rec["calibration_kib"]
    cb = rec["calibration_copy_bytes"]
    sf, sw = cb / (cal["FETCH_SIZE"] * 1024.0), cb / (cal["WRITE_SIZE"] * 1024.0)
    T = "double" if dtype == "f64" else "float"
    total, found = 0.0, 0
    for pat in PHASE_KERNELS[phase]:
        pat = pat.format(T=T)
        for name, v in rec["kernels"].items():
            if name.startswith(pat):
                total += v["FETCH_SIZE"] * 1024.0 * sf + v["WRITE_SIZE"] * 1024.0 * sw
                found += 1
    return total if found else None


def run_pcg(fx, P, N, d, steps, warmup):
    import torch

    sess = fx.PCGSession(P, N, d, max_iter=steps + warmup, rtol=0.0, no_early_exit=True)
    sess.iterate(warmup)
    torch.cuda.synchronize()
    sess.set_timing(True)
    sess.read_timing()
    # the library launches on torch's current stream, where these events go too
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    sess.iterate(steps)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    phases = sess.read_timing()
    x, valid, info, st = sess.finish()
    sess.close()
    ms = e0.elapsed_time(e1) / steps
    return ms, wall, info, phases


def measure(w, dev, steps, warmup):
    import torch

    from paper_2603_19600_amd import furax as fx

    P, N, d = make_inputs(w, dev)
    ms, wall, info, phases = run_pcg(fx, P, N, d, steps, warmup)
    S = w.n_det * w.n_samp
    res = {"ms_per_step": ms, "value": S / (ms * 1e-3), "wall_s": wall, "iters": info.iters,
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
        res["kernels"][k] = row
    ob = operator_bytes(w)
    res["operator"] = {"alg_bytes_per_iter": ob, "B_alg_per_sample": ob / S,
                       "GB_s": ob / (ms * 1e-3) / 1e9, "frac_hbm_peak": ob / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    log(f"{w.name}: {ms:.3f} ms/iter, {res['value']:.4g} samples/s, rel resid {info.rel_resid:.3e}")
    log("phases: " + ", ".join(f"{k} {v['ms']:.3f} ms" + (f" {v['GB_s']:.0f} GB/s" if "GB_s" in v else "")
                               for k, v in res["kernels"].items()))
    del P, N, d
    torch.cuda.empty_cache()
    return res


def cpu_baseline(w, n_det):
    """The FP64 NumPy oracle's P^T N^-1 P on a detector prefix of the same workload,
    on one host core (BLAS/OpenMP pools limited to one thread)."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import mapmaker as omm
    from paper_2603_19600_amd import synth

    pt = synth.pointing(w, n_det=n_det)
    lags = synth.toeplitz_lags(w) if w.noise == "band" else None
    hwp = (w.hwp_num, w.hwp_den, 0.0) if w.hwp else None
    prob = omm.Problem(w.nside, pt.theta.double().numpy(), pt.phi.double().numpy(),
                       pt.psi.double().numpy(), w.noise,
                       inv_var=None if lags is not None else np.ones(n_det), lags=lags, hwp=hwp)
    x = synth.sky_map(w).numpy()
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        c0 = time.process_time()
        pix, c, s = prob.geometry()           # pointing is expanded at every application
        omm.normal_apply(prob, pix, c, s, x)
        cpu = time.process_time() - c0
        dt = time.perf_counter() - t0
    S = n_det * w.n_samp
    return {"value": S / dt, "unit": "samples/s", "cores": 1, "kind": "oracle",
            "sample": f"one application of P^T N^-1 P (FP64 NumPy oracle, pointing expanded, "
                      f"FFT band-Toeplitz) on a {n_det}-detector x {w.n_samp}-sample prefix of "
                      f"the workload, {dt:.1f} s wall, {cpu:.1f} s CPU",
            "seconds": dt}


def host_info():
    info = {"nproc": os.cpu_count(), "machine": platform.machine()}
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=2, help="workload number (2, 3 or 5)")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32 variant")
    ap.add_argument("--no-quat", action="store_true",
                    help="skip the boresight-quaternion pointing variants")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-dets", type=int, default=64)
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the map-making path is built and measured on a single "
              "MI355X (multi-GPU sharding by detector is a design note, not part of this build).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2603_19600_amd import synth

    dev = torch.device("cuda:0")
    # a plain 1 GiB device copy: the reference that scales rocprofv3's
    # FETCH_SIZE / WRITE_SIZE counters to bytes (it reads and writes 1 GiB)
    src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    w = synth.WORKLOADS[args.config]
    primary = measure(w, dev, args.steps, args.warmup)
    fp32 = None
    if not args.no_fp32 and w.dtype == "f64":
        w32 = synth.WORKLOADS[3] if args.config == 2 else w.with_(dtype="f32")
        fp32 = measure(w32, dev, args.steps, args.warmup)

    quat = {}
    if not args.no_quat:
        for wq in ([w] + ([synth.WORKLOADS[3]] if fp32 is not None and args.config == 2 else [])):
            r = measure(wq.with_(pointing="quat"), dev, args.steps, args.warmup)
            quat[wq.dtype] = {"workload": wq.name + "_quat", "value": r["value"],
                              "ms_per_step": r["ms_per_step"], "kernels": r["kernels"],
                              "operator": r["operator"]}

    # the dominant operator kernel of the iteration
    name, k = max(((n, v) for n, v in primary["kernels"].items() if "alg_bytes" in v),
                  key=lambda kv: kv[1]["ms"])
    traffic = measured_traffic(name, w.dtype)
    roofline = {"bound": "hbm", "kernel": name, "achieved": k["GB_s"], "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": k["GB_s"] / HBM_PEAK_GBS, "traffic": traffic,
                "alg_bytes_per_launch": k["alg_bytes"], "ms_per_launch": k["ms"]}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w, args.cpu_dets)
        log(f"cpu baseline: {cpu['value']:.4g} samples/s ({cpu['seconds']:.1f} s)")

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
        "dtype": w.dtype,
        "data": "synthetic (seeded spin+precession scan, random IQU sky, white noise data, 1/f band-Toeplitz weights)",
        "config": {"workload": w.name, "nside": w.nside, "n_det": w.n_det, "n_samp": w.n_samp,
                   "samples": S, "noise": w.noise, "bandwidth": w.bandwidth, "hwp": w.hwp,
                   "pcg_precision": w.dtype, "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernels": primary["kernels"],
        "operator": primary["operator"],
        "fp32": None if fp32 is None else {
            "workload": synth.WORKLOADS[3].name if args.config == 2 else w.name + "_f32",
            "value": fp32["value"], "ms_per_step": fp32["ms_per_step"],
            "kernels": fp32["kernels"], "operator": fp32["operator"],
            "speedup_vs_fp64": fp32["value"] / primary["value"]},
        "quat": quat or None,
        "host": host_info(),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

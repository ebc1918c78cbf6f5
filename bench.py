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
per time sample and one per detector, expanded per sample in the kernels) and
with template deprojection (the weight F_T of Eq. (3): white weights with
Legendre baselines of degree 0..3 removed from every 4096-sample segment) in
place of the band-Toeplitz N^-1.  An FP32 workload (--config 5: nside 1024,
1024 detectors x 2^20 samples, 8192 lags) is measured beside its FP64
counterpart.

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
    elif w.noise == "deproj":
        N = fx.Noise("deproj", w.n_det, w.n_samp,
                     inv_var=torch.full((w.n_det,), 1.0 / w.sigma ** 2, dtype=torch.float64,
                                        device=dev),
                     seg_len=w.tmpl_seg_len, order=w.tmpl_order)
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
    "noise": ["fx::k_os_r32x<{T}>", "fx::k_os_r32<{T}>", "fx::k_overlap_save<{T}, "],
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
    return {"workload": w.name.replace(f"band{w.bandwidth}", f"gapfill{w.bandwidth}"),
            "missing_fraction": float(gaps.double().mean()), "cg_iters": iters,
            "rel_resid": rel, "ms_total": dt * 1e3, "ms_per_cg_iter": dt * 1e3 / max(iters, 1),
            "samples_per_s_per_cg_iter": S / (dt / max(iters, 1))}


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
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def traffic_record(fetch_dir, write_dir, out, commands):
    """The FETCH_SIZE / WRITE_SIZE record measured_traffic() reads: KiB per
    dispatch of every library kernel, the 1 GiB calibration copy's counts, and
    the fingerprint of the sources they were taken on."""
    import collections
    import sqlite3

    vals = collections.defaultdict(lambda: collections.defaultdict(list))
    calib = {}
    for d in (fetch_dir, write_dir):
        for db in _rocpd_dbs(d):
            con = sqlite3.connect(db)
            for name, cname, v, grid in con.execute(
                    "select kernel_name, counter_name, value, grid_size from counters_collection "
                    "order by dispatch_id"):
                if "copy" in name and grid == (1 << 26) and cname not in calib:
                    calib[cname] = v
                if "fx::" in name:
                    vals[_short_kernel(name)][cname].append(v)
    rec = {"calibration_copy_bytes": 1 << 30, "calibration_kib": calib, "commands": commands,
           "source_sha256": source_fingerprint(), "kernels": {}}
    for k, d in vals.items():
        rec["kernels"][k] = {c: sum(v) / len(v) for c, v in d.items()}
        rec["kernels"][k]["dispatches"] = len(d.get("FETCH_SIZE", []))
    with open(out, "w") as fh:
        json.dump(rec, fh, indent=1, sort_keys=True)


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
    ap.add_argument("--config", type=int, default=2, help="workload number (2, 3 or 5)")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32 variant")
    ap.add_argument("--no-fp64", action="store_true",
                    help="skip the FP64 variant of an FP32 workload")
    ap.add_argument("--no-quat", action="store_true",
                    help="skip the boresight-quaternion pointing variants")
    ap.add_argument("--no-deproj", action="store_true",
                    help="skip the template-deprojection variants")
    ap.add_argument("--no-gapfill", action="store_true",
                    help="skip the gap-filling measurement")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-dets", type=int, default=64)
    ap.add_argument("--summarize-trace", metavar="DIR",
                    help="write the kernel-trace summary of a rocprofv3 output directory to --out")
    ap.add_argument("--traffic-record", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write the FETCH_SIZE / WRITE_SIZE record of two rocprofv3 --pmc runs "
                         "to --out")
    ap.add_argument("--counter-summary", nargs="+", metavar="DIR",
                    help="write the per-kernel counter table of rocprofv3 --pmc outputs to --out")
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
        traffic_record(args.traffic_record[0], args.traffic_record[1], args.out, args.command)
        return

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
    fp64 = None
    if not args.no_fp64 and w.dtype == "f32" and args.config != 3:
        w64 = w.with_(dtype="f64", name=w.name.replace("_f32", "_f64"))
        fp64 = measure(w64, dev, args.steps, args.warmup)

    quat = {}
    if not args.no_quat:
        for wq in ([w] + ([synth.WORKLOADS[3]] if fp32 is not None and args.config == 2 else [])):
            r = measure(wq.with_(pointing="quat"), dev, args.steps, args.warmup)
            quat[wq.dtype] = {"workload": wq.name + "_quat", "value": r["value"],
                              "ms_per_step": r["ms_per_step"], "kernels": r["kernels"],
                              "operator": r["operator"]}

    deproj = {}
    if not args.no_deproj:
        for wd in ([w] + ([synth.WORKLOADS[3]] if fp32 is not None and args.config == 2 else [])):
            r = measure(wd.with_(noise="deproj"), dev, args.steps, args.warmup)
            deproj[wd.dtype] = {"workload": wd.name.replace(f"band{wd.bandwidth}",
                                                            f"deproj{wd.tmpl_seg_len}o{wd.tmpl_order}"),
                                "value": r["value"], "ms_per_step": r["ms_per_step"],
                                "kernels": r["kernels"], "operator": r["operator"]}

    gapfill = None
    if not args.no_gapfill and w.dtype == "f64" and w.bandwidth <= 4096:
        gapfill = measure_gapfill(w, dev)

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
        "fp64": None if fp64 is None else {
            "workload": w64.name,
            "value": fp64["value"], "ms_per_step": fp64["ms_per_step"],
            "kernels": fp64["kernels"], "operator": fp64["operator"],
            "fp32_speedup": primary["value"] / fp64["value"]},
        "quat": quat or None,
        "deproj": deproj or None,
        "gapfill": gapfill,
        "host": host_info(),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

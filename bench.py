"""Throughput of the per-pixel 3x3 Hermitian inverse + determinant on one MI355X.

Workload (the step): an 8192x8192 synthetic PolSAR image, N=3 looks (the
fewest for full rank), every pixel with its own covariance Sigma whose
eigenvalues are log-uniform in [1e-8, 1] (condition numbers up to ~1e8;
about a fifth of the pixels fail the FP32 error bound and are recomputed in
FP64), seed 2; FP32 planes (36 B in, 40 B out per pixel).  One step = one
polsar_inv_det call over the whole image with the adjugate method,
compensated FP32 arithmetic and FP64 recompute of flagged pixels, in the
library's default launch, data resident in HBM.

Beside it (unless --no-rows): every other inverse form on the same image and
on an 8192x8192 image of the 4096x4096 recipe, default and autotuned, with
the adjugate-over-Cholesky ratios; the 4096x4096 image (N=4, 4x4 regions,
eigenvalues in [1e-3, 1], seed 1) with all forms, a plane copy of the same
byte count (its launch swept: the measured bandwidth ceiling), the Wishart
forward+backward, the fused multilook front ends, the nonlocal-means filter
and the out-of-core streamer.  Then (unless --no-workloads) the 2048x2048
Wishart image, the 64-image batch (default and autotuned launch) and the
paper's Table 2 shapes.  The CPU oracle is timed on the host.  Prints one
JSON line.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-rows] [--no-workloads]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

PEAK_HBM_GBS = 8000.0
SETTLE_S = 0.3
WORKLOAD = {"workload": "polsar-8192x8192-N3-per-pixel-sigma-lam1e-8", "height": 8192, "width": 8192,
            "n_looks": 3, "sigma": "per pixel, eigenvalues log-uniform in [1e-8, 1]", "seed": 2,
            "method": "adjugate", "precision": "fp32-compensated+fp64-reroute", "planes": "SoA 9 in, 9+1 out",
            "launch": "library default (table op 6: images of >= 2^25 pixels)"}
SCALE_WORKLOAD = {"workload": "polsar-4096x4096-N4-16regions-lam1e-3", "height": 4096, "width": 4096,
                  "n_looks": 4, "regions": "4x4", "lam_range": [1e-3, 1.0], "seed": 1}
BYTES_PER_PX = {"f32": 76, "f64": 152}         # 9 planes in + 9 inverse planes + det
WISHART_BYTES_PER_PX = {"f32": 108, "f64": 216}  # fused fwd+bwd: S, Z in (72) + grad out (36)


# the sources the inverse kernel (the step) is compiled from
STEP_SOURCES = ("common.hpp", "pixel.hpp", "polsar.hip")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(HERE, "paper_1807_08084_amd", "csrc")
    for name in STEP_SOURCES:
        h.update(open(os.path.join(csrc, name), "rb").read())
    return h.hexdigest()[:16]


TRAFFIC_RECORD = "hbm_traffic_inv_det_8192_precision.txt"


def traffic_from_profiles(kernel: str, n_px: int):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current kernel sources over an image of n_px pixels; else
    None."""
    path = os.path.join(HERE, "profiles", TRAFFIC_RECORD)
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            rec[k.strip()] = v.strip()
    if rec.get("source_hash") != kernel_source_hash() or rec.get("kernel") != kernel:
        return None
    if rec.get("pixels") != str(n_px):
        return None
    try:
        return float(rec["bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def warm(fn, warmup: int, torch, min_seconds: float = 0.0) -> int:
    """At least `warmup` untimed calls, continued until `min_seconds` of wall
    time have passed (the GPU leaves its idle clocks); returns the count."""
    t0 = time.perf_counter()
    done = 0
    while done < warmup or time.perf_counter() - t0 < min_seconds:
        for _ in range(max(1, warmup)):
            fn()
        done += max(1, warmup)
        torch.cuda.synchronize()
    return done


def time_calls(fn, steps: int, warmup: int, torch, min_warm_seconds: float = 0.0):
    warm(fn, warmup, torch, min_warm_seconds)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps  # ms per call


def launch_spread(fn, n: int, torch) -> dict:
    """n single launches, each between its own pair of events: min, median,
    mean, max and standard deviation in ms."""
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
    for a, b in evs:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    per = np.array([a.elapsed_time(b) for a, b in evs])
    return {"n": int(per.size), "min": round(float(per.min()), 4), "median": round(float(np.median(per)), 4),
            "mean": round(float(per.mean()), 4), "max": round(float(per.max()), 4),
            "std": round(float(per.std()), 4)}


# Table 2 of the paper (ms over 1000 replicates on a GeForce 940M, OpenCL,
# precision not stated): context for the paper-shaped rows, not a target.
PAPER_TABLE2_MS = {
    "simulated_5469354": {"adjugate": {"min": 223.06, "mean": 231.51, "max": 273.08, "std": 6.11},
                          "cholesky": {"min": 498.89, "mean": 507.54, "max": 556.79, "std": 9.34}},
    "airsar_450x600": {"adjugate": {"min": 11.18, "mean": 12.98, "max": 28.59, "std": 1.44},
                       "cholesky": {"min": 24.68, "mean": 28.35, "max": 62.60, "std": 2.55}},
}


def cpu_baseline(z64: np.ndarray, n_px: int, min_seconds: float = 10.0):
    import oracle
    threads = oracle.threads()
    oracle.ge(z64[:, :1024], nthreads=threads)  # load + warm
    t0 = time.perf_counter()
    passes = 0
    while True:
        oracle.ge(z64, nthreads=threads)
        passes += 1
        el = time.perf_counter() - t0
        if el >= min_seconds or passes >= 1000:
            break
    # the same oracle on one core, over the first 2^20 pixels, for about 4 s
    m = min(n_px, 1 << 20)
    sub = np.ascontiguousarray(z64[:, :m])
    t1 = time.perf_counter()
    passes1 = 0
    while True:
        oracle.ge(sub, nthreads=1)
        passes1 += 1
        el1 = time.perf_counter() - t1
        if el1 >= 4.0 or passes1 >= 1000:
            break
    # the other oracle forms beside it, about 2 s each: the FP64 Cholesky form
    # over the whole image, the __float128 elimination on a 2^16-pixel sample
    def rate(fn, px):
        t, k = time.perf_counter(), 0
        while True:
            fn()
            k += 1
            e = time.perf_counter() - t
            if e >= 2.0 or k >= 1000:
                return k * px / e / 1e9, k, e
    chol_rate, chol_k, chol_e = rate(lambda: oracle.chol(z64, nthreads=threads), n_px)
    q = min(n_px, 1 << 16)
    sub128 = np.ascontiguousarray(z64[:, :q])
    q_rate, q_k, q_e = rate(lambda: oracle.ge128(sub128, nthreads=threads), q)
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), model)
    except OSError:
        pass
    return {"value": passes * n_px / el / 1e9, "unit": "Gpixel/s", "cores": threads, "kind": "oracle",
            "sample": f"FP64 Gaussian-elimination oracle (OpenMP, {threads} threads) over the whole "
                      f"{n_px}-pixel image, {passes} passes, {el:.1f} s",
            "value_1core": passes1 * m / el1 / 1e9,
            "sample_1core": f"same oracle, 1 thread, first {m} pixels, {passes1} passes, {el1:.1f} s",
            "value_cholesky_f64": chol_rate,
            "sample_cholesky_f64": f"FP64 Cholesky oracle, {threads} threads, whole image, {chol_k} passes, "
                                   f"{chol_e:.1f} s",
            "value_ge_float128": q_rate,
            "sample_ge_float128": f"__float128 Gaussian-elimination oracle, {threads} threads, first {q} "
                                  f"pixels, {q_k} passes, {q_e:.1f} s",
            "cpu_model": model}


def rate_row(n: int, ms: float, bpp: float | None, **extra) -> dict:
    """Gpx/s and, for rows whose working set exceeds the caches, HBM GB/s
    and the fraction of the 8 TB/s peak."""
    r = {"gpx_s": round(n / ms / 1e6, 3), "ms": round(ms, 4)}
    if bpp is not None:
        gbs = bpp * n / (ms * 1e-3) / 1e9
        r.update({"GB_s": round(gbs, 1), "frac_hbm": round(gbs / PEAK_HBM_GBS, 4)})
    r.update(extra)
    return r


F32_FORMS = [("adjugate", "compensated"), ("adjugate", "plain"), ("adjugate", "wide"),
             ("cholesky", "plain"), ("cholesky", "compensated"), ("cholesky", "wide")]
F64_FORMS = [("adjugate", "compensated"), ("adjugate", "plain"), ("cholesky", "plain")]
TUNED_F32_FORMS = [("adjugate", "compensated"), ("cholesky", "compensated"), ("cholesky", "wide")]


COPY_SHAPES = ((64, 16, 5), (64, 16, 4), (64, 16, 6), (64, 8, 8), (128, 16, 3), (128, 8, 0), (128, 8, 6),
               (256, 16, 2), (256, 8, 0), (256, 16, 0))


def copy_ceiling(torch, ops, src, dst, n_in: int, n_out: int, n: int, steps: int):
    """Best time of the plane-copy probe (n_in planes in, n_out out, no
    arithmetic) over a sweep of launch shapes (block, access width,
    resident-block cap): the practical streaming ceiling of that mix of
    plane streams.  Returns (ms, launch)."""
    dt = src.dtype
    keep = ops.get_launch(4, dt, "adjugate", "plain")
    best = None
    for cb, cvb, cbpc in COPY_SHAPES:
        cfg = dict(block=cb, unroll=1, grid_per_cu=0, nontemporal=1, vector_bytes=cvb, blocks_per_cu=cbpc)
        ops.set_launch(4, dt, "adjugate", "plain", cfg)
        ms = time_calls(lambda: ops.stream_copy(src, dst, n_in, n_out, n), steps, 2, torch)
        if best is None or ms < best[0]:
            best = (ms, cfg)
    ops.set_launch(4, dt, "adjugate", "plain", keep)
    return best


def inverse_forms(torch, ops, dev, planes64: np.ndarray, steps: int, tag: str, tune: bool,
                  z32=None) -> dict:
    """Every inverse form on one image, FP32 and FP64, at the library's default
    launch for that size; with tune, the FP32 forms the equal-accuracy
    comparison uses again after the autotuner has installed its pick for this
    size (the default is restored afterwards)."""
    rows = {}
    n = planes64.shape[1]
    for dt, tn, forms in ((torch.float32, "f32", F32_FORMS), (torch.float64, "f64", F64_FORMS)):
        z = z32 if (dt == torch.float32 and z32 is not None) else ops.upload_planes(planes64, dt, dev)
        o = ops.empty_planes(10, n, dt, dev)
        for m, p in forms:
            # each form warms for 0.1 s first: the power management settles
            # on each kernel's own draw (the first calls after a switch or a
            # fresh output buffer run up to 15% slow)
            ms = time_calls(lambda m=m, p=p: ops.inv_det(z, m, p, inv=o[:9], det=o[9]), steps, 3, torch, 0.1)
            rows[f"{m}_{p}_{tn}"] = rate_row(n, ms, BYTES_PER_PX[tn],
                                             launch=ops.get_launch(ops.inv_det_launch_op(n), dt, m, p))
        if tune and dt == torch.float32:
            op = ops.inv_det_launch_op(n)
            for m, p in TUNED_F32_FORMS:
                keep = ops.get_launch(op, dt, m, p)
                cfg, _ = ops.autotune_inv_det(z, m, p, reps=5)
                ms = time_calls(lambda m=m, p=p: ops.inv_det(z, m, p, inv=o[:9], det=o[9]), steps, 3, torch, 0.1)
                rows[f"{m}_{p}_{tn}_autotuned"] = rate_row(n, ms, BYTES_PER_PX[tn], launch=cfg)
                ops.set_launch(op, dt, m, p, keep)
        del z, o
        torch.cuda.empty_cache()
    print(f"# {tag}: inverse forms done", file=sys.stderr, flush=True)
    return rows


def equal_accuracy(rows: dict) -> dict:
    """Cholesky time over adjugate time per pairing (above 1: adjugate faster).
    The FP32 comparisons at equal accuracy pit the compensated adjugate with
    its FP64 recompute against the Cholesky forms that also meet the FP32
    bar: FP64 arithmetic on FP32 storage (wide), and FP32 with FP64 fallback
    on pivot failure (that one meets the bar only up to kappa ~1e6)."""
    r = {"f32_plain": round(rows["cholesky_plain_f32"]["ms"] / rows["adjugate_plain_f32"]["ms"], 3),
         "f32_compensated_vs_cholesky_wide": round(rows["cholesky_wide_f32"]["ms"] /
                                                   rows["adjugate_compensated_f32"]["ms"], 3),
         "f32_compensated_vs_cholesky_fallback": round(rows["cholesky_compensated_f32"]["ms"] /
                                                       rows["adjugate_compensated_f32"]["ms"], 3),
         "f64_plain": round(rows["cholesky_plain_f64"]["ms"] / rows["adjugate_plain_f64"]["ms"], 3),
         "f64_compensated_vs_cholesky": round(rows["cholesky_plain_f64"]["ms"] /
                                              rows["adjugate_compensated_f64"]["ms"], 3)}
    if "adjugate_compensated_f32_autotuned" in rows:
        r["f32_compensated_vs_cholesky_wide_autotuned"] = round(
            rows["cholesky_wide_f32_autotuned"]["ms"] / rows["adjugate_compensated_f32_autotuned"]["ms"], 3)
        r["f32_compensated_vs_cholesky_fallback_autotuned"] = round(
            rows["cholesky_compensated_f32_autotuned"]["ms"] / rows["adjugate_compensated_f32_autotuned"]["ms"], 3)
    return r


def scale_rows(torch, ops, dev, img, steps: int) -> dict:
    """The 4096x4096 image: all inverse forms, the copy ceiling, the Wishart
    forward+backward, the fused multilook front ends, three-band
    block-diagonal pixels, the boxcar multilook, the nonlocal-means filter
    and the out-of-core streamer."""
    from paper_1807_08084_amd import synth
    z64 = img.planes.reshape(9, -1)
    n_px = z64.shape[1]
    rows = inverse_forms(torch, ops, dev, z64, steps, "4096^2", tune=False)
    for dt, tname in ((torch.float32, "f32"), (torch.float64, "f64")):
        zt = ops.upload_planes(z64, dt, dev)
        # measured ceiling: the same 9-in / 10-out plane streams with no
        # arithmetic, best of a sweep of launch shapes
        dst = ops.empty_planes(10, n_px, dt, dev)
        c_ms, ccfg = copy_ceiling(torch, ops, zt, dst, 9, 10, n_px, steps)
        rows[f"copy_9to10_{tname}"] = rate_row(n_px, c_ms, BYTES_PER_PX[tname], launch=ccfg)
        del dst
        # and the Wishart kernel's mix, 18 planes in and 9 out
        src18 = ops.empty_planes(18, n_px, dt, dev)
        dst9 = ops.empty_planes(9, n_px, dt, dev)
        c_ms, ccfg = copy_ceiling(torch, ops, src18, dst9, 18, 9, n_px, steps)
        rows[f"copy_18to9_{tname}"] = rate_row(n_px, c_ms, WISHART_BYTES_PER_PX[tname], launch=ccfg)
        del src18, dst9
        # Wishart forward+backward (fused): S = Z + 0.1 tr(Z)/3 I against Z
        sig = ops.empty_planes(9, n_px, dt, dev)
        sig.copy_(zt)
        tr = (zt[0] + zt[1] + zt[2]) * (0.1 / 3.0)
        for k in range(3):
            sig[k] += tr
        ws = torch.empty(max(1, ops.workspace_bytes(dt, n_px) // 8 + 1), dtype=torch.float64, device=dev)
        w_ms = time_calls(lambda: ops.wishart_loglik(sig, zt, 4.0, forward=True, backward=True, workspace=ws),
                          steps, 3, torch, 0.1)
        rows[f"wishart_fwd_bwd_{tname}"] = rate_row(n_px, w_ms, WISHART_BYTES_PER_PX[tname])
        del sig, ws, zt
        torch.cuda.empty_cache()
    # fused multilook front end (N=4 looks in, inverse + det out), FP32
    lk = ops.upload_planes(img.looks.reshape(24, -1).astype(np.float32), torch.float32, dev)
    for want_z, tag in ((False, "multilook_fused_f32"), (True, "multilook_fused_with_z_f32")):
        m_ms = time_calls(lambda: ops.multilook_inv_det(lk, 4, "adjugate", "compensated", want_z=want_z),
                          steps, 3, torch, 0.1)
        mb = 24 * 4 + 40 + (36 if want_z else 0)
        rows[tag] = rate_row(n_px, m_ms, mb, bytes_per_px=mb)
    # the multilook's mix without arithmetic: 24 planes in, 10 out
    dst10 = ops.empty_planes(10, n_px, torch.float32, dev)
    c_ms, ccfg = copy_ceiling(torch, ops, lk, dst10, 24, 10, n_px, steps)
    rows["copy_24to10_f32"] = rate_row(n_px, c_ms, 136, launch=ccfg)
    del dst10
    del lk
    torch.cuda.empty_cache()
    # block-diagonal pixels of three bands (multifrequency), FP32 compensated:
    # band 0 the image, bands 1 and 2 the image with its pixels rotated by a
    # third and two thirds (other matrices at every pixel); 27 planes in, 27
    # inverse planes and the determinant product out: 220 B per px
    bands = np.concatenate([np.roll(z64, (b * n_px) // 3, axis=1) for b in range(3)], axis=0)
    zb = ops.upload_planes(bands.astype(np.float32), torch.float32, dev)
    del bands
    b_ms = time_calls(lambda: ops.blockdiag_inv_det(zb, 3, "adjugate", "compensated"), steps, 3, torch, 0.1)
    rows["blockdiag_3_bands_f32"] = rate_row(n_px, b_ms, 220, bytes_per_px=220)
    dst28 = ops.empty_planes(28, n_px, torch.float32, dev)
    c_ms, ccfg = copy_ceiling(torch, ops, zb, dst28, 27, 28, n_px, steps)
    rows["copy_27to28_f32"] = rate_row(n_px, c_ms, 220, launch=ccfg)
    del zb, dst28
    torch.cuda.empty_cache()
    # spatial (boxcar) multilook of a single-look image, 3x3 and 7x7 windows,
    # inverse + det out; 24 B in + 40 B out per px
    sl = ops.upload_planes(synth.workload_boxcar().astype(np.float32).reshape(6, 4096, 4096), torch.float32, dev)
    for r in (1, 3):
        b_ms = time_calls(lambda: ops.boxcar_inv_det(sl, r, "adjugate", "compensated"), steps, 3, torch, 0.1)
        rows[f"boxcar_r{r}_f32"] = rate_row(n_px, b_ms, 64, bytes_per_px=64, window=f"{2 * r + 1}x{2 * r + 1}")
    del sl
    torch.cuda.empty_cache()
    # nonlocal-means filter, 23x23 window, on the image's inverse / det
    z32 = ops.upload_planes(z64, torch.float32, dev)
    inv, det, _ = ops.inv_det(z32, "adjugate", "compensated")
    zimg = z32.view(9, 4096, 4096)
    inv_img, det_img = inv.view(9, 4096, 4096), det.view(4096, 4096).contiguous()
    for dist, aux in (("kl", inv_img), ("bhattacharyya", det_img)):
        f = (lambda dist=dist, aux=aux: ops.nlm_wishart(zimg, aux, 4.0, 11, 16.0, dist))
        n_ms = time_calls(f, 5, 1, torch)
        rows[f"nlm_{dist}_r11_f32"] = {"gpx_s": round(n_px / n_ms / 1e6, 4), "ms": round(n_ms, 3),
                                       "pairs_per_s": float(f"{n_px * 529 / (n_ms * 1e-3):.4g}"),
                                       "window": "23x23"}
    del z32, inv, det, zimg, inv_img, det_img
    torch.cuda.empty_cache()
    # host-resident image through the out-of-core streamer (PCIe included)
    zh = torch.empty((9, n_px), dtype=torch.float32, pin_memory=True)
    zh.copy_(torch.from_numpy(z64.astype(np.float32)))
    ih = torch.empty((9, n_px), dtype=torch.float32, pin_memory=True)
    dh = torch.empty(n_px, dtype=torch.float32, pin_memory=True)
    streamer = ops.Streamer(torch.float32, 1 << 21, "adjugate", "compensated")
    streamer.run(zh, ih, dh)
    t0 = time.perf_counter()
    reps = 3
    for _ in range(reps):
        streamer.run(zh, ih, dh)
    s_ms = (time.perf_counter() - t0) * 1e3 / reps
    streamer.close()
    rows["streamer_host_f32"] = {"gpx_s": round(n_px / s_ms / 1e6, 3), "ms": round(s_ms, 3),
                                 "GB_s_pcie": round(BYTES_PER_PX["f32"] * n_px / (s_ms * 1e-3) / 1e9, 1),
                                 "chunk_px": 1 << 21, "note": "host pinned in and out, wall clock"}
    del zh, ih, dh
    torch.cuda.empty_cache()
    print(f"# 4096^2 rows done", file=sys.stderr, flush=True)
    return rows


OTHER_WORKLOADS = ("wishart", "batch", "paper")


def other_workloads(torch, ops, dev, steps, which=OTHER_WORKLOADS, tune_launch=True):
    """Each remaining workload timed on its own input (device time, data
    resident); with tune_launch, again at the launch the tuner picks."""
    from paper_1807_08084_amd import synth, tune
    from paper_1807_08084_amd.batch import BatchPlan
    res = {}
    if "wishart" in which:
        res.update(_wishart_workload(torch, ops, dev, steps, tune_launch))
    if "batch" in which:
        res.update(_batch_workload(torch, ops, dev, steps, tune_launch))
    if "paper" in which:
        res.update(_paper_workloads(torch, ops, dev))
    return res


def _wishart_workload(torch, ops, dev, steps, tune_launch):
    from paper_1807_08084_amd import synth, tune
    res = {}
    # Wishart: 2048^2, N=8; fused forward + backward.  One image's inputs and
    # gradient (453 MB in FP32) fit largely in the 256 MB last-level cache
    # after a call, so the calls rotate over four copies (1.8 / 3.6 GB) to
    # stream them from HBM as a fresh image would be
    img, sig = synth.workload_wishart()
    n = img.planes[0].size
    copies = 4
    for dt, tn, bpp in ((torch.float32, "f32", 108), (torch.float64, "f64", 216)):
        sets = []
        for _ in range(copies):
            sets.append((ops.upload_planes(sig.reshape(9, -1), dt, dev), ops.upload_planes(img.planes.reshape(9, -1), dt, dev),
                         ops.empty_planes(9, n, dt, dev)))
        ws = torch.empty(ops.workspace_bytes(dt, n) // 8 + 1, dtype=torch.float64, device=dev)
        k = [0]

        def call():
            st, zt, gt = sets[k[0] % copies]
            k[0] += 1
            ops.wishart_loglik(st, zt, 8.0, forward=True, backward=True, workspace=ws, grad=gt)
        steps_w = max(steps, 4 * copies)
        ms = time_calls(call, steps_w, copies, torch)
        res[f"wishart_2048_fwd_bwd_{tn}"] = rate_row(n, ms, bpp, input_copies=copies)
        if tune_launch:
            # again with the launch the Wishart tuner picks on this image
            wop = ops.wishart_launch_op(n)
            keep = ops.get_launch(wop, dt, "adjugate", "plain")
            cfg, _ = tune.tune_wishart(sets[0][0], sets[0][1], 8.0, reps=10)
            ms = time_calls(call, steps_w, copies, torch)
            res[f"wishart_2048_fwd_bwd_{tn}_autotuned"] = rate_row(n, ms, bpp, input_copies=copies, launch=cfg)
            ops.set_launch(wop, dt, "adjugate", "plain", keep)
        del sets, ws
        torch.cuda.empty_cache()
    print(f"# wishart workload done", file=sys.stderr, flush=True)
    return res


def _batch_workload(torch, ops, dev, steps, tune_launch):
    from paper_1807_08084_amd import synth, tune
    from paper_1807_08084_amd.batch import BatchPlan
    res = {}
    # batch: 64 images, FP32 compensated inverse + Wishart fwd + bwd, one graph
    # vs per-image loop; the graph again at the launch tune_batch picks
    imgs = synth.workload_batch()
    items = []
    for im in imgs:
        zf = im.planes.reshape(9, -1)
        items.append({"z": ops.upload_planes(zf, torch.float32, dev),
                      "sigma": ops.upload_planes(synth.wishart_sigma0(zf), torch.float32, dev),
                      "n_looks": float(im.n_looks)})
    del imgs
    n = sum(it["z"].shape[1] for it in items)
    plan = BatchPlan(items, "adjugate", "compensated", status=False)
    g_ms = time_calls(plan.run, steps, 3, torch, 0.1)
    plan.close()
    ws = torch.empty(ops.workspace_bytes(torch.float32, max(it["z"].shape[1] for it in items)) // 8 + 1,
                     dtype=torch.float64, device=dev)
    outs = [(ops.empty_planes(10, it["z"].shape[1], torch.float32, dev)) for it in items]

    def loop():
        for it, ob in zip(items, outs):
            ops.inv_det(it["z"], "adjugate", "compensated", inv=ob[:9], det=ob[9])
            ops.wishart_loglik(it["sigma"], it["z"], it["n_looks"], forward=True, backward=True, workspace=ws)
    l_ms = time_calls(loop, steps, 3, torch, 0.1)
    del outs, ws
    # the batch's mix without arithmetic: Z and S in (18 planes), inverse, det
    # and gradient out (19), over as many pixels as the 64 images hold
    src18 = ops.empty_planes(18, n, torch.float32, dev)
    dst19 = ops.empty_planes(19, n, torch.float32, dev)
    c_ms, c_cfg = copy_ceiling(torch, ops, src18, dst19, 18, 19, n, steps)
    del src18, dst19
    torch.cuda.empty_cache()
    default_cfg = ops.get_launch(3, torch.float32, "adjugate", "compensated")
    rec = {"pixels": n, "graph_ms": round(g_ms, 4), "loop_ms": round(l_ms, 4),
           "graph_gpx_s": round(n / g_ms / 1e6, 3), "loop_gpx_s": round(n / l_ms / 1e6, 3),
           "graph_GB_s": round(148 * n / g_ms / 1e6, 1),
           "graph_frac_hbm": round(148 * n / g_ms / 1e6 / PEAK_HBM_GBS, 4), "launch": default_cfg,
           "copy_18to19_GB_s": round(148 * n / c_ms / 1e6, 1),
           "copy_18to19_frac_hbm": round(148 * n / c_ms / 1e6 / PEAK_HBM_GBS, 4),
           "graph_frac_of_copy_ceiling": round(c_ms / g_ms, 4), "copy_launch": c_cfg,
           "bytes_per_px": 148, "ops": "inverse+det of Z, Wishart fwd+bwd of S against Z (FP32 compensated)"}
    if tune_launch:
        t_cfg, _ = tune.tune_batch(items, reps=5)
        plan = BatchPlan(items, "adjugate", "compensated", status=False)
        t_ms = time_calls(plan.run, steps, 3, torch, 0.1)
        plan.close()
        ops.set_launch(3, torch.float32, "adjugate", "compensated", default_cfg)
        rec.update({"autotuned_graph_ms": round(t_ms, 4), "autotuned_graph_gpx_s": round(n / t_ms / 1e6, 3),
                    "autotuned_graph_frac_hbm": round(148 * n / t_ms / 1e6 / PEAK_HBM_GBS, 4),
                    "autotuned_launch": t_cfg})
    res["batch_64_images"] = rec
    del items
    torch.cuda.empty_cache()
    print(f"# batch workload done", file=sys.stderr, flush=True)
    return res


def _paper_workloads(torch, ops, dev):
    from paper_1807_08084_amd import synth
    res = {}
    # the paper's Table 2 shapes: 5,469,354 simulated M M^H matrices and a
    # 450 x 600 image, both forms, single launches like the paper's replicates
    shapes = (("simulated_5469354", synth.workload_paper_simulated()),
              ("airsar_450x600", synth.workload_airsar_standin().planes.reshape(9, -1)))
    paper = {}
    for name, planes in shapes:
        n = planes.shape[1]
        rec = {"pixels": n, "paper_ms": PAPER_TABLE2_MS[name]}
        for dt, tn in ((torch.float32, "f32"), (torch.float64, "f64")):
            z = ops.upload_planes(planes, dt, dev)
            o = ops.empty_planes(10, n, dt, dev)
            for method, prec in (("adjugate", "plain"), ("cholesky", "plain"), ("adjugate", "compensated")):
                f = lambda: ops.inv_det(z, method, prec, inv=o[:9], det=o[9])
                warm(f, 10, torch)
                rec[f"{method}_{prec}_{tn}_ms"] = launch_spread(f, 1000, torch)
            del z, o
        paper[name] = rec
    res["paper_table2_shapes"] = paper
    print(f"# paper-shaped workloads done", file=sys.stderr, flush=True)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-rows", action="store_true")
    ap.add_argument("--tune", action="store_true", help="autotune the step's launch before timing")
    ap.add_argument("--launch", type=str, default=None,
                    help="JSON launch shape to install for the step before timing (e.g. an autotuned one)")
    ap.add_argument("--workloads", action="store_true",
                    help="time the other workloads too (the default unless --no-rows or --no-workloads)")
    ap.add_argument("--no-workloads", action="store_true",
                    help="skip the 2048^2 Wishart, 64-image batch and paper-shaped workloads")
    ap.add_argument("--workload", action="append", choices=OTHER_WORKLOADS,
                    help="time only these of the other workloads (repeatable; implies --workloads)")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the autotuned rows of the other workloads")
    ap.add_argument("--no-8192-rows", action="store_true",
                    help="skip the rows of the two 8192^2 images (keep the 4096^2 rows; for profiling)")
    ap.add_argument("--probe", action="store_true",
                    help="after the timed steps, run a one-plane copy of the same pixel count "
                         "(known bytes: calibrates the HBM traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU; --gpus {args.gpus} is not supported "
              "(every pixel is independent: an image shards by rows across GPUs, and only the "
              "Wishart loss, one FP64 scalar, would need an all-reduce)", file=sys.stderr)
        sys.exit(2)

    from paper_1807_08084_amd import synth
    t = time.perf_counter()
    img = synth.workload_precision()
    z64 = img.planes.reshape(9, -1)
    del img
    n_px = z64.shape[1]
    print(f"# generated {n_px} px in {time.perf_counter() - t:.1f} s", file=sys.stderr, flush=True)

    import torch
    from paper_1807_08084_amd import ops
    dev = torch.device("cuda:0")
    # device layout: planes at the recommended pitch; the 9 inverse planes and
    # the det plane share one buffer.  FP32 planes are the RN rounding of the
    # generator's FP64 values.
    z32 = ops.upload_planes(z64.astype(np.float32), torch.float32, dev)
    outp = ops.empty_planes(10, n_px, torch.float32, dev)
    inv, det = outp[:9], outp[9]
    launch_op = ops.inv_det_launch_op(n_px)
    if args.launch:
        ops.set_launch(launch_op, torch.float32, "adjugate", "compensated", json.loads(args.launch))
    if args.tune:
        cfg, ms = ops.autotune_inv_det(z32, "adjugate", "compensated", reps=5)
        print(f"# tuned {json.dumps(cfg)} {ms:.3f} ms", file=sys.stderr, flush=True)
    launch = ops.get_launch(launch_op, torch.float32, "adjugate", "compensated")

    def step():
        ops.inv_det(z32, "adjugate", "compensated", inv=inv, det=det)

    # Settle: after the host-side set-up the GPU is idle, and its power
    # management takes ~25 ms of load to reach a steady clock (the first
    # calls of a cold start run 0.84, 0.90, then 1.3 ms, settling at
    # 0.87-0.88 ms).  A plane copy of the same image (no arithmetic, not a
    # step) runs for SETTLE_S first; then exactly `warmup` untimed steps and
    # exactly `steps` timed ones between two events on the stream the kernels
    # run on (torch's current stream).
    settle_dst = ops.empty_planes(10, n_px, torch.float32, dev)
    settle_calls = warm(lambda: ops.stream_copy(z32, settle_dst, 9, 10, n_px), 1, torch, SETTLE_S)
    del settle_dst
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ms = time_calls(step, args.steps, 0, torch)
    # the spread of single launches (after the timed region; not part of the value)
    launch_stats = launch_spread(step, args.steps, torch)
    launch_stats["gpx_s_at_median"] = round(n_px / launch_stats["median"] / 1e6, 3)
    # the status counters of one more call: pixels recomputed in FP64
    ctr = torch.zeros(3, dtype=torch.int64, device=dev)
    ops.inv_det(z32, "adjugate", "compensated", inv=inv, det=det, counters=ctr)
    c = ctr.tolist()
    if args.probe:
        src1 = z32[0:1]
        dst1 = ops.empty_planes(1, n_px, torch.float32, dev)
        for _ in range(args.steps):
            ops.stream_copy(src1, dst1, 1, 1, n_px)
        torch.cuda.synchronize()
        print(f"# probe: k_copy 1->1 plane, {n_px * 4} bytes read and written per launch",
              file=sys.stderr, flush=True)
        del dst1
    value = n_px / (ms * 1e-3) / 1e9
    achieved = BYTES_PER_PX["f32"] * n_px / (ms * 1e-3) / 1e9
    kname = "k_inv_det<float, ADJ_COMP>"
    traffic_bytes = traffic_from_profiles(kname, n_px)
    traffic = None if traffic_bytes is None else round(traffic_bytes / (ms * 1e-3) / 1e9, 1)
    out = {
        "metric": "Gpixel/s inv+det & %HBM roofline, adjugate vs Cholesky, 1 MI355X",
        "value": round(value, 3), "unit": "Gpixel/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": WORKLOAD,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic,
                     "traffic_bytes_per_launch": traffic_bytes,
                     "kernel": kname, "algorithmic_bytes_per_px": BYTES_PER_PX["f32"],
                     "launch_op": launch_op, "launch": launch},
        "launch_ms": launch_stats,
        "settle": {"kernel": "9->10 plane copy of the image (no arithmetic; not a step)", "seconds": SETTLE_S,
                   "calls": settle_calls},
        "status_counts": {"not_pd": c[0], "rerouted": c[1], "nonfinite": c[2],
                          "rerouted_fraction": round(c[1] / n_px, 4)},
    }
    if not args.no_rows:
        ksteps = max(10, args.steps // 2)
        # the step's access mix without arithmetic on the same image (9 planes
        # in, 10 out; launch swept): the practical streaming ceiling at 8192^2
        c_ms, c_cfg = copy_ceiling(torch, ops, z32, outp, 9, 10, n_px, ksteps)
        out["copy_ceiling_8192"] = {"kernel": "9->10 plane copy of the step's image", "ms": round(c_ms, 4),
                                    "GB_s": round(BYTES_PER_PX["f32"] * n_px / c_ms / 1e6, 1),
                                    "frac_hbm": round(BYTES_PER_PX["f32"] * n_px / c_ms / 1e6 / PEAK_HBM_GBS, 4),
                                    "launch": c_cfg, "step_frac_of_ceiling": round(c_ms / ms, 4),
                                    "launch_median_frac_of_ceiling": round(c_ms / launch_stats["median"], 4)}
        out["speedup_adjugate_vs_cholesky"] = {}
        if not args.no_8192_rows:
            # the other forms on the same image; the default step again
            prec_rows = inverse_forms(torch, ops, dev, z64, ksteps, "precision 8192^2", tune=True, z32=z32)
            out["precision_8192_rows"] = prec_rows
            out["speedup_adjugate_vs_cholesky"]["precision_8192"] = equal_accuracy(prec_rows)
            img8 = synth.workload_scale8192()
            s8 = img8.planes.reshape(9, -1)
            del img8
            rows8 = inverse_forms(torch, ops, dev, s8, ksteps, "scale 8192^2", tune=True)
            del s8
            out["scale_8192_rows"] = rows8
            out["speedup_adjugate_vs_cholesky"]["scale_8192"] = equal_accuracy(rows8)
        simg = synth.workload_scale(with_looks=True)
        srows = scale_rows(torch, ops, dev, simg, ksteps)
        del simg
        out["scale_4096_rows"] = srows
        out["scale_4096_config"] = SCALE_WORKLOAD
        out["speedup_adjugate_vs_cholesky"]["scale_4096"] = equal_accuracy(srows)
        out["speedup_adjugate_vs_cholesky"]["paper_context"] = "about 2.2x on a GeForce 940M, OpenCL (Table 2)"
        out["copy_ceiling_frac_4096"] = round(srows["copy_9to10_f32"]["ms"] / srows["adjugate_compensated_f32"]["ms"], 4)
    if args.workload or args.workloads or not (args.no_rows or args.no_workloads):
        out["workloads"] = other_workloads(torch, ops, dev, max(10, args.steps // 4),
                                           tuple(args.workload or OTHER_WORKLOADS), not args.no_tune)
    del z32, outp, inv, det
    torch.cuda.empty_cache()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(z64.astype(np.float32).astype(np.float64), n_px)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

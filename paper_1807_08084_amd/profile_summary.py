"""Summarise rocprofv3 result databases (SQLite) into short text records.

    python -m paper_1807_08084_amd.profile_summary trace <kt_results.db> <out.txt> "<command>"
    python -m paper_1807_08084_amd.profile_summary traffic <fetch.db> <write.db> <out.txt> "<commands>" [n_px] [label]
    python -m paper_1807_08084_amd.profile_summary counters <pmc.db> <out.txt> "<command>"
    python -m paper_1807_08084_amd.profile_summary traffic_rows <fetch.db> <write.db> <out.txt> "<commands>"
    python -m paper_1807_08084_amd.profile_summary traffic_kernel <fetch.db> <write.db> <out.txt> "<commands>" \
        <kernel-prefix> <n_px> <alg_read_B_px> <alg_write_B_px> "<label>"

``trace`` lists each kernel's calls and mean duration (the --kernel-trace
--stats view).  ``traffic`` turns per-dispatch FETCH_SIZE / WRITE_SIZE (KiB)
into HBM bytes per launch of the inverse kernel, each scaled by what the same
counter reads for the one-plane copy probe of known size (bench.py --probe).
"""
from __future__ import annotations

import hashlib
import os
import sqlite3
import statistics
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


# the sources the per-call kernels (the inverse among them) are compiled from
STEP_SOURCES = ("common.hpp", "pixel.hpp", "polsar.hip")


def source_hash(names=STEP_SOURCES) -> str:
    h = hashlib.sha256()
    csrc = os.path.join(HERE, "csrc")
    for name in names:
        h.update(open(os.path.join(csrc, name), "rb").read())
    return h.hexdigest()[:16]


def all_sources_hash() -> str:
    csrc = os.path.join(HERE, "csrc")
    return source_hash(sorted(n for n in os.listdir(csrc) if n.endswith((".hip", ".hpp"))))


def _hash_lines() -> str:
    return (f"# source_hash = {source_hash()}  (common.hpp, pixel.hpp, polsar.hip)\n"
            f"# all_sources_hash = {all_sources_hash()}  (every .hip and .hpp, the batch kernel's included)\n")


def short(name: str) -> str:
    return name.replace("(anonymous namespace)::", "").split("(")[0].replace("void ", "")


def trace(db: str, out: str, command: str) -> None:
    con = sqlite3.connect(db)
    rows = con.execute("select name, total_calls, total_duration, average, percentage from top_kernels").fetchall()
    with open(out, "w") as fh:
        fh.write(f"# rocprofv3 --kernel-trace --stats summary\n# command: {command}\n")
        fh.write(_hash_lines())
        fh.write(f"{'kernel':60s} {'calls':>6s} {'total_us':>12s} {'avg_us':>10s} {'pct':>6s}\n")
        for name, calls, total, avg, pct in rows:
            fh.write(f"{short(name):60s} {calls:6d} {total:12.3f} {avg:10.3f} {pct:6.2f}\n")
    print(open(out).read())


def _counter(db: str, counter: str, main_grid: bool = False):
    """Mean value per dispatch, by kernel; with main_grid, over the kernel's
    dispatches at its most frequent grid size only."""
    con = sqlite3.connect(db)
    rows = con.execute("select kernel_name, value, grid_size from counters_collection where counter_name=?",
                       (counter,)).fetchall()
    agg = {}
    for k, v, g in rows:
        agg.setdefault(short(k), {}).setdefault(g if main_grid else 0, []).append(v)
    return {k: statistics.mean(max(by.values(), key=len)) for k, by in agg.items()}


def traffic(fetch_db: str, write_db: str, out: str, command: str, n_px: int = 4096 * 4096,
            label: str = "4096x4096 image") -> None:
    """HBM bytes per launch of the FP32 compensated inverse kernel over an
    n_px-pixel image (its dispatches at the most frequent grid size)."""
    f = _counter(fetch_db, "FETCH_SIZE", main_grid=True)
    w = _counter(write_db, "WRITE_SIZE", main_grid=True)
    def one_plane_copy(k):  # k_copy<float, V, 1, 1[, NT]>
        args = k[k.find("<") + 1:k.rfind(">")].split(", ")
        return k.startswith("k_copy<float,") and args[2:4] == ["1", "1"]
    probe = next(k for k in f if one_plane_copy(k))
    kern = next(k for k in f if k.startswith("k_inv_det<float, 1,"))
    probe_bytes = 4 * n_px
    f_scale = probe_bytes / (f[probe] * 1024)
    w_scale = probe_bytes / (w[probe] * 1024)
    rd = f[kern] * 1024 * f_scale
    wr = w[kern] * 1024 * w_scale
    alg_rd, alg_wr = 36 * n_px, 40 * n_px
    with open(out, "w") as fh:
        fh.write(f"# HBM traffic of the FP32 compensated adjugate inverse kernel ({kern}), {label}\n")
        fh.write(f"# command: {command}\n")
        fh.write(f"# FETCH_SIZE probe {f[probe]:.1f} KiB for {probe_bytes} B read  -> scale {f_scale:.5f}\n")
        fh.write(f"# WRITE_SIZE probe {w[probe]:.1f} KiB for {probe_bytes} B written -> scale {w_scale:.5f}\n")
        fh.write(f"# kernel FETCH_SIZE {f[kern]:.1f} KiB, WRITE_SIZE {w[kern]:.1f} KiB per dispatch\n")
        fh.write(f"# read {rd:.0f} B (algorithmic {alg_rd}, ratio {rd / alg_rd:.5f}); "
                 f"write {wr:.0f} B (algorithmic {alg_wr}, ratio {wr / alg_wr:.5f})\n")
        fh.write(f"kernel = k_inv_det<float, ADJ_COMP>\n")
        fh.write(f"pixels = {n_px}\n")
        fh.write(f"source_hash = {source_hash()}\n")
        fh.write(f"read_bytes_per_launch = {rd:.0f}\n")
        fh.write(f"write_bytes_per_launch = {wr:.0f}\n")
        fh.write(f"bytes_per_launch = {rd + wr:.0f}\n")
    print(open(out).read())


def traffic_kernel(fetch_db: str, write_db: str, out: str, command: str, prefix: str, n_px: int,
                   alg_read: float, alg_write: float, label: str) -> None:
    """HBM bytes per pixel of one kernel (the first whose name starts with
    prefix; its dispatches at the most frequent grid size) over n_px pixels,
    against its algorithmic bytes per pixel, FETCH_SIZE and WRITE_SIZE scaled
    by the one-plane copy probe (4 bytes per pixel of the probe's grid)."""
    f = _counter(fetch_db, "FETCH_SIZE", main_grid=True)
    w = _counter(write_db, "WRITE_SIZE", main_grid=True)
    fg = _counter_grid(fetch_db, "FETCH_SIZE")

    def one_plane_copy(k):
        args = k[k.find("<") + 1:k.rfind(">")].split(", ")
        return k.startswith("k_copy<float,") and args[2:4] == ["1", "1"]
    probe = next(k for k in f if one_plane_copy(k))
    probe_px = fg[probe] * int(probe[probe.find("<") + 1:].split(", ")[1])  # threads x pixels per lane
    kern = next(k for k in f if k.startswith(prefix))
    f_scale = 4 * probe_px / (f[probe] * 1024)
    w_scale = 4 * probe_px / (w[probe] * 1024)
    rd = f[kern] * 1024 * f_scale / n_px
    wr = w[kern] * 1024 * w_scale / n_px
    with open(out, "w") as fh:
        fh.write(f"# HBM traffic of {kern}, {label}\n# command: {command}\n")
        fh.write(_hash_lines())
        fh.write(f"# scales from the one-plane copy probe ({probe_px} pixels): FETCH_SIZE x{f_scale:.5f}, "
                 f"WRITE_SIZE x{w_scale:.5f}\n")
        fh.write(f"# kernel FETCH_SIZE {f[kern]:.1f} KiB, WRITE_SIZE {w[kern]:.1f} KiB per dispatch\n")
        fh.write(f"read B/px {rd:.3f} (algorithmic {alg_read}, ratio {rd / alg_read:.5f})\n")
        fh.write(f"write B/px {wr:.3f} (algorithmic {alg_write}, ratio {wr / alg_write:.5f})\n")
    print(open(out).read())


def _counter_grid(db: str, counter: str):
    """Most frequent grid size (threads) of each kernel's dispatches."""
    con = sqlite3.connect(db)
    rows = con.execute("select kernel_name, grid_size from counters_collection where counter_name=?",
                       (counter,)).fetchall()
    by = {}
    for k, g in rows:
        by.setdefault(short(k), []).append(g)
    return {k: max(set(v), key=v.count) for k, v in by.items()}


# Kernels of the bench rows on the 4096x4096 image and their algorithmic
# bytes per pixel (read, written).
ROW_KERNELS = [
    ("k_inv_det<float, 1, 2, 1, true>", "FP32 compensated adjugate", 36, 40),
    ("k_inv_det<double, 1, 2, 1, true>", "FP64 compensated adjugate", 72, 80),
    ("k_inv_det<float, 3, 2, 1, true>", "FP32 plain Cholesky", 36, 40),
    ("k_wishart<float, 4, 1, true>", "FP32 Wishart fwd+bwd", 72, 36),
    ("k_wishart<double, 1, 1, true>", "FP64 Wishart fwd+bwd", 144, 72),
    ("k_boxcar_shift<float, 1, 1>", "boxcar 3x3 (halo rows: +2/32 of the reads)", 24, 40),
    ("k_boxcar_grouped<float, 1, 3>", "boxcar 7x7 (halo rows: +6/64 of the reads)", 24, 40),
    ("k_blockdiag<float, 1, 4, true>", "three-band block-diagonal inverse (27 planes in, 27 + det out)", 108, 112),
    ("k_nlm<float, 0, 2>", "nonlocal means 23x23, KL (Z and its inverse in, filtered Z out)", 72, 36),
    ("k_nlm<float, 1, 2>", "nonlocal means 23x23, Bhattacharyya (Z and det in)", 40, 36),
]


def traffic_rows(fetch_db: str, write_db: str, out: str, command: str, n_px: int = 4096 * 4096) -> None:
    """HBM bytes per pixel of the bench rows' kernels (FETCH_SIZE / WRITE_SIZE
    per dispatch, scaled by the one-plane copy probe: 4 bytes per pixel of
    the probe's grid) against their algorithmic bytes.  Each kernel's
    dispatches at its most frequent grid size are used (the image; the
    streamer's chunks share kernel names)."""
    f = _counter(fetch_db, "FETCH_SIZE", main_grid=True)
    w = _counter(write_db, "WRITE_SIZE", main_grid=True)
    fg = _counter_grid(fetch_db, "FETCH_SIZE")

    def one_plane_copy(k):
        args = k[k.find("<") + 1:k.rfind(">")].split(", ")
        return k.startswith("k_copy<float,") and args[2:4] == ["1", "1"]
    probe = next(k for k in f if one_plane_copy(k))
    probe_px = fg[probe] * int(probe[probe.find("<") + 1:].split(", ")[1])  # threads x pixels per lane
    f_scale = 4 * probe_px / (f[probe] * 1024)
    w_scale = 4 * probe_px / (w[probe] * 1024)
    with open(out, "w") as fh:
        fh.write("# HBM traffic per pixel of the bench rows' kernels, 4096x4096 image\n")
        fh.write(f"# command: {command}\n")
        fh.write(_hash_lines())
        fh.write(f"# scales from the one-plane copy probe ({probe_px} pixels): FETCH_SIZE x{f_scale:.5f}, "
                 f"WRITE_SIZE x{w_scale:.5f}\n")
        fh.write(f"{'kernel':36s} {'read B/px':>10s} {'alg':>5s} {'ratio':>7s} {'write B/px':>11s} {'alg':>5s} "
                 f"{'ratio':>7s}  what\n")
        for name, what, ar, aw in ROW_KERNELS:
            if name not in f or name not in w:
                continue
            rd = f[name] * 1024 * f_scale / n_px
            wr = w[name] * 1024 * w_scale / n_px
            fh.write(f"{name:36s} {rd:10.2f} {ar:5d} {rd / ar:7.4f} {wr:11.2f} {aw:5d} {wr / aw:7.4f}  {what}\n")
    print(open(out).read())


def counters(db: str, out: str, command: str, n_px: int = 4096 * 4096) -> None:
    """Mean of each counter per dispatch, by kernel and grid size, and the
    VALU lane-instructions per pixel (SQ_INSTS_VALU x 64 / n_px) for
    dispatches that cover an n_px-pixel image."""
    con = sqlite3.connect(db)
    rows = con.execute("select kernel_name, grid_size, counter_name, value from counters_collection").fetchall()
    agg = {}
    for k, g, cn, v in rows:
        agg.setdefault((short(k), g), {}).setdefault(cn, []).append(v)
    names = sorted({cn for d in agg.values() for cn in d})
    with open(out, "w") as fh:
        fh.write(f"# rocprofv3 --pmc summary: mean per dispatch\n# command: {command}\n")
        fh.write(_hash_lines())
        fh.write(f"# valu_per_px = SQ_INSTS_VALU * 64 / {n_px} (meaningful where the dispatch covers the image)\n")
        fh.write(f"{'kernel':44s} {'grid':>10s} {'calls':>5s} " + " ".join(f"{n:>15s}" for n in names)
                 + f" {'valu_per_px':>11s}\n")
        for key in sorted(agg, key=lambda t: (t[0], t[1])):
            d = agg[key]
            calls = max(len(v) for v in d.values())
            means = [statistics.mean(d[n]) if n in d else float("nan") for n in names]
            vpp = statistics.mean(d["SQ_INSTS_VALU"]) * 64 / n_px if "SQ_INSTS_VALU" in d else float("nan")
            fh.write(f"{key[0][:44]:44s} {key[1]:10d} {calls:5d} " + " ".join(f"{m:15.0f}" for m in means)
                     + f" {vpp:11.1f}\n")
    print(open(out).read())


if __name__ == "__main__":
    if sys.argv[1] == "trace":
        trace(sys.argv[2], sys.argv[3], sys.argv[4])
    elif sys.argv[1] == "counters":
        counters(sys.argv[2], sys.argv[3], sys.argv[4], *([int(sys.argv[5])] if len(sys.argv) > 5 else []))
    elif sys.argv[1] == "traffic_kernel":
        traffic_kernel(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5], sys.argv[6], int(sys.argv[7]),
                       float(sys.argv[8]), float(sys.argv[9]), sys.argv[10])
    elif sys.argv[1] == "traffic_rows":
        traffic_rows(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5])
    else:
        traffic(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5],
                *([int(sys.argv[6])] if len(sys.argv) > 6 else []), *sys.argv[7:8])

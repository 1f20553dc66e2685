"""The measurement plumbing on the CPU: the bench's one-GPU contract and its
copy-ceiling sweep, the profile summariser on a small
synthetic counter database, and the bench's lookup of the committed HBM
traffic record (used only while it was taken on the current sources)."""
import os
import sqlite3

import pytest

import bench
from paper_1807_08084_amd import profile_summary as ps

N_PX = 4096 * 4096


def _db(path, counter, rows):
    con = sqlite3.connect(path)
    con.execute("create table counters_collection (kernel_name text, grid_size integer, counter_name text, "
                "value real, workgroup_size integer)")
    con.executemany("insert into counters_collection values (?, ?, ?, ?, 256)",
                    [(k, g, counter, v) for k, g, v in rows])
    con.commit()
    con.close()


def test_source_hashes_agree():
    assert ps.source_hash() == bench.kernel_source_hash()


def test_traffic_rows_scales_by_the_probe_and_takes_the_main_grid(tmp_path):
    probe = "void (anonymous namespace)::k_copy<float, 4, 1, 1, true>(float const*, long)"
    inv = "void (anonymous namespace)::k_inv_det<float, 1, 2, 1, true>((anonymous namespace)::InvDetArgs)"
    kib = 4 * N_PX / 1024
    # FETCH_SIZE reads half the bytes (scale 2), WRITE_SIZE all of them; the
    # inverse kernel's main grid has three dispatches, a smaller one two
    _db(tmp_path / "f.db", "FETCH_SIZE", [(probe, 4194304, kib / 2)] * 2
        + [(inv, 8388608, 9 * kib / 2)] * 3 + [(inv, 1048576, kib / 8)] * 2)
    _db(tmp_path / "w.db", "WRITE_SIZE", [(probe, 4194304, kib)] * 2
        + [(inv, 8388608, 10 * kib)] * 3 + [(inv, 1048576, kib / 4)] * 2)
    out = tmp_path / "t.txt"
    ps.traffic_rows(str(tmp_path / "f.db"), str(tmp_path / "w.db"), str(out), "cmd")
    line = next(ln for ln in open(out) if ln.startswith("k_inv_det<float, 1, 2, 1, true>"))
    rd, alg_r, ratio_r, wr, alg_w, ratio_w = line.split()[5:11]
    assert float(rd) == pytest.approx(36.0) and float(ratio_r) == pytest.approx(1.0)
    assert float(wr) == pytest.approx(40.0) and float(ratio_w) == pytest.approx(1.0)


def test_bench_reads_traffic_only_for_the_current_sources(tmp_path, monkeypatch):
    rec = tmp_path / "profiles"
    rec.mkdir()
    text = ("# header\nkernel = k_inv_det<float, ADJ_COMP>\npixels = 16777216\nsource_hash = {h}\n"
            "bytes_per_launch = 1275000000\n")
    monkeypatch.setattr(bench, "HERE", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "abc")
    (rec / bench.TRAFFIC_RECORD).write_text(text.format(h="abc"))
    assert bench.traffic_from_profiles("k_inv_det<float, ADJ_COMP>", N_PX) == 1275000000.0
    assert bench.traffic_from_profiles("k_inv_det<double, ADJ_COMP>", N_PX) is None
    assert bench.traffic_from_profiles("k_inv_det<float, ADJ_COMP>", 4 * N_PX) is None  # another image
    (rec / bench.TRAFFIC_RECORD).write_text(text.format(h="stale"))
    assert bench.traffic_from_profiles("k_inv_det<float, ADJ_COMP>", N_PX) is None
    os.remove(rec / bench.TRAFFIC_RECORD)
    assert bench.traffic_from_profiles("k_inv_det<float, ADJ_COMP>", N_PX) is None


def test_bench_refuses_more_than_one_gpu():
    """bench.py runs on one GPU: --gpus 2 exits with status 2 and says why,
    before anything touches a GPU."""
    import subprocess
    import sys
    p = subprocess.run([sys.executable, bench.__file__, "--gpus", "2"], capture_output=True, text=True, timeout=120)
    assert p.returncode == 2 and "runs on one GPU" in p.stderr and p.stdout == ""


def test_copy_ceiling_keeps_the_launch_table(monkeypatch):
    """The bench's copy-ceiling sweep restores the probe's launch entry and
    returns the fastest shape it timed."""
    calls, table = [], {"cfg": {"block": 128}}

    class FakeOps:
        @staticmethod
        def get_launch(op, dt, m, p):
            return table["cfg"]

        @staticmethod
        def set_launch(op, dt, m, p, cfg):
            table["cfg"] = cfg

        @staticmethod
        def stream_copy(src, dst, n_in, n_out, n):
            calls.append(table["cfg"])

    class FakeSrc:
        dtype = "f32"

    times = iter(range(100, 0, -1))
    monkeypatch.setattr(bench, "time_calls", lambda fn, steps, warmup, torch, *a: (fn(), float(next(times)))[1])
    ms, cfg = bench.copy_ceiling(None, FakeOps, FakeSrc(), None, 9, 10, 1000, 3)
    assert table["cfg"] == {"block": 128}
    last = bench.COPY_SHAPES[-1]
    assert (cfg["block"], cfg["vector_bytes"], cfg["blocks_per_cu"]) == last and ms == 100 - len(bench.COPY_SHAPES) + 1

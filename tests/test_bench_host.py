"""Host-side pieces of bench.py (no GPU): byte accounting, the counter-traffic record, the one-GPU guard."""
import json
import os
import sqlite3
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_algorithmic_bytes_of_the_single_point_workload():
    # 150 bins of a 1600 x 1600 complex64 kernel, one column: kernel 3.072 GB, the product adds the
    # spectrum in and out (8 B per bin and trace each), an apply adds the time vector in and out
    kernel, product, apply = bench.algorithmic_bytes(512, 150, 1600, 1)
    assert kernel == 8 * 150 * 1600 * 1600 == 3_072_000_000
    assert product == kernel + 2 * 8 * 150 * 1600 == 3_075_840_000
    assert apply == kernel + 2 * 4 * 512 * 1600


def _counter_db(path, counter, rows):
    con = sqlite3.connect(path)
    con.execute("create table counters_collection (kernel_name text, counter_name text, value real)")
    con.executemany("insert into counters_collection values (?, ?, ?)", [(k, counter, v) for k, v in rows])
    con.commit()
    con.close()


def test_write_traffic_scales_counters_by_the_copy_calibration(tmp_path, monkeypatch):
    copy_kib = bench.COPY_BYTES / 1024
    fwd = "void mdc::(anonymous namespace)::gemv_fwd_kernel<0, 1, 4, 1>(char const*, float const*)"
    adj = "void mdc::(anonymous namespace)::gemv_adj_kernel<0, 1, 16>(char const*, float const*)"
    # the copy reads as twice its bytes on FETCH_SIZE and as its bytes on WRITE_SIZE
    _counter_db(tmp_path / "f.db", "FETCH_SIZE",
                [("__amd_rocclr_copyBuffer", 2 * copy_kib)] * 3 + [(fwd, 3000.0), (fwd, 3002.0), (adj, 4000.0),
                                                                  ("rfft_trunc_kernel<256>", 99.0)])
    _counter_db(tmp_path / "w.db", "WRITE_SIZE",
                [("__amd_rocclr_copyBuffer", copy_kib)] * 3 + [(fwd, 10.0), (fwd, 10.0), (adj, 20.0)])
    out = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(out))
    bench.write_traffic(str(tmp_path / "f.db"), str(tmp_path / "w.db"))
    rec = json.loads(out.read_text())
    assert rec["copy_calibration"]["fetch_factor"] == 0.5 and rec["copy_calibration"]["write_factor"] == 1.0
    k = rec["kernels"]
    assert set(k) == {"gemv_fwd_kernel<0, 1, 4, 1>", "gemv_adj_kernel<0, 1, 16>"}  # transforms left out
    assert k["gemv_fwd_kernel<0, 1, 4, 1>"]["fetch_bytes"] == round(3001.0 * 1024 * 0.5)
    assert k["gemv_adj_kernel<0, 1, 16>"]["write_bytes"] == 20 * 1024
    per_launch = ((3001.0 * 512 + 10 * 1024) + (4000.0 * 512 + 20 * 1024)) / 2
    assert rec["bytes_per_launch"] == round(per_launch)
    assert rec["source_sha256_16"] == bench.source_hash(bench.PRODUCT_SRC)
    assert rec["workload"] == bench.WORKLOAD


def test_committed_traffic_record_is_consistent():
    """The stored record's per-launch bytes follow from its own per-kernel counters and calibration,
    and it describes the benchmark's workload (the source hash is checked by bench.py at run time)."""
    with open(bench.TRAFFIC_FILE) as fh:
        rec = json.load(fh)
    assert rec["workload"] == bench.WORKLOAD
    ff, wf = rec["copy_calibration"]["fetch_factor"], rec["copy_calibration"]["write_factor"]
    per = [v["fetch_KiB_raw"] * 1024 * ff + v["write_KiB_raw"] * 1024 * wf for v in rec["kernels"].values()]
    assert abs(sum(per) / len(per) - rec["bytes_per_launch"]) < 1e-3 * rec["bytes_per_launch"]
    W = bench.WORKLOAD
    assert rec["algorithmic_bytes_per_launch"] == bench.algorithmic_bytes(W["nt"], W["nfmax"], W["nx"] ** 2, W["nv"])[1]


@pytest.mark.parametrize("flags,env", [(["--gpus", "2"], {}), ([], {"WORLD_SIZE": "4"})])
def test_more_than_one_gpu_is_refused(flags, env):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *flags], capture_output=True, text=True,
                       env={**os.environ, **env}, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""

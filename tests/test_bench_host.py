"""Host logic of bench.py on the CPU: spectrum parsing, the roofline
arithmetic, the HBM-traffic summary of two counter runs (scaling by the
calibration copies, averaging over the timed launches), the check that a
summary is used only while the kernel sources are unchanged, and the one-GPU
exit."""
import json
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_parse_spectrum():
    assert bench.parse_spectrum("mono") == (0, 0.0)
    assert bench.parse_spectrum("bb:5e4") == (1, 5e4)
    assert bench.parse_spectrum("pl:4") == (2, 4.0)
    assert bench.spectrum_config((1, 5e4)) == {"kind": "blackbody", "T_K": 5e4}
    assert bench.spectrum_config((0, 0.0)) == "mono"
    for bad in ("bb", "xx:3", "pl:"):
        with pytest.raises(SystemExit):
            bench.parse_spectrum(bad)


def test_launch_params():
    assert bench.launch_params("lognormal-128-64src") == (16, 64)
    assert bench.launch_params("lognormal-128-64src", 1) == (64, 64)
    assert bench.launch_params("clustered-512-32768src", 1) == (16, 256)
    assert bench.launch_params("lognormal-256-4096src-bubbles") is None


def test_roofline_arithmetic():
    res = dict(segments_per_s_kernel=5e10, avg_launch_ms=2.0, launches=20,
               segments_per_step=10 ** 9, steps=2, graph=True)
    r = bench.roofline("mixed", res, None)
    assert r["achieved"] == pytest.approx(48 * 5e10 / 1e9)  # 48 B per mixed segment
    assert r["frac"] == pytest.approx(2400.0 / 8000.0)
    assert r["algorithmic_bytes_per_launch"] == pytest.approx(48 * 1e9 * 2 / 20)
    assert r["traffic"] is None and r["mode"] == "graph" and r["bound"] == "hbm"
    f = bench.roofline("fp64", dict(res, graph=False), None)
    assert f["achieved"] == pytest.approx(48 * 5e10 / 1e9) and f["mode"] == "host"
    # the summary's traffic is used only for the launch mode it was measured in
    c = {"mixed_mode": "graph", "mixed_traffic_bytes_per_launch": "4e9"}
    rc = bench.roofline("mixed", res, c, copy_gbs=5000.0)
    assert rc["traffic"] == 4e9
    # measured traffic over the launch time against the peak: 4 GB / 2 ms
    assert rc["hbm_frac_measured"] == pytest.approx(2000.0 / 8000.0)
    assert rc["copy_GBs"] == 5000.0 and rc["frac_of_copy"] == pytest.approx(2400.0 / 5000.0)
    assert bench.roofline("mixed", dict(res, graph=False), c)["traffic"] is None


def _write_run(d, tag, copy_kib, march_kib, launches, **config):
    """A counter CSV and bench line as rocprofv3 and bench.py write them:
    three calibration copies, a larger copy, then march dispatches of which
    the last `launches` belong to the timed step."""
    rows = ["Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value"]
    for i in range(3):
        rows.append(f"{i + 1},__amd_rocclr_copyBuffer,X,{copy_kib}")
    # a field upload after the calibration: not a calibration copy
    rows.append(f"4,__amd_rocclr_copyBuffer,X,{100 * copy_kib}")
    for i, v in enumerate(march_kib):
        rows.append(f"{100 + i},\"void nrt::k_march<true, 2, true, false>(nrt::MarchArgs)\",X,{v}")
    open(os.path.join(d, f"{tag}_counter_collection.csv"), "w").write("\n".join(rows) + "\n")
    line = {"steps": 1, "config": {"path": "mixed", "workload": "lognormal-128-64src", **config},
            "roofline": {"launches": launches, "mode": "graph"}}
    open(os.path.join(d, f"{tag}_bench.json"), "w").write("log line\n" + json.dumps(line) + "\n")


def test_counter_summary_and_staleness(tmp_path, monkeypatch):
    copy_bytes = 3 * 1024 * 2 ** 20
    # the copies read as 0.5 (fetch) and 1.0 (write) of their true bytes
    fetch_copy_kib = 0.5 * copy_bytes / 3 / 1024
    write_copy_kib = 1.0 * copy_bytes / 3 / 1024
    # two warm-up dispatches, then three timed ones
    _write_run(tmp_path, "fetch", fetch_copy_kib, [9e9, 9e9, 100.0, 200.0, 300.0], 3)
    _write_run(tmp_path, "write", write_copy_kib, [7e9, 50.0, 60.0, 70.0], 3)
    out = tmp_path / "k_march_counters_lognormal-128-64src.txt"
    monkeypatch.setattr(bench, "counters_file", lambda w: str(tmp_path / f"k_march_counters_{w}.txt"))
    bench.summarize_counters(str(tmp_path))
    kv = dict(l.split(" = ", 1) for l in out.read_text().splitlines() if " = " in l)
    assert float(kv["copy_factor_fetch"]) == pytest.approx(0.5)
    assert float(kv["copy_factor_write"]) == pytest.approx(1.0)
    fetch = 200.0 * 1024 / 0.5  # mean of the timed launches, scaled by the copy factor
    write = 60.0 * 1024 / 1.0
    assert float(kv["mixed_fetch_bytes_per_launch"]) == pytest.approx(fetch, rel=1e-6)
    assert float(kv["mixed_write_bytes_per_launch"]) == pytest.approx(write, rel=1e-6)
    assert float(kv["mixed_traffic_bytes_per_launch"]) == pytest.approx(fetch + write, rel=1e-6)
    assert kv["mixed_mode"] == "graph" and kv["kernel_sha"] == bench.kernel_hash()
    # a summary is used only while the march kernel's sources are unchanged
    assert float(bench.read_counters("lognormal-128-64src")["mixed_traffic_bytes_per_launch"]) \
        == pytest.approx(fetch + write, rel=1e-6)
    assert bench.read_counters("clustered-512-32768src") is None  # no summary for it
    monkeypatch.setattr(bench, "kernel_hash", lambda: "0" * 16)
    assert bench.read_counters("lognormal-128-64src") is None


def test_counter_summary_of_a_spectrum_subset_run(tmp_path, monkeypatch):
    """A blackbody run on a source subset is summarized under a name of its
    own, so that it never stands for the plain workload's traffic."""
    copy_kib = 0.5 * 1024 * 2 ** 20 / 1024
    cfg = dict(spectrum={"kind": "blackbody", "T_K": 50000.0}, subset=64)
    _write_run(tmp_path, "fetch", copy_kib, [1.0, 2.0], 1, **cfg)
    _write_run(tmp_path, "write", 2 * copy_kib, [3.0, 4.0], 1, **cfg)
    monkeypatch.setattr(bench, "counters_file", lambda w: str(tmp_path / f"k_march_counters_{w}.txt"))
    bench.summarize_counters(str(tmp_path))
    out = tmp_path / "k_march_counters_lognormal-128-64src-bb50000-64src-subset.txt"
    assert "--spectrum bb:50000 --sources 64" in out.read_text()
    assert not (tmp_path / "k_march_counters_lognormal-128-64src.txt").exists()


def test_more_than_one_gpu_exits():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2 and "one GPU" in p.stderr

"""Host-side checks of bench.py: the one-GPU contract, the roofline
arithmetic, the gate that keeps counter figures tied to the kernel sources
they were measured on, and that every committed profile summary was made by
a command that runs committed files only."""
import importlib.util
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_knn_roofline_arithmetic():
    b = _bench()
    n, ms = 134217728, 720.0
    r = b.knn_roofline(n, ms, "k_knn_density", n / 0.785, fused=True)
    # the method's bytes: sorted position 12 + tie key 4 in, 64 indices and
    # the density out
    assert r["bytes_per_particle"] == 280
    assert r["overhead_bytes_per_particle"] == 72
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    achieved = 280 * n / (ms / 1e3) / 1e9
    assert abs(r["achieved"] - achieved) < 0.01
    assert abs(r["frac"] - achieved / 8000.0) < 1e-5
    assert abs(r["frac_with_overhead"] - 352 * n / (ms / 1e3) / 1e9 / 8000.0) < 1e-5
    # not the box kernel: no counter figures
    r2 = b.knn_roofline(1 << 20, 5.0, "k_knn_batch", 1e8)
    assert r2["traffic"] is None and r2["valu"] is None
    assert r2["overhead_bytes_per_particle"] == 0


def test_counter_figures_follow_the_source_hash(tmp_path):
    b = _bench()
    h = b.knn_source_hash()
    good = tmp_path / "good.txt"
    good.write_text(f"# comment: not a value\nsource_hash: {h}\ntraffic_bytes_per_launch: 123\n")
    stale = tmp_path / "stale.txt"
    stale.write_text("source_hash: 0000000000000000\ntraffic_bytes_per_launch: 123\n")
    assert b._summary(str(good))["traffic_bytes_per_launch"] == "123"
    assert b._summary(str(stale)) is None
    assert b._summary(str(tmp_path / "missing.txt")) is None
    # the committed summaries: reported exactly when they match the sources
    for path, fn in ((b.TRAFFIC_FILE, b.measured_traffic),
                     (b.VALU_FILE, lambda: b.measured_valu(134217728, 720.0))):
        with open(path) as f:
            m = re.search(r"^source_hash:\s*(\w+)", f.read(), re.M)
        assert m, path
        assert (fn() is not None) == (m.group(1) == h), path


def test_valu_figures_from_the_summary():
    b = _bench()
    v = b.measured_valu(134217728, 720.0)
    if v is None:
        pytest.skip("the VALU summary was measured on other kernel sources")
    kv = b._summary(b.VALU_FILE)
    insts = float(kv["SQ_INSTS_VALU_per_launch"])
    assert abs(v["insts_per_bucket"] - insts / (134217728 // 64)) < 0.1
    assert abs(v["achieved_lane_ops"] - insts * 64 / 0.72) / v["achieved_lane_ops"] < 1e-9
    assert v["peak_lane_ops"] == 256 * 4 * 16 * 2.4e9
    assert 0.0 < v["valu_busy"] < 1.0


def test_profile_commands_run_committed_files():
    pdir = os.path.join(ROOT, "profiles")
    names = sorted(os.listdir(pdir))
    assert names
    for name in names:
        text = open(os.path.join(pdir, name)).read()
        cmds = [l for l in text.splitlines() if "rocprofv3" in l]
        assert cmds, f"{name}: no command recorded"
        for c in cmds:
            assert "_work" not in c, f"{name}: {c}"
            prog = c.split(" -- ", 1)[1].split()
            assert prog[0] in ("python3", "python"), f"{name}: {c}"
            script = prog[1]
            assert os.path.isfile(os.path.join(ROOT, script)), f"{name}: {script} is not in the repository"

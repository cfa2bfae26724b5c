"""The benchmark's bookkeeping, on the CPU: the measured HBM traffic it reports belongs to the kernel
and planner source and the level-0 choice it was measured with; the roofline arithmetic; a run on
more than one GPU is refused."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _entry():
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
        return json.load(fh)["640x480"]


def test_traffic_is_reported_only_for_the_source_and_choice_it_was_measured_with(monkeypatch):
    e = _entry()
    if e["kernel_sha"] != bench.kernel_sha():
        pytest.skip("traffic.json predates the current kernel or planner source (re-measured on the GPU)")
    measured = {(m["choice"]["mode"], m["choice"]["K"], m["choice"]["rows"]): m["bytes_per_launch"]
                for m in e["entries"]}
    assert measured
    for (mode, K, rows), b in measured.items():
        choice = {"mode": mode, "K": K, "rows": rows, "us_per_iter": 1.0}
        assert bench.measured_traffic("640x480", choice) == b
        # one field away from a measured choice, unless that is measured as well
        for other in ((8, K, rows), (mode, K + 7, rows), (mode, K, rows + 16)):
            if other not in measured:
                c = dict(zip(("mode", "K", "rows"), other))
                assert bench.measured_traffic("640x480", c) is None, other
    choice = dict(e["entries"][0]["choice"])
    assert bench.measured_traffic("640x480", None) is None
    assert bench.measured_traffic("1920x1080", choice) is None
    monkeypatch.setattr(bench, "kernel_sha", lambda: "0" * 16)
    assert bench.measured_traffic("640x480", choice) is None


def test_kernel_hash_covers_the_tile_planner(tmp_path, monkeypatch):
    """The hash reads the iteration kernels and the planner: a planner change alone changes it."""
    csrc = tmp_path / "paper_2011_10979_amd" / "csrc"
    csrc.mkdir(parents=True)
    for f in ("admm.hip", "admm_tb.hip", "admm_args.hpp", "tb_plan.cpp"):
        (csrc / f).write_text(f)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.kernel_sha()
    (csrc / "tb_plan.cpp").write_text("changed")
    assert bench.kernel_sha() != h0


def test_roofline_arithmetic():
    # 35 launches of 23.35 MB (76 B x 640 x 480) in 0.56 ms over one step: 16 us per launch
    px = 640 * 480
    r = bench.roofline(ms=0.56, launches=35, iters=250, px=px, has_w=False, kernel="k", traffic=None, reps=1)
    assert r["bytes_per_launch"] == 76 * px
    assert r["avg_launch_us"] == pytest.approx(16.0)
    assert r["achieved"] == pytest.approx(76 * px / 16e-6 / 1e9, abs=0.1)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0, abs=1e-4)
    assert r["one_pass_equivalent_GBs"] == pytest.approx(76 * px * 250 / 0.56e-3 / 1e9, abs=0.1)
    assert r["bound"] == "hbm" and r["peak"] == 8000.0 and r["launches_per_step_level0"] == 35


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""

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
    """The hash reads the iteration kernels, the planner and the tile geometry: a change to any one
    of them alone changes it."""
    csrc = tmp_path / "paper_2011_10979_amd" / "csrc"
    csrc.mkdir(parents=True)
    files = ("admm.hip", "admm_tb.hip", "admm_rows.hip", "admm_args.hpp", "tb_plan.cpp", "geometry.cpp")
    for f in files:
        (csrc / f).write_text(f)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    for f in files:
        h0 = bench.kernel_sha()
        (csrc / f).write_text(f + " changed")
        assert bench.kernel_sha() != h0, f


def test_roofline_arithmetic():
    # 35 launches over 250 iterations of a 640 x 480 level in 0.56 ms: 16 us per launch, 7.14
    # iterations per launch, priced at 68 B per pixel-iteration; one pass per launch is 76 B per pixel
    px = 640 * 480
    r = bench.roofline(ms=0.56, launches=35, iters=250, px=px, has_w=False, kernel="k", traffic=None, reps=1)
    assert r["px_iter_per_launch"] == round(px * 250 / 35)
    assert r["bytes_per_launch"] == round(68 * px * 250 / 35)
    assert r["avg_launch_us"] == pytest.approx(16.0)
    assert r["achieved"] == pytest.approx(68 * px * 250 / 0.56e-3 / 1e9, abs=0.1)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0, abs=1e-4)
    assert r["one_pass_per_launch"]["GBs"] == pytest.approx(76 * px / 16e-6 / 1e9, abs=0.1)
    assert r["bound"] == "hbm" and r["peak"] == 8000.0 and r["launches_per_step_level0"] == 35
    assert r["traffic"] is None and "dram_GBs" not in r
    t = bench.roofline(ms=0.56, launches=35, iters=250, px=px, has_w=False, kernel="k", traffic=27.3e6, reps=1)
    assert t["dram_GBs"] == pytest.approx(27.3e6 / 16e-6 / 1e9, abs=0.1) and t["traffic_source"]
    w = bench.roofline(ms=0.56, launches=35, iters=250, px=px, has_w=True, kernel="k", traffic=None, reps=1)
    assert w["per_unit"].startswith("92 B") and w["one_pass_per_launch"]["per_unit"].startswith("100 B")


def test_batch_traffic_needs_the_source_and_every_stage_choice(monkeypatch, tmp_path):
    """Per-stage DRAM records combine into bytes per launch weighted by each stage's launches
    (ceil(iters / K) per warp), and only when every stage of the run was measured on this source
    with the same choice (order, tile code, K, width); records without a code are general tiles."""
    csrc = tmp_path / "paper_2011_10979_amd" / "csrc"
    csrc.mkdir(parents=True)
    for f in ("admm_tb.hip", "admm_rows.hip", "admm_args.hpp", "tb_plan.cpp", "multi.cpp", "geometry.cpp"):
        (csrc / f).write_bytes(open(os.path.join(ROOT, "paper_2011_10979_amd", "csrc", f), "rb").read())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    rec = {"batch64": {"kernel_sha": bench.batch_sha(),
                       "stages": [{"level": 0, "order": 0, "K": 5, "ew": 64, "bytes_per_launch": 1.5e9},
                                  {"level": 0, "order": 0, "nt": 3073, "K": 8, "ew": 64, "bytes_per_launch": 1.2e9},
                                  {"level": 1, "order": 0, "K": 10, "ew": 64, "bytes_per_launch": 0.3e9},
                                  {"level": 1, "order": 0, "K": 5, "ew": 128, "bytes_per_launch": 0.4e9}]}}
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(rec))
    # 50 iterations: 10 launches of level 0 per warp, 5 of level 1 at K = 10
    assert bench.batch_traffic([[0, 0, 1025, 5, 64], [1, 0, 1025, 10, 64]], 50) == round((10 * 1.5e9 + 5 * 0.3e9) / 15)
    assert bench.batch_traffic([[0, 0, 1025, 5, 64], [1, 0, 1025, 5, 128]], 50) == round((1.5e9 + 0.4e9) / 2)
    assert bench.batch_traffic([[0, 0, 1025, 5, 64]], 50) == 1.5e9
    assert bench.batch_traffic([[0, 0, 3073, 8, 64]], 50) == 1.2e9
    assert bench.batch_traffic([[0, 0, 2049, 8, 64]], 50) is None
    assert bench.batch_traffic([[0, 0, 1025, 6, 64], [1, 0, 1025, 10, 64]], 50) is None
    assert bench.batch_traffic([[0, 1, 1025, 5, 64]], 50) is None
    assert bench.batch_traffic("built-in", 50) is None
    (csrc / "multi.cpp").write_text("changed")
    assert bench.batch_traffic([[0, 0, 1025, 5, 64]], 50) is None


def test_pair_px_sums_the_pyramid():
    assert bench.pair_px(480, 640, 5) == 409200
    assert bench.pair_px(1080, 1920, 6) == 2764200


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""

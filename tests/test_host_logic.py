"""The library's host code on the CPU, under AddressSanitizer and UndefinedBehaviorSanitizer: the
runtime, planner, batch and serving sources built with g++ against a fake HIP runtime whose toy
kernels have the real kernels' memory footprint (tests/host/fake_device.cpp), driven by
tests/host/host_logic_test.cpp -- the first-fit serving arena against a model, tile coverage and
capacity of every planner, and pairs solved alone, batched and served in randomised submit / step /
poll orders giving bitwise the same results within the budget and slot limits."""
import concurrent.futures as cf
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2011_10979_amd", "csrc")
HOST = os.path.join(ROOT, "tests", "host")
SOURCES = [os.path.join(CSRC, f) for f in ("runtime.cpp", "geometry.cpp", "context.cpp", "tb_plan.cpp", "autotune.cpp",
                                           "batch.cpp", "multi.cpp", "serve.cpp")]
SOURCES += [os.path.join(HOST, "fake_device.cpp"), os.path.join(HOST, "host_logic_test.cpp")]
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]
FLAGS = ["-std=c++17", "-O1", "-g", "-Wall", "-Wno-unused-variable", "-I", os.path.join(HOST, "fake"),
         "-I", os.path.join(ROOT, "include"), "-I", CSRC] + SAN


@pytest.fixture(scope="module")
def binary(tmp_path_factory):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no g++")
    out = tmp_path_factory.mktemp("host_logic")

    def compile_one(src):
        obj = str(out / (os.path.basename(src) + ".o"))
        r = subprocess.run([cxx] + FLAGS + ["-c", src, "-o", obj], capture_output=True, text=True)
        assert r.returncode == 0, f"{src}\n{r.stderr[-4000:]}"
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    exe = str(out / "host_logic_test")
    r = subprocess.run([cxx] + SAN + objs + ["-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    return exe


@pytest.mark.parametrize("seed", [1, 2])
def test_host_logic_under_sanitizers(binary, seed):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([binary, str(seed)], capture_output=True, text=True, timeout=600, env=env)
    print(r.stdout[-2000:])
    assert r.returncode == 0 and "HOST LOGIC OK" in r.stdout, (r.stdout[-3000:], r.stderr[-6000:])

"""The C ABI's host code under AddressSanitizer: the three translation units
compiled for the host only with -fsanitize=address (no device code: nothing
here launches a kernel), linked with tests/asan/abi_host_driver.cpp, which
exercises every path that runs without a GPU (validation, workspace sizing,
context set-up including the compact filter's host tables at the smallest and
longest lines, call-order and argument errors).  A memory error aborts the
driver; a wrong return code fails it."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1812_02459_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_abi_host_code_under_address_sanitizer(tmp_path):
    san = ["-Xarch_host", "-fsanitize=address", "-fno-omit-frame-pointer", "-g", "-O1"]
    # host code only; relocatable device code leaves the (empty) device link to
    # the final link, so no kernel is compiled
    common = ["-std=c++17", "-fgpu-rdc", "--offload-host-only", "-fPIC", "-I",
              os.path.join(ROOT, "include")]
    objs = []
    for src in ("lbm2p.hip", "lbm2p_f64.hip", "lbm2p_f32.hip",
                os.path.join(ROOT, "tests", "asan", "abi_host_driver.cpp")):
        path = src if os.path.isabs(src) else os.path.join(CSRC, src)
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        if path.endswith(".cpp"):
            cmd = [HIPCC, "-std=c++17", "-I", os.path.join(ROOT, "include")] + san + [
                "-x", "c++", "-c", path, "-o", obj]
        else:
            cmd = [HIPCC] + common + san + ["-c", path, "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        objs.append(obj)
    exe = str(tmp_path / "abi_host_driver")
    r = subprocess.run([HIPCC, "-fgpu-rdc", "--hip-link", "--offload-arch=gfx950",
                        "-Xarch_host", "-fsanitize=address"] + objs + ["-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    print(r.stdout, r.stderr[-2000:])
    assert r.returncode == 0, r.stderr[-3000:]
    assert "abi host driver: ok" in r.stdout


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_sanitizer_build_reports_a_planted_overflow(tmp_path):
    """The same compile and link lines on a program with a heap read past the
    end: the run must stop with the sanitizer's report."""
    src = os.path.join(ROOT, "tests", "asan", "planted_overflow.cpp")
    obj, exe = str(tmp_path / "p.o"), str(tmp_path / "p")
    r = subprocess.run([HIPCC, "-std=c++17", "-Xarch_host", "-fsanitize=address", "-g", "-O1",
                        "-x", "c++", "-c", src, "-o", obj], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    r = subprocess.run([HIPCC, "-fgpu-rdc", "--hip-link", "--offload-arch=gfx950",
                        "-Xarch_host", "-fsanitize=address", obj, "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=60)
    assert r.returncode != 0
    assert "heap-buffer-overflow" in r.stderr

"""The oracle and the library's host-side logic built with AddressSanitizer and
UndefinedBehaviorSanitizer (host code only; nothing here touches a device).  Each
build runs a small driver under tests/sanitize/ that must exit cleanly with no
sanitizer report."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_1902_05132_amd", "csrc")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="4")


def _run(exe, env):
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    return out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no C compiler")
def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_run")
    subprocess.run(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-fopenmp", "-o", exe, os.path.join(ROOT, "oracle", "oracle.c"),
                    os.path.join(SAN, "oracle_run.c"), "-lm"], check=True)
    # libgomp keeps its thread pool until exit: leak checks on the oracle's own allocations only
    out = _run(exe, dict(ENV, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1"))
    assert "oracle run: ok" in out


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="no hipcc")
def test_host_driver_under_address_and_ub_sanitizers(tmp_path):
    objs = [os.path.join(CSRC, "lfmm_kernels.o"), os.path.join(CSRC, "lfmm_mlp.o")]
    if not all(os.path.exists(o) for o in objs):
        pytest.skip("library objects not built")
    host_o = str(tmp_path / "lfmm_host_san.o")
    exe = str(tmp_path / "host_run")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-fno-gpu-sanitize"]
    base = ["hipcc", "--offload-arch=gfx950", "-O1", "-g", "-fno-omit-frame-pointer", "-std=c++17",
            "-I", os.path.join(ROOT, "include")]
    subprocess.run(base + san + ["-c", os.path.join(CSRC, "lfmm_host.hip"), "-o", host_o], check=True)
    run_o = str(tmp_path / "host_run.o")
    subprocess.run(base + san + ["-c", os.path.join(SAN, "host_run.cpp"), "-o", run_o], check=True)
    subprocess.run(base + san + [run_o, host_o] + objs + ["-o", exe], check=True)
    out = _run(exe, dict(ENV, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1"))
    assert "host run:" in out and "ok" in out

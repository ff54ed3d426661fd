"""The C-ABI's host argument checks (csrc/qc_hostcheck.cpp, compiled into
libqc.so) built on their own with the host address and undefined-behaviour
sanitizers and run over malformed and edge-case inputs
(tests/hostcheck_driver.cpp).  CPU only: the checks need no device."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(ROOT, "paper_2412_10072_amd", "csrc", "qc_hostcheck.cpp")
DRIVER = os.path.join(HERE, "hostcheck_driver.cpp")


def test_host_checks_under_sanitizers(tmp_path):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no g++")
    exe = str(tmp_path / "hostcheck")
    cmd = [cxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-Wall", "-Werror", f"-I{os.path.join(ROOT, 'include')}", SRC, DRIVER,
           "-o", exe]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, f"build failed:\n{res.stdout}\n{res.stderr}"
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    print(run.stdout)
    assert run.returncode == 0, f"driver failed:\n{run.stdout}\n{run.stderr}"
    assert "0 failures" in run.stdout
    assert "ERROR: AddressSanitizer" not in run.stderr and "runtime error" not in run.stderr

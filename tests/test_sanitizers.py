"""Host code under the address and undefined-behaviour sanitizers (no GPU):
the launch plans and workspace layout of the library's host side, and the
CPU oracle running its own pins."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_plans_and_layouts_under_sanitizers(tmp_path):
    exe = tmp_path / "plan_test"
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", "-I", os.path.join(ROOT, "include"),
                    "-I", os.path.join(ROOT, "paper_1907_04839_amd", "csrc"),
                    os.path.join(ROOT, "tests", "cpp", "plan_test.cpp"), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "plans ok" in out.stdout


def _runtime(name):
    path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True,
                          text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.slow
def test_oracle_pins_under_sanitizers(tmp_path):
    """The oracle built with -fsanitize=address,undefined (aborting on the first
    report) passes every one of its CPU pins."""
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("gcc's sanitizer runtimes are not installed")
    sys.path.insert(0, ROOT)
    from oracle import build as oracle_build
    lib = oracle_build.build(out=str(tmp_path / "liboracle_san.so"), sanitize=True)
    env = {**os.environ, "ORACLE_LIB": lib, "LD_PRELOAD": f"{asan}:{ubsan}",
           "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
           "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"}
    out = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                          os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                         capture_output=True, text=True, timeout=1200, env=env, cwd=ROOT)
    tail = (out.stdout + out.stderr)[-3000:]
    assert out.returncode == 0, tail
    assert "runtime error" not in out.stderr and "AddressSanitizer" not in out.stderr, tail

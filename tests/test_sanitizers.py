"""Host sanitizer builds (CPU): the FP64 oracle's C code (oracle/ray_oracle.c)
and the ABI's input checks (paper_2202_05628_amd/csrc/validate.h) compiled
with AddressSanitizer and UndefinedBehaviorSanitizer (errors fatal) and run on
the drivers in tests/sanitize/.  A control program with a planted
out-of-bounds read shows that the same flags catch such a fault here."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _need(tool):
    if shutil.which(tool) is None:
        pytest.skip(f"{tool} not found")


def _build_and_run(cmd, exe):
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, f"build failed:\n{r.stderr}"
    return subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=120)


def test_sanitizers_catch_a_planted_fault(tmp_path):
    _need("gcc")
    src = tmp_path / "oob.c"
    src.write_text("#include <stdlib.h>\nint main(void){int*a=malloc(4*sizeof(int));int v=a[4];free(a);return v&0;}\n")
    exe = str(tmp_path / "oob")
    r = _build_and_run(["gcc", *SAN, str(src), "-o", exe], exe)
    assert r.returncode != 0 and ("heap-buffer-overflow" in r.stderr or "runtime error" in r.stderr)


def test_oracle_under_asan_ubsan(tmp_path):
    _need("gcc")
    exe = str(tmp_path / "oracle_san")
    r = _build_and_run(["gcc", "-std=c99", *SAN, os.path.join(ROOT, "oracle", "ray_oracle.c"),
                        os.path.join(ROOT, "tests", "sanitize", "oracle_sanitize.c"), "-lm", "-o", exe], exe)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
    assert "all checks passed" in r.stdout


def test_abi_input_checks_under_asan_ubsan(tmp_path):
    _need("g++")
    exe = str(tmp_path / "validate_san")
    r = _build_and_run(["g++", "-std=c++17", *SAN, "-I", os.path.join(ROOT, "paper_2202_05628_amd", "csrc"),
                        os.path.join(ROOT, "tests", "sanitize", "validate_sanitize.cpp"), "-o", exe], exe)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
    assert "all checks passed" in r.stdout

"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the CPU code: the
oracle (oracle/amrmg_oracle.c) and the product's host hierarchy code
(paper_1812_03689_amd/csrc/amrmg_hier.cpp), each driven by its own small
program in tests/native/ through every function it exports.  Host code only
(gcc / g++; no GPU code is built here).  Any invalid access, leak or
undefined behaviour aborts the driver, and the test fails with its report."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NATIVE = os.path.join(ROOT, "tests", "native")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def run(cmd, exe):
    b = subprocess.run(cmd + ["-o", exe], capture_output=True, text=True)
    assert b.returncode == 0, b.stderr
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=600)
    assert r.returncode == 0, (r.returncode, r.stdout[-2000:], r.stderr[-6000:])
    assert "runtime error" not in r.stderr and "ERROR: " not in r.stderr, r.stderr[-6000:]
    return r.stdout


def test_oracle_under_sanitizers(tmp_path):
    out = run(["gcc", "-std=c99"] + SAN + [os.path.join(NATIVE, "oracle_sanitize.c"),
                                           os.path.join(ROOT, "oracle", "amrmg_oracle.c"), "-lm"],
              str(tmp_path / "oracle_sanitize"))
    assert "oracle sanitize ok" in out


def test_host_hierarchy_under_sanitizers(tmp_path):
    csrc = os.path.join(ROOT, "paper_1812_03689_amd", "csrc")
    out = run(["g++", "-std=c++17", "-I" + csrc] + SAN + [os.path.join(NATIVE, "hier_sanitize.cpp"),
                                                           os.path.join(csrc, "amrmg_hier.cpp")],
              str(tmp_path / "hier_sanitize"))
    assert "hier sanitize ok" in out

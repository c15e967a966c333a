"""The library's host-only code and the oracle built with AddressSanitizer and
UndefinedBehaviorSanitizer (host code only; no GPU): tests/sanitize/host_fuzz.cpp drives
parameter validation, workspace layouts and the host input check over tens of thousands of
valid and invalid parameter sets, tests/sanitize/oracle_fuzz.c runs every oracle scheme on
tiny inputs.  Any memory error or undefined behaviour fails the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600, **kw)
    assert r.returncode == 0, (cmd, r.stdout[-3000:], r.stderr[-3000:])
    return r


@pytest.fixture(scope="module")
def outdir(tmp_path_factory):
    if not shutil.which("g++") or not shutil.which("gcc"):
        pytest.skip("no host compiler")
    return tmp_path_factory.mktemp("sanitize")


def test_host_runtime_under_sanitizers(outdir):
    exe = str(outdir / "host_fuzz")
    _run(["g++", "-std=c++17", *SAN, "-I", os.path.join(ROOT, "include"), "-o", exe,
          os.path.join(ROOT, "tests", "sanitize", "host_fuzz.cpp"),
          os.path.join(ROOT, "paper_2411_09605_amd", "csrc", "pic_host.cpp")])
    r = _run([exe], env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1",
                             UBSAN_OPTIONS="print_stacktrace=1"))
    assert r.stdout.startswith("ok"), r.stdout


def test_oracle_under_sanitizers(outdir):
    exe = str(outdir / "oracle_fuzz")
    _run(["gcc", "-std=gnu11", *SAN, "-ffp-contract=off", "-o", exe,
          os.path.join(ROOT, "tests", "sanitize", "oracle_fuzz.c"),
          os.path.join(ROOT, "oracle", "pic_oracle.c"), "-lm"])
    r = _run([exe], env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1",
                             UBSAN_OPTIONS="print_stacktrace=1"))
    assert r.stdout.startswith("ok"), r.stdout

"""Host sanitizer builds (AddressSanitizer + UndefinedBehaviorSanitizer) of
the oracle and of the library's host code (operators and geometry), each run
by a small driver under tests/c/; and the library's device-budget knob, which
turns a problem larger than ESDG_DEVICE_BUDGET into ESDG_ENOMEM before any
device work."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
           OMP_NUM_THREADS="2")


def build_and_run(tmp_path, cmd, exe):
    r = subprocess.run(cmd + ["-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=240)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    return r.stdout


def test_oracle_under_sanitizers(tmp_path):
    out = build_and_run(tmp_path, ["gcc", "-std=gnu11", "-fopenmp"] + SAN +
                        [os.path.join(ROOT, "tests", "c", "oracle_sanitize.c"), "-lm"],
                        str(tmp_path / "oracle_sanitize"))
    assert "oracle sanitize ok" in out


def test_host_ops_under_sanitizers(tmp_path):
    csrc = os.path.join(ROOT, "paper_2112_10517_amd", "csrc")
    out = build_and_run(tmp_path, ["g++", "-std=c++17", "-pthread"] + SAN +
                        ["-I", csrc, os.path.join(csrc, "host_ops.cpp"),
                         os.path.join(ROOT, "tests", "c", "host_ops_sanitize.cpp")],
                        str(tmp_path / "host_ops_sanitize"))
    assert "host_ops sanitize ok" in out


def test_device_budget_gives_enomem(monkeypatch):
    from paper_2112_10517_amd import esdg, build
    if not os.path.exists(esdg.LIB_PATH):
        build.build()
    need = esdg.footprint(3, 3, (4, 4, 4), warp=0.1)
    monkeypatch.setenv("ESDG_DEVICE_BUDGET", str(need - 1))
    with pytest.raises(esdg.EsdgError) as ei:
        esdg.Problem(3, 3, (4, 4, 4), warp=0.1)
    assert ei.value.status == esdg.ENOMEM
    assert "ESDG_DEVICE_BUDGET" in str(ei.value)

"""Host code under the address and undefined-behaviour sanitizers (gcc):
the oracle (every collision, force and wall option, the convergence loop,
the observables) and the library's host thermodynamics (critical points,
Maxwell construction, EOS values).  A sanitizer report fails the run."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
         "-fno-sanitize-recover=all"]


def _run(cmd, exe):
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
    return r.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    out = _run(["gcc"] + FLAGS + ["-ffp-contract=off", os.path.join(HERE, "sanitize_oracle_main.c"),
                                  "-o", exe, "-lm"], exe)
    assert "ok" in out


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not found")
def test_host_thermodynamics_under_sanitizers(tmp_path):
    exe = str(tmp_path / "thermo_san")
    out = _run(["g++", "-std=c++17"] + FLAGS + [
        os.path.join(HERE, "sanitize_thermo_main.cpp"),
        os.path.join(ROOT, "paper_1906_09530_amd", "csrc", "thermo.cpp"), "-o", exe], exe)
    assert "ok" in out
